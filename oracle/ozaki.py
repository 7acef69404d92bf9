"""Oracle: FP64 matrix products from exact integer products of 8-bit slices
(the Ozaki splitting scheme).  The paper fixes no such form; it is the
model for an FP64-accurate split renormalisation on the integer matrix
units (8-bit operands, 32-bit accumulation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Scheme (for C = A B, A m x k, B k x n, beta = 7 bits per slice):

* every row i of A is scaled by 2^-e_i, e_i = floor(log2 max_j |A_ij|) + 1,
  so that the scaled row lies in (-1, 1); every column j of B likewise by
  2^-f_j;
* the scaled value x is cut into s slices of beta bits, highest first:
  x_1 = trunc(x 2^beta), x_t = trunc((x - sum_{u<t} x_u 2^-beta u) 2^beta t),
  every x_t an integer in [-127, 127], and x = sum_t x_t 2^-beta t + r with
  |r| < 2^-beta s;
* C_ij ~ 2^(e_i + f_j) sum_{t + u <= s + 1} 2^-beta(t+u) (A_t B_u)_ij, every
  slice product an exact integer matrix product (here in int64; on the
  hardware in int32, exact while k 127^2 < 2^31), the terms with
  t + u > s + 1 dropped.

Error (``error_bound``).  Per term of the inner sum, the truncation
remainders contribute less than 2 2^-beta s, and the dropped slice products
(t + u >= s + 2, at most s - 1 of them per value of t + u, each below
2^-beta (t+u-2)) less than 1.008 (s - 1) 2^-beta s, together less than
(s + 2) 2^-beta s; the FP64 accumulation of the s (s + 1) / 2 exact slice
products (each partial sum below 1.02 k) adds at most s (s + 1) / 2 rounding
errors of 2^-53 of that.  So
    |C_ij - (AB)_ij| <= 2^(e_i + f_j) k ((s + 2) 2^-beta s + s (s + 1) 2^-53).
"""
import numpy as np

BETA = 7


def exponents(A, axis):
    """e with max |A| along the other axis < 2^e, per row (axis=1) or per
    column (axis=0); rows or columns that are all zero get e = 0."""
    mx = np.max(np.abs(A), axis=axis)
    e = np.zeros(mx.shape, dtype=np.int64)
    nz = mx > 0
    e[nz] = np.floor(np.log2(mx[nz])).astype(np.int64) + 1
    return e


def slices(X, s):
    """Integer slices x_1..x_s (int64 arrays) of X with entries in (-1, 1)."""
    X = np.asarray(X, dtype=np.float64)
    assert np.all(np.abs(X) < 1.0)
    out = []
    rem = X.copy()
    for t in range(1, s + 1):
        xt = np.trunc(np.ldexp(rem, BETA * t))
        out.append(xt.astype(np.int64))
        rem = rem - np.ldexp(xt, -BETA * t)  # exact: xt has at most beta bits at that scale
    return out


def ozaki_matmul(A, B, s):
    """C ~ A B from s slices of each operand (module docstring)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    e = exponents(A, axis=1)
    f = exponents(B, axis=0)
    As = slices(np.ldexp(A, -e[:, None]), s)
    Bs = slices(np.ldexp(B, -f[None, :]), s)
    k = A.shape[1]
    C = np.zeros((A.shape[0], B.shape[1]))
    for t in range(1, s + 1):
        for u in range(1, s + 2 - t):
            P = As[t - 1] @ Bs[u - 1]  # exact integer product
            assert np.abs(P).max(initial=0) <= k * 127 * 127
            C += np.ldexp(P.astype(np.float64), -BETA * (t + u))
    return np.ldexp(C, e[:, None] + f[None, :])


def n_products(s):
    """Number of slice products of the scheme: s (s + 1) / 2."""
    return s * (s + 1) // 2


def error_bound(A, B, s):
    e = exponents(np.asarray(A, dtype=np.float64), axis=1)
    f = exponents(np.asarray(B, dtype=np.float64), axis=0)
    k = np.asarray(A).shape[1]
    per = k * ((s + 2.0) * 2.0 ** (-BETA * s) + s * (s + 1) * 2.0 ** -53)
    return np.ldexp(np.full((len(e), len(f)), per), e[:, None] + f[None, :])
