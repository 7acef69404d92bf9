"""Oracle: the split-precision product model of the H_eff GEMMs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper runs its products on tensor-core units beyond the FP64 ceiling
(Fig. 2, Sec. IV) without fixing a number format; the split forms here are
the reading recorded in the design notes:

* FP32 form: operands rounded to binary32, products accumulated in binary32.
* 3xBF16 form: every binary32 operand element v is split into two bfloat16
  numbers, hi = RNE(v) and lo = RNE(v - hi), and a product of two elements
  is approximated by  hi_a*lo_b + lo_a*hi_b + hi_a*hi_b  (lo*lo dropped),
  accumulated in binary32.
* 6xBF16 form: v is split into three bfloat16 numbers, hi = RNE(v),
  mid = RNE(v - hi), lo = RNE(v - hi - mid) (each difference exact in
  binary32), and a product is approximated by the six terms down to
  2^-16 relative: hi*lo + lo*hi + mid*mid + hi*mid + mid*hi + hi*hi
  (mid*lo, lo*mid and lo*lo dropped), accumulated in binary32 -- about the
  accuracy of binary32 operands at the bfloat16 product rate.

bfloat16 is the upper half of a binary32 word: sign, the 8 exponent bits and
the top 7 stored significand bits (8 significant bits).  RNE rounds the
dropped lower 16 bits to nearest, ties to an even kept word.

The model below evaluates the split product *exactly up to FP64 rounding*
(products of bfloat16 numbers are exact in binary64, sums carry FP64
rounding only), so it differs from a binary32-accumulating kernel only by
that kernel's accumulation rounding.  Finite inputs only (no NaN / Inf).
"""
import numpy as np


def bf16_rne(x):
    """Round binary32 values to bfloat16 (round to nearest, ties to even);
    returns the rounded values as float32 arrays."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> 16) & 1
    r = (u + 0x7FFF + keep_lsb) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split_bf16(x):
    """(hi, lo) with hi = RNE_bf16(x), lo = RNE_bf16(x - hi); x - hi is exact
    in binary32 (hi holds the leading bits of x)."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def split3_bf16(x):
    """(hi, mid, lo): hi = RNE_bf16(x), mid = RNE_bf16(x - hi),
    lo = RNE_bf16(x - hi - mid); both differences are exact in binary32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    r1 = (x - hi).astype(np.float32)
    mid = bf16_rne(r1)
    lo = bf16_rne((r1 - mid).astype(np.float32))
    return hi, mid, lo


def fold_alpha(alpha, A):
    """alpha op(A) as the split forms stage it: the product rounded to
    binary32 before any split."""
    return (np.float32(alpha) * np.asarray(A, dtype=np.float32)).astype(np.float32)


def product_bf16x3(A, B):
    """The 3xBF16 product of binary32 matrices A (m x k) and B (k x n), in
    FP64: hi_A lo_B + lo_A hi_B + hi_A hi_B."""
    ah, al = (v.astype(np.float64) for v in split_bf16(A))
    bh, bl = (v.astype(np.float64) for v in split_bf16(B))
    return ah @ bl + al @ bh + ah @ bh


def product_bf16x6(A, B):
    """The 6xBF16 product of binary32 matrices A and B, in FP64: the terms
    hi*lo + lo*hi + mid*mid + hi*mid + mid*hi + hi*hi of the three-way
    splits."""
    ah, am, al = (v.astype(np.float64) for v in split3_bf16(A))
    bh, bm, bl = (v.astype(np.float64) for v in split3_bf16(B))
    return ah @ bl + al @ bh + am @ bm + ah @ bm + am @ bh + ah @ bh


def product_fp32(A, B):
    """The FP32 product model: binary32 operands, exact products (in FP64)."""
    return np.asarray(A, dtype=np.float32).astype(np.float64) @ np.asarray(B, dtype=np.float32).astype(np.float64)


def error_bound_bf16x3(A, B):
    """Elementwise bound of |product_bf16x3(A, B) - A B| for binary32 A, B:
    |a - hi - lo| <= 2^-16 |a| and |lo| <= 2^-8 |a| give, per term,
    |ab - (hi_a lo_b + lo_a hi_b + hi_a hi_b)| <= (2^-16 + 2^-16 + 2^-16 +
    higher order) |a||b| < 3.1 * 2^-16 |a||b|."""
    return 3.1 * 2.0 ** -16 * (np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64)))


def error_bound_bf16x6(A, B):
    """Elementwise bound of |product_bf16x6(A, B) - A B| for binary32 A, B:
    a = hi + mid + lo + e with |mid| <= 2^-8 |a|, |lo| <= 2^-16 |a| and
    |e| <= 2^-24 |a| (each RNE_bf16 keeps the relative error of its part to
    2^-8); the dropped terms mid*lo', lo*mid', lo*lo' and the representation
    errors e*b, a*e' give at most (4 + higher order) 2^-24 |a||b| < 4.1 *
    2^-24 |a||b| per term."""
    return 4.1 * 2.0 ** -24 * (np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64)))
