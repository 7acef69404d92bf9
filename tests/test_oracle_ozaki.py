"""Pins of the oracle's model of FP64 products from 8-bit slices
(oracle/ozaki.py; the FP64-accurate split form of the renormalisation
products, a form the paper does not fix).

* Slicing: every slice is an integer in [-127, 127]; s slices rebuild a
  value of (-1, 1) to within 2^-7s, exactly when it has at most 7s
  significant bits; the row and column exponents put the largest entry in
  [1/2, 1).
* Exactness: integer matrices whose rows and columns stay below 128 are
  multiplied exactly (against numpy's int64 product).
* Accuracy against the exact rational product (fractions): the error stays
  within the stated bound for every slice count 1..8 and shrinks by about
  2^-7 per slice until FP64 rounding; at 8 slices the result is as close to
  the exact product as numpy's FP64 product.
* Power-of-two row and column scalings pass through exactly (per-row and
  per-column exponents), also across a range of 2^+-300.
* A mistake planted in the oracle (the last slice dropped) breaks the bound.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ozaki


def _exact(A, B):
    Af = [[Fraction(float(x)) for x in row] for row in A]
    Bf = [[Fraction(float(x)) for x in row] for row in B]
    k = len(Bf)
    return [[sum(Af[i][t] * Bf[t][j] for t in range(k)) for j in range(len(Bf[0]))] for i in range(len(Af))]


def _err(C, E):
    return np.array([[abs(Fraction(float(C[i, j])) - E[i][j]) for j in range(C.shape[1])] for i in range(C.shape[0])],
                    dtype=np.float64)


def test_slices_and_exponents():
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (50, 7)) * 0.999999
    for s in (1, 3, 8):
        sl = ozaki.slices(X, s)
        assert all(np.abs(x).max() <= 127 for x in sl)
        back = sum(np.ldexp(x.astype(np.float64), -7 * (t + 1)) for t, x in enumerate(sl))
        assert np.abs(X - back).max() < 2.0 ** (-7 * s)
    # a value with exactly 21 significant bits below the point: 3 slices are exact
    m = rng.integers(-(2 ** 21) + 1, 2 ** 21, size=40)
    Y = np.ldexp(m.astype(np.float64), -21)
    sl = ozaki.slices(Y, 3)
    assert np.array_equal(sum(np.ldexp(x.astype(np.float64), -7 * (t + 1)) for t, x in enumerate(sl)), Y)
    A = rng.standard_normal((6, 9)) * np.ldexp(1.0, rng.integers(-30, 30, size=(6, 1)))
    e = ozaki.exponents(A, axis=1)
    r = np.abs(A).max(axis=1) * 2.0 ** -e.astype(np.float64)
    assert np.all((r >= 0.5) & (r < 1.0))
    assert ozaki.exponents(np.zeros((2, 3)), axis=1).tolist() == [0, 0]


def test_small_integers_are_exact():
    rng = np.random.default_rng(2)
    A = rng.integers(-127, 128, size=(9, 40))
    B = rng.integers(-127, 128, size=(40, 7))
    for s in (1, 2, 8):
        C = ozaki.ozaki_matmul(A.astype(np.float64), B.astype(np.float64), s)
        assert np.array_equal(C, (A @ B).astype(np.float64))


def test_error_against_the_exact_product():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((5, 12))
    B = rng.standard_normal((12, 4))
    A[1] *= 1e-5  # rows and columns of different magnitudes
    B[:, 2] *= 3e4
    E = _exact(A, B)
    errs = []
    for s in range(1, 9):
        err = _err(ozaki.ozaki_matmul(A, B, s), E)
        assert np.all(err <= ozaki.error_bound(A, B, s)), s
        errs.append(err.max() / ozaki.error_bound(A, B, 1).max())
    for s in range(1, 6):  # about 2^-7 per slice while truncation dominates
        assert errs[s] < errs[s - 1] / 30, (s, errs)
    # at 8 slices as accurate as the FP64 product (relative to |A||B|)
    scale = np.abs(A) @ np.abs(B)
    C8 = ozaki.ozaki_matmul(A, B, 8)
    assert np.all(_err(C8, E) <= 12 * 2.0 ** -52 * scale)
    assert np.all(_err(A @ B, E) <= 12 * 2.0 ** -52 * scale)
    assert ozaki.n_products(8) == 36


def test_power_of_two_scalings_pass_through_exactly():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 10))
    B = rng.standard_normal((10, 5))
    p = rng.integers(-300, 300, size=6)
    q = rng.integers(-300, 300, size=5)
    C = ozaki.ozaki_matmul(A, B, 6)
    Cs = ozaki.ozaki_matmul(np.ldexp(A, p[:, None]), np.ldexp(B, q[None, :]), 6)
    assert np.array_equal(Cs, np.ldexp(C, p[:, None] + q[None, :]))


def test_planted_dropped_slice_breaks_the_bound(monkeypatch):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((4, 8))
    B = rng.standard_normal((8, 3))
    E = _exact(A, B)
    s = 4
    real = ozaki.slices

    def fewer(X, s_):
        out = real(X, s_)
        out[-1] = np.zeros_like(out[-1])
        return out
    monkeypatch.setattr(ozaki, 'slices', fewer)
    err = _err(ozaki.ozaki_matmul(A, B, s), E)
    assert np.any(err > ozaki.error_bound(A, B, s))
