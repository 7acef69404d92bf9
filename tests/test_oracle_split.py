"""Pins of the split-precision product model (oracle.split) against what the
number formats fix: bfloat16 rounding against an independent library
conversion and hand-built ties, the split of numbers built from known parts,
the closed forms of the three- and six-product sums on such numbers, and the
error bounds of the models against the exact product."""
import numpy as np
import pytest

from oracle import split as S

torch = pytest.importorskip('torch')


def test_bf16_rounding_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000), rng.standard_normal(2000) * 1e-30,
                        rng.standard_normal(2000) * 1e30, [0.0, -0.0, 1.0, -1.0, 3.0e38]]).astype(np.float32)
    lib = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(S.bf16_rne(x).view(np.uint32), lib.view(np.uint32))


def test_bf16_ties_go_to_even():
    # 1 + 2^-8 lies halfway between 1 (even) and 1 + 2^-7 (odd): rounds down;
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even): rounds up
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 1 + 2.0 ** -8 + 2.0 ** -20], np.float32)
    want = np.array([1.0, 1 + 2.0 ** -6, -1.0, 1 + 2.0 ** -7], np.float32)
    assert np.array_equal(S.bf16_rne(x), want)


def _known_parts(rng, shape):
    """Binary32 numbers a = h + l with h an 8-significant-bit number and l an
    integer multiple of 2^(e-16) below half an ulp of h, so that by
    construction RNE_bf16(a) = h and a - h = l is itself a bfloat16."""
    e = rng.integers(-3, 4, size=shape)
    # 8-bit significand of h; not a power of two, where the spacing below h halves
    mh = rng.integers(129, 256, size=shape)
    h = mh * 2.0 ** (e - 7)
    ml = rng.integers(-127, 128, size=shape)                  # |l| < 2^(e-8) = half ulp of h
    l = ml * 2.0 ** (e - 15)
    s = rng.choice([-1.0, 1.0], size=shape)
    return (s * h).astype(np.float32), (s * l).astype(np.float32)


def test_split_of_numbers_with_known_parts():
    rng = np.random.default_rng(1)
    h, l = _known_parts(rng, 5000)
    a = (h.astype(np.float64) + l).astype(np.float32)
    assert np.array_equal(a.astype(np.float64), h.astype(np.float64) + l)   # a exact in binary32
    hi, lo = S.split_bf16(a)
    assert np.array_equal(hi, h) and np.array_equal(lo, l)


def test_three_product_sum_closed_form():
    """On numbers with known parts the model is the exact product minus the
    lo*lo term: (H+L)(H'+L') - L L' = H H' + H L' + L H'."""
    rng = np.random.default_rng(2)
    Ha, La = _known_parts(rng, (7, 11))
    Hb, Lb = _known_parts(rng, (11, 5))
    A = (Ha.astype(np.float64) + La).astype(np.float32)
    B = (Hb.astype(np.float64) + Lb).astype(np.float32)
    H64a, L64a, H64b, L64b = (v.astype(np.float64) for v in (Ha, La, Hb, Lb))
    want = (H64a + L64a) @ (H64b + L64b) - L64a @ L64b
    got = S.product_bf16x3(A, B)
    assert np.allclose(got, want, rtol=0, atol=1e-15 * np.abs(want).max())
    # and it is not the exact product: the dropped lo*lo term is visible
    assert np.abs(got - A.astype(np.float64) @ B.astype(np.float64)).max() > 0


@pytest.mark.parametrize('k', [1, 7, 64, 300])
def test_model_within_error_bound_of_exact_product(k):
    rng = np.random.default_rng(10 + k)
    A = rng.standard_normal((40, k)).astype(np.float32)
    B = (rng.standard_normal((k, 30)) * 10.0 ** rng.integers(-3, 4, size=(k, 30))).astype(np.float32)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    err = np.abs(S.product_bf16x3(A, B) - exact)
    bound = S.error_bound_bf16x3(A, B)
    assert np.all(err <= bound)
    # a product that dropped one of the cross terms breaks the bound
    ah, al = (v.astype(np.float64) for v in S.split_bf16(A))
    bh, bl = (v.astype(np.float64) for v in S.split_bf16(B))
    assert np.any(np.abs(ah @ bh + al @ bh - exact) > bound)
    # the model is far more accurate than a single bfloat16 product
    one = np.abs(ah @ bh - exact)
    assert err.max() < 0.05 * one.max()


def _known_three_parts(rng, shape):
    """Binary32 numbers a = h + m + l with h, m, l bfloat16 numbers chosen so
    that RNE_bf16(a) = h, RNE_bf16(a - h) = m and a - h - m = l: m below half
    an ulp of h and l below half an ulp of m (h and m with 8-bit significands
    that are not powers of two, so the spacing is the same on both sides),
    and a exact in binary32."""
    e = rng.integers(-3, 4, size=shape)
    h = rng.integers(129, 256, size=shape) * 2.0 ** (e - 7)
    # m: |m| < 2^(e-8), 8-bit significand with exponent e-9 (so m >= 2^(e-9))
    m = rng.integers(129, 256, size=shape) * 2.0 ** (e - 16)
    # l: |l| < half ulp of m = 2^(e-17), on the binary32 grid of a (last bit
    # 2^(e-23), 24 bits below the leading bit of h): at most 6 bits
    l = rng.integers(1, 64, size=shape) * 2.0 ** (e - 23)
    sm = rng.choice([-1.0, 1.0], size=shape)
    sl = rng.choice([-1.0, 1.0], size=shape)
    s = rng.choice([-1.0, 1.0], size=shape)
    return (s * h).astype(np.float32), (s * sm * m).astype(np.float32), (s * sl * l).astype(np.float32)


def test_three_way_split_of_numbers_with_known_parts():
    rng = np.random.default_rng(3)
    h, m, l = _known_three_parts(rng, 5000)
    a64 = h.astype(np.float64) + m + l
    a = a64.astype(np.float32)
    assert np.array_equal(a.astype(np.float64), a64)   # a exact in binary32 (24 bits span)
    hi, mid, lo = S.split3_bf16(a)
    assert np.array_equal(hi, h) and np.array_equal(mid, m) and np.array_equal(lo, l)


def test_six_product_sum_closed_form():
    """On numbers with known parts the model is the exact product minus the
    three smallest terms: (H+M+L)(H'+M'+L') - M L' - L M' - L L'."""
    rng = np.random.default_rng(4)
    Ha, Ma, La = _known_three_parts(rng, (9, 13))
    Hb, Mb, Lb = _known_three_parts(rng, (13, 6))
    A = (Ha.astype(np.float64) + Ma + La).astype(np.float32)
    B = (Hb.astype(np.float64) + Mb + Lb).astype(np.float32)
    h, m, l = (v.astype(np.float64) for v in (Ha, Ma, La))
    h2, m2, l2 = (v.astype(np.float64) for v in (Hb, Mb, Lb))
    want = (h + m + l) @ (h2 + m2 + l2) - m @ l2 - l @ m2 - l @ l2
    got = S.product_bf16x6(A, B)
    assert np.allclose(got, want, rtol=0, atol=1e-15 * np.abs(want).max())
    assert np.abs(got - A.astype(np.float64) @ B.astype(np.float64)).max() > 0


@pytest.mark.parametrize('k', [1, 7, 64, 300])
def test_six_product_model_within_error_bound(k):
    rng = np.random.default_rng(20 + k)
    A = rng.standard_normal((40, k)).astype(np.float32)
    B = (rng.standard_normal((k, 30)) * 10.0 ** rng.integers(-3, 4, size=(k, 30))).astype(np.float32)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    err = np.abs(S.product_bf16x6(A, B) - exact)
    bound = S.error_bound_bf16x6(A, B)
    assert np.all(err <= bound)
    # dropping the mid*mid term (2^-16 relative) breaks the 2^-24 bound
    ah, am, al = (v.astype(np.float64) for v in S.split3_bf16(A))
    bh, bm, bl = (v.astype(np.float64) for v in S.split3_bf16(B))
    assert np.any(np.abs(ah @ bl + al @ bh + ah @ bm + am @ bh + ah @ bh - exact) > bound)
    # about 2^8 more accurate than the three-product form
    assert err.max() < 2.0 ** -6 * np.abs(S.product_bf16x3(A, B) - exact).max()
