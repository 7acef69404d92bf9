"""Kernel-level parity of the grouped sector-block GEMM (mdmrg_gemm_grouped)
against plain numpy products on random uneven groups: every combination of
transposed / identity operands, ragged tails, outputs routed to both the
64x64 workgroup tiles and the 32x32 wave tiles, K concatenated over many
segments, accumulate and overwrite.  FP64: |C - C_ref| <= 1e-13 * sum|A||B|.

Split forms (mdmrg_gemm_grouped_split, FP32 buffers) against the oracle's
product model of the same form, evaluated in FP64: the kernel may differ
from it only by binary32 accumulation, |C - C_model| <= 2^-24 (4K + 16)
(|C0| + sum|alpha A||B|) with K the summed depth of the output; the 3xBF16
form also stays within the model's error bound of the exact product.
"""
import numpy as np
import pytest

from oracle import split as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _ctx():
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    return mdmrg, mdmrg.Context(0)


def _case(rng, n_out, big):
    A_parts, B_parts, segs, outs, refs, absrefs = [], [], [], [], [], []
    a_len = b_len = c_len = 0
    alphas = []
    C0 = []
    for o in range(n_out):
        if big:
            m, n = int(rng.integers(40, 170)), int(rng.integers(40, 170))
        else:
            m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        ldc = n + int(rng.integers(0, 3))
        acc = int(rng.integers(0, 2))
        c0 = rng.standard_normal((m, ldc))
        ref = c0[:, :n].copy() if acc else np.zeros((m, n))
        aref = np.abs(ref)
        seg_begin = len(segs)
        for _ in range(int(rng.integers(1, 6))):
            k = int(rng.integers(1, 90))
            flags = int(rng.integers(0, 4))
            if rng.random() < 0.15:   # identity left factor (k = m)
                k = m
                flags |= 4
            al = float(rng.standard_normal())
            if flags & 4:
                Aop = np.eye(m)
                a_off, lda = 0, 0
            elif flags & 1:       # A stored k x m
                lda = m + int(rng.integers(0, 3))
                Am = rng.standard_normal((k, lda))
                Aop = Am[:, :m].T
                a_off = a_len
                A_parts.append(Am.ravel())
                a_len += Am.size
            else:
                lda = k + int(rng.integers(0, 3))
                Am = rng.standard_normal((m, lda))
                Aop = Am[:, :k]
                a_off = a_len
                A_parts.append(Am.ravel())
                a_len += Am.size
            if flags & 2:         # B stored n x k
                ldb = k + int(rng.integers(0, 3))
                Bm = rng.standard_normal((n, ldb))
                Bop = Bm[:, :k].T
            else:
                ldb = n + int(rng.integers(0, 3))
                Bm = rng.standard_normal((k, ldb))
                Bop = Bm[:, :n]
            b_off = b_len
            B_parts.append(Bm.ravel())
            b_len += Bm.size
            segs.append([0, a_off, lda, 1, b_off, ldb, k, flags])
            alphas.append(al)
            ref += al * Aop @ Bop
            aref += abs(al) * np.abs(Aop) @ np.abs(Bop)
        outs.append([2, c_len, m, n, ldc, seg_begin, len(segs) - seg_begin, acc])
        C0.append(c0.ravel())
        refs.append((c_len, m, n, ldc, ref, aref))
        c_len += c0.size
    A = np.concatenate(A_parts) if A_parts else np.zeros(1)
    B = np.concatenate(B_parts)
    C = np.concatenate(C0)
    return A, B, C, np.array(outs), np.array(segs), np.array(alphas), refs


@pytest.mark.parametrize('variant', [0, 1, 2, 3])
@pytest.mark.parametrize('big,n_out,seed', [(False, 300, 0), (True, 40, 1), (False, 2000, 2), (True, 7, 3)])
def test_grouped_gemm_matches_numpy(big, n_out, seed, variant):
    """Every tile variant (forced), FP64."""
    mdmrg, ctx = _ctx()
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, variant)
    rng = np.random.default_rng(seed)
    A, B, C, outs, segs, alphas, refs = _case(rng, n_out, big)
    dA = torch.from_numpy(A).to('cuda:0')
    dB = torch.from_numpy(B).to('cuda:0')
    dC = torch.from_numpy(C).to('cuda:0')
    print(f'[gemm parity] variant={variant} big={big} outputs={n_out} segments={len(segs)}', flush=True)
    ctx.gemm_grouped([dA, dB, dC], outs, segs, alphas)
    Cg = dC.cpu().numpy()
    for (off, m, n, ldc, ref, aref) in refs:
        got = Cg[off:off + m * ldc].reshape(m, ldc)[:, :n]
        assert np.all(np.abs(got - ref) <= 1e-13 * (aref + 1.0))
        # padding columns of C are untouched
    for (off, m, n, ldc, ref, aref) in refs:
        if ldc > n:
            assert np.array_equal(Cg[off:off + m * ldc].reshape(m, ldc)[:, n:],
                                  C[off:off + m * ldc].reshape(m, ldc)[:, n:])


def test_grouped_gemm_rejects_out_of_range():
    mdmrg, ctx = _ctx()
    dA = torch.zeros(100, dtype=torch.float64, device='cuda:0')
    dB = torch.zeros(100, dtype=torch.float64, device='cuda:0')
    dC = torch.zeros(100, dtype=torch.float64, device='cuda:0')
    # B operand 10 x 11 does not fit in 100 doubles
    outs = np.array([[2, 0, 5, 11, 11, 0, 1, 0]])
    segs = np.array([[0, 0, 10, 1, 0, 11, 10, 0]])
    with pytest.raises(mdmrg.MdmrgError) as e:
        ctx.gemm_grouped([dA, dB, dC], outs, segs, np.ones(1))
    assert e.value.code == mdmrg.EINVAL
    # output larger than its buffer
    outs = np.array([[2, 50, 10, 10, 10, 0, 0, 0]])
    with pytest.raises(mdmrg.MdmrgError):
        ctx.gemm_grouped([dA, dB, dC], outs, np.zeros((0, 8)), np.zeros(0))


def _operand_views(A, B, seg, m, n):
    """op(A) (m x k) and op(B) (k x n) of one segment descriptor, read from
    the flat host buffers; an identity A is returned as None."""
    _, a_off, lda, _, b_off, ldb, k, flags = (int(v) for v in seg)
    if flags & 4:
        Aop = None
    elif flags & 1:
        Aop = A[a_off:a_off + k * lda].reshape(k, lda)[:, :m].T
    else:
        Aop = A[a_off:a_off + m * lda].reshape(m, lda)[:, :k]
    if flags & 2:
        Bop = B[b_off:b_off + n * ldb].reshape(n, ldb)[:, :k].T
    else:
        Bop = B[b_off:b_off + k * ldb].reshape(k, ldb)[:, :n]
    return Aop, Bop, k


@pytest.mark.parametrize('variant', [0, 1, 2, 3])
@pytest.mark.parametrize('prec_name', ['FP32', 'BF16X3', 'BF16X6'])
@pytest.mark.parametrize('big,n_out,seed', [(False, 300, 0), (True, 40, 1), (True, 7, 3)])
def test_split_grouped_gemm_matches_product_model(prec_name, big, n_out, seed, variant):
    mdmrg, ctx = _ctx()
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, variant)
    prec = getattr(mdmrg, prec_name)
    rng = np.random.default_rng(100 + seed)
    A, B, C, outs, segs, alphas, _ = _case(rng, n_out, big)
    A32, B32, C32 = (np.ascontiguousarray(v, dtype=np.float32) for v in (A, B, C))
    dA, dB, dC = (torch.from_numpy(v).to('cuda:0') for v in (A32, B32, C32))
    print(f'[gemm parity {prec_name}] variant={variant} big={big} outputs={n_out} segments={len(segs)}', flush=True)
    ctx.gemm_grouped([dA, dB, dC], outs, segs, alphas, prec=prec)
    Cg = dC.cpu().numpy()
    model = {'FP32': S.product_fp32, 'BF16X3': S.product_bf16x3, 'BF16X6': S.product_bf16x6}[prec_name]
    split_bound = {'BF16X3': S.error_bound_bf16x3, 'BF16X6': S.error_bound_bf16x6}.get(prec_name)
    worst = 0.0
    for (_, off, m, n, ldc, s0, ns, acc) in outs:
        c0 = C32[off:off + m * ldc].reshape(m, ldc)[:, :n].astype(np.float64)
        want = c0.copy() if acc else np.zeros((m, n))
        exact = want.copy()
        scale = np.abs(want)
        bound = np.zeros((m, n))
        ktot = 0
        for q in range(s0, s0 + ns):
            Aop, Bop, k = _operand_views(A32, B32, segs[q], m, n)
            if Aop is None:
                Aop = np.eye(m, dtype=np.float32)
            Af = S.fold_alpha(alphas[q], Aop)
            want += model(Af, Bop)
            exact += Af.astype(np.float64) @ Bop.astype(np.float64)
            scale += np.abs(Af.astype(np.float64)) @ np.abs(Bop.astype(np.float64))
            if split_bound is not None:
                bound += split_bound(Af, Bop)
            ktot += k
        got = Cg[off:off + m * ldc].reshape(m, ldc)[:, :n].astype(np.float64)
        tol = 2.0 ** -24 * (4 * ktot + 16) * (scale + 1e-30)
        assert np.all(np.abs(got - want) <= tol), (prec_name, off)
        worst = max(worst, float((np.abs(got - exact) / (scale + 1e-30)).max()))
        if split_bound is not None:
            assert np.all(np.abs(got - exact) <= bound + tol)
        if ldc > n:
            assert np.array_equal(Cg[off:off + m * ldc].reshape(m, ldc)[:, n:],
                                  C32[off:off + m * ldc].reshape(m, ldc)[:, n:])
    print(f'[gemm parity {prec_name}] max |C - exact| / sum|A||B| = {worst:.2e}', flush=True)
    # different arithmetic: 3xBF16 is visibly less exact; 6xBF16 keeps the
    # mid*mid and hi*mid terms and is as exact as the FP32 form
    if prec_name == 'BF16X3':
        assert worst > 2.0 ** -22
    else:
        assert worst < 2.0 ** -19


def test_split_grouped_gemm_rejects_bad_precision():
    mdmrg, ctx = _ctx()
    d = torch.zeros(100, dtype=torch.float32, device='cuda:0')
    outs = np.array([[2, 0, 5, 5, 5, 0, 1, 0]])
    segs = np.array([[0, 0, 5, 1, 0, 5, 5, 0]])
    with pytest.raises(mdmrg.MdmrgError) as e:
        ctx.gemm_grouped([d, d, d], outs, segs, np.ones(1), prec=mdmrg.FP64 + 7)
    assert e.value.code == mdmrg.EUNSUP


def test_forced_variant_option_rejects_unknown_variant():
    mdmrg, ctx = _ctx()
    with pytest.raises(mdmrg.MdmrgError) as e:
        ctx.set_option(mdmrg.OPT_GEMM_VARIANT, 4)
    assert e.value.code == mdmrg.EINVAL


@pytest.mark.parametrize('variant', [0, 1, 2, 3])
def test_tall_output_beyond_16bit_tile_rows(variant):
    """One output with more tile rows than a 16-bit index holds (the a3
    operator accumulation at D=4096 produces such outputs: one row per
    operator element).  Regression test for tile indices that wrapped."""
    mdmrg, ctx = _ctx()
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, variant)
    m, k, n = 64 * 32768 + 1000, 5, 3
    rng = np.random.default_rng(7)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    dA = torch.from_numpy(A.ravel()).to('cuda:0')
    dB = torch.from_numpy(B.ravel()).to('cuda:0')
    dC = torch.zeros(m * n, dtype=torch.float64, device='cuda:0')
    print(f'[gemm tall] variant={variant} m={m}', flush=True)
    outs = np.array([[2, 0, m, n, n, 0, 1, 0]])
    segs = np.array([[0, 0, k, 1, 0, n, k, 0]])
    ctx.gemm_grouped([dA, dB, dC], outs, segs, np.array([1.5]))
    got = dC.cpu().numpy().reshape(m, n)
    ref = 1.5 * (A @ B)
    assert np.all(np.abs(got - ref) <= 1e-13 * (1.5 * np.abs(A) @ np.abs(B) + 1.0))


@pytest.mark.parametrize('variant', [0, 1, 2, 3])
def test_degenerate_groups(variant):
    """Degenerate shapes, exact results: a launch with no outputs leaves C
    alone; an output whose segments all have k = 0 (or that has no
    segment) is zero when overwritten and unchanged when accumulated; 1x1
    outputs and 1-deep products."""
    mdmrg, ctx = _ctx()
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, variant)
    A = torch.arange(1.0, 65.0, dtype=torch.float64, device='cuda:0')
    B = torch.arange(2.0, 66.0, dtype=torch.float64, device='cuda:0')
    C = torch.full((64,), 7.0, dtype=torch.float64, device='cuda:0')
    ctx.gemm_grouped([A, B, C], np.zeros((0, 8)), np.zeros((0, 8)), np.zeros(0))
    assert torch.all(C == 7.0)
    outs = np.array([
        [2, 0, 3, 4, 4, 0, 1, 0],     # k = 0, overwrite -> zeros
        [2, 12, 3, 4, 4, 1, 1, 1],    # k = 0, accumulate -> unchanged
        [2, 24, 2, 2, 2, 2, 0, 0],    # no segment, overwrite -> zeros
        [2, 28, 1, 1, 1, 2, 1, 1],    # 1x1, k = 1, accumulate: 7 + 0.5 * A[5] * B[9]
        [2, 29, 1, 1, 1, 3, 1, 0],    # 1x1, k = 64 (row of A times column of B)
    ])
    segs = np.array([
        [0, 0, 1, 1, 0, 4, 0, 0],
        [0, 0, 1, 1, 0, 4, 0, 0],
        [0, 5, 1, 1, 9, 1, 1, 0],
        [0, 0, 64, 1, 0, 1, 64, 0],
    ])
    ctx.gemm_grouped([A, B, C], outs, segs, np.array([1.0, 1.0, 0.5, 1.0]))
    c = C.cpu().numpy()
    a, b = np.arange(1.0, 65.0), np.arange(2.0, 66.0)
    assert np.all(c[0:12] == 0.0)
    assert np.all(c[12:24] == 7.0)
    assert np.all(c[24:28] == 0.0)
    assert c[28] == 7.0 + 0.5 * a[5] * b[9]
    assert c[29] == float(a @ b)            # integers: exact in FP64
    assert np.all(c[30:] == 7.0)
