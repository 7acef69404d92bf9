"""Kernel-level parity of the grouped sector-block GEMM (mdmrg_gemm_grouped)
against plain numpy products on random uneven groups: every combination of
transposed / identity operands, ragged tails, outputs routed to both the
64x64 workgroup tiles and the 32x32 wave tiles, K concatenated over many
segments, accumulate and overwrite.  FP64: |C - C_ref| <= 1e-13 * sum|A||B|.
"""
import numpy as np
import pytest

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


@pytest.mark.parametrize('big,n_out,seed', [(False, 300, 0), (True, 40, 1), (False, 2000, 2), (True, 7, 3)])
def test_grouped_gemm_matches_numpy(big, n_out, seed):
    mdmrg, ctx = _ctx()
    rng = np.random.default_rng(seed)
    A, B, C, outs, segs, alphas, refs = _case(rng, n_out, big)
    dA = torch.from_numpy(A).to('cuda:0')
    dB = torch.from_numpy(B).to('cuda:0')
    dC = torch.from_numpy(C).to('cuda:0')
    print(f'[gemm parity] big={big} outputs={n_out} segments={len(segs)}', flush=True)
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
