"""The allocation-free grouped GEMM (mdmrg_gemm_grouped_noalloc) against the
allocating entry point (mdmrg_gemm_grouped) through the C ABI: two calls in
a row on the same context, the second with a smaller input, each bitwise
equal to the allocating call (every tile variant accumulates in the same
order) and within the FP64 bound of the numpy product; a plan whose
descriptors exceed the static staging array is refused with EINVAL and
leaves the context usable."""
import numpy as np
import pytest

from test_gpu_gemm import _case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _ctx():
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    return mdmrg, mdmrg.Context(0)


def _run_both(ctx, rng, n_out, big):
    A, B, C, outs, segs, alphas, refs = _case(rng, n_out, big)
    dA = torch.from_numpy(A).to('cuda:0')
    dB = torch.from_numpy(B).to('cuda:0')
    c_alloc = torch.from_numpy(C).to('cuda:0')
    c_static = torch.from_numpy(C).to('cuda:0')
    print(f'[no-alloc] outputs={n_out} big={big} segments={len(segs)}', flush=True)
    ctx.gemm_grouped([dA, dB, c_alloc], outs, segs, alphas)
    ctx.gemm_grouped_noalloc([dA, dB, c_static], outs, segs, alphas)
    torch.cuda.synchronize()
    got, want = c_static.cpu().numpy(), c_alloc.cpu().numpy()
    assert np.array_equal(got, want)
    for (off, m, n, ldc, ref, aref) in refs:
        blk = got[off:off + m * ldc].reshape(m, ldc)
        assert np.all(np.abs(blk[:, :n] - ref) <= 1e-13 * (aref + 1.0))
        assert np.array_equal(blk[:, n:], C[off:off + m * ldc].reshape(m, ldc)[:, n:])


def test_noalloc_matches_allocating_entry_point_twice():
    mdmrg, ctx = _ctx()
    rng = np.random.default_rng(41)
    _run_both(ctx, rng, 60, True)     # first call: large blocks, many tiles
    _run_both(ctx, rng, 9, False)     # second call on the same staging array: smaller
    ctx.close()


def test_noalloc_forced_variants_and_oversized_plan():
    mdmrg, ctx = _ctx()
    rng = np.random.default_rng(42)
    for v in (0, 3):
        ctx.set_option(mdmrg.OPT_GEMM_VARIANT, v)
        _run_both(ctx, rng, 25, True)
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, -1)
    # 600000 1x1 outputs without segments: descriptors and tiles need more
    # than the 16 MiB staging array; refused on the host before any launch
    n = 600000
    outs = np.zeros((n, 8), dtype=np.int64)
    outs[:, 0] = 0
    outs[:, 1] = np.arange(n)
    outs[:, 2] = outs[:, 3] = outs[:, 4] = 1
    c = torch.zeros(n, dtype=torch.float64, device='cuda:0')
    print('[no-alloc] oversized plan', flush=True)
    with pytest.raises(mdmrg.MdmrgError) as ei:
        ctx.gemm_grouped_noalloc([c], outs, np.zeros((0, 8), dtype=np.int64), np.zeros(0))
    assert ei.value.code == mdmrg.EINVAL and 'static staging limit' in str(ei.value)
    _run_both(ctx, rng, 5, False)     # the context still works
    ctx.close()
