"""Context options that change how a step is computed, not what it computes.

* Keep modes of the block environments (MDMRG_OPT_KEEP_ENVS 0-3): a walk of
  three steps to the right from the same MPS and start vector gives bitwise
  the same energies and final vector in every mode (modes that dropped a
  block rebuild it with the same plans; every tile variant accumulates in
  the same order).
* Davidson and mixed-precision options (restart size, Olsen correction, the
  FP32 stage between 3xBF16 and FP64, the Ritz-vector hand-over, the
  defect-corrected split stages): every combination reaches the FP64
  residual tolerance 1e-7 (checked with an FP64 product of the returned
  vector) and the energy of a tight FP64 solve (1e-10) to 1e-9 relative,
  the split-precision target
  (Sec. II.A: the eigenpair is the FP64 one whatever precision carried the
  iterations).

Workload: Hubbard 6x6 torus (t=1, U=4, 18 up + 18 down), momentum basis,
U(1)xU(1), Fock-count sector profile at D=384, seeded random isometries.
"""
import numpy as np
import pytest

import seeded_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _setup(keep=1, l=15, D=384):
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    T, V = mdmrg.build_lattice(mdmrg.HUBBARD, mdmrg.MOMENTUM, 6, 6, 1.0, 4.0)
    n, spin, target = 36, True, (18, 18)
    bonds = si.bond_profile(n, spin, target, D)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, V, target)
    ctx.set_option(mdmrg.OPT_KEEP_ENVS, keep)
    ctx.set_mps(*si.flatten_mps(bonds, si.random_mps(bonds, spin, 1, l), spin))
    ctx.prepare_bond(l)
    return mdmrg, ctx, D


def _walk(keep):
    mdmrg, ctx, D = _setup(keep)
    _, ne = ctx.psi_layout()
    x = torch.from_numpy(si.random_vector(ne, 3)).to('cuda:0')
    energies = []
    for step in range(3):
        print(f'[options] keep={keep} step {step} dim {ne}', flush=True)
        e, r, nmv, ok = ctx.davidson(x, tol=1e-8, max_iter=400)
        assert ok
        energies.append(e)
        ctx.decimate(x, D, +1)
        ctx.renormalize(+1)
        _, ne = ctx.psi_layout()
        x2 = torch.empty(ne, dtype=torch.float64, device='cuda:0')
        ctx.stvec(x, x2)
        x = x2
    out = (energies, x.cpu().numpy())
    ctx.close()
    return out


def test_keep_modes_walk_identically():
    e1, x1 = _walk(1)
    for keep in (0, 2, 3):
        e, x = _walk(keep)
        assert e == e1, (keep, e, e1)
        assert np.array_equal(x, x1), keep


def test_davidson_and_mixed_options_reach_the_fp64_energy():
    mdmrg, ctx, D = _setup()
    _, ne = ctx.psi_layout()
    x0 = torch.from_numpy(si.random_vector(ne, 3)).to('cuda:0')
    x = x0.clone()
    e_ref, r, n, ok = ctx.davidson(x, tol=1e-10, max_iter=800)
    assert ok
    tol = 1e-7
    cases = [(opt, val) for opt, val in ((mdmrg.OPT_DAVIDSON_KEEP, 6), (mdmrg.OPT_DAVIDSON_OLSEN, 1))]
    for opt, val in cases:
        ctx.set_option(opt, val)
        x = x0.clone()
        e, r, n, ok = ctx.davidson(x, tol=tol, max_iter=800)
        print(f'[options] FP64 option {opt}={val}: {n} products, E={e:.12f}', flush=True)
        assert ok and r <= tol and abs(e - e_ref) <= 1e-9 * abs(e_ref)
        ctx.set_option(opt, 2 if opt == mdmrg.OPT_DAVIDSON_KEEP else 0)
    for ladder, hand, olsen, corr in ((0, 1, 0, 1), (0, 1, 0, 0), (1, 1, 0, 1), (0, 4, 0, 0), (1, 3, 1, 1)):
        ctx.set_option(mdmrg.OPT_MIXED_LADDER, ladder)
        ctx.set_option(mdmrg.OPT_MIXED_HANDOVER, hand)
        ctx.set_option(mdmrg.OPT_DAVIDSON_OLSEN, olsen)
        ctx.set_option(mdmrg.OPT_MIXED_CORRECT, corr)
        for prec in (mdmrg.FP32, mdmrg.BF16X3, mdmrg.BF16X6):
            x = x0.clone()
            e, r, n64, ns, ok = ctx.davidson_mixed(x, tol=tol, tol_split=tol, prec_split=prec, max_iter=800)
            print(f'[options] mixed prec={prec} ladder={ladder} handover={hand} olsen={olsen} correct={corr}: '
                  f'{ns} split + {n64} FP64 products, E={e:.12f}', flush=True)
            assert ok and r <= tol, (prec, ladder, hand, olsen, corr, r)
            assert abs(e - e_ref) <= 1e-9 * abs(e_ref), (prec, ladder, hand, olsen, corr, e, e_ref)
            assert n64 >= 1
            # the returned vector meets tol on the FP64 operator
            hx = torch.empty_like(x)
            ctx.heff_apply(x, hx)
            th = float(torch.dot(x, hx))
            assert float(torch.linalg.vector_norm(hx - th * x)) <= 1.01 * tol
    ctx.set_option(mdmrg.OPT_MIXED_CORRECT, 0)
    for opt in (mdmrg.OPT_MIXED_HANDOVER, mdmrg.OPT_DAVIDSON_KEEP):
        with pytest.raises(mdmrg.MdmrgError):
            ctx.set_option(opt, 0)
    ctx.close()
