"""Graph replay and tile-variant autotuning of the H_eff product.

* The first products of a bond run the kernel's tile variants in turn (the
  autotuner's trials) and then the fastest; every variant accumulates each
  output in the same order, so all these products must agree bit for bit.
* With MDMRG_OPT_GRAPH the product is captured once and replayed; every
  replay, with eager work and synchronisations of the program in between,
  must agree bit for bit with the eager product of a second context, in FP64
  and in both split forms (FP32, 3xBF16).
* A Davidson solve driven by graph replays reaches the same energy.
"""
import numpy as np
import pytest

import seeded_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _lib():
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    return mdmrg


def _context(mdmrg, l=9):
    # spinless 4x5 torus in real space, D=300: tens of thousands of tiles per launch
    T, V = mdmrg.build_lattice(mdmrg.SPINLESS, mdmrg.REAL, 4, 5, 1.0, 1.0)
    n, target = 20, (10, 0)
    bonds = si.bond_profile(n, False, target, 300)
    tens = si.random_mps(bonds, False, 4, l)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, False, T, V, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, False))
    ctx.prepare_bond(l)
    return ctx


def test_variants_and_graph_replays_are_bitwise_identical():
    mdmrg = _lib()
    dev = 'cuda:0'
    a, b = _context(mdmrg), _context(mdmrg)
    _, ne = a.psi_layout()
    x0 = torch.from_numpy(si.random_vector(ne, 1)).to(dev)
    ys = []
    for _ in range(6):   # four variant trials, then the decision, which runs the chosen variant
        y = torch.zeros_like(x0)
        a.heff_apply(x0, y)
        ys.append(y)
    for y in ys[1:]:
        assert torch.equal(y, ys[0])
    print(f'[graph] {len(ys)} eager products agree bitwise, |psi| = {ne}', flush=True)
    # the split forms' variants agree bit for bit too (same K order per element)
    for prec in (mdmrg.FP32, mdmrg.BF16X3, mdmrg.BF16X6):
        ys = []
        for _ in range(5):
            y = torch.zeros_like(x0)
            a.heff_apply(x0, y, prec=prec)
            ys.append(y)
        for y in ys[1:]:
            assert torch.equal(y, ys[0]), prec
    a.set_option(mdmrg.OPT_GRAPH, 1)
    # every form has finished its variant trials above; 8 products each,
    # with capture at the first of them
    for prec in (mdmrg.FP64, mdmrg.FP32, mdmrg.BF16X3, mdmrg.BF16X6):
        for r in range(8):
            x = torch.from_numpy(si.random_vector(ne, 10 + r)).to(dev)
            yg, ye = torch.zeros_like(x), torch.zeros_like(x)
            a.heff_apply(x, yg, prec=prec)
            b.heff_apply(x, ye, prec=prec)      # eager work of another context in between
            torch.cuda.synchronize()
            _ = (x * 2.0).sum().item()          # and some eager torch work
            assert torch.equal(yg, ye), (prec, r)
    st = a.stats()
    assert st['graph64_launches'] >= 1 and st['graph32_launches'] >= 1 and st['graphbf3_launches'] >= 1
    assert st['graphbf6_launches'] >= 1
    print(f"[graph] replays: FP64 {int(st['graph64_launches'])}, FP32 {int(st['graph32_launches'])}, "
          f"3xBF16 {int(st['graphbf3_launches'])}, 6xBF16 {int(st['graphbf6_launches'])}", flush=True)
    a.close()
    b.close()


def test_davidson_with_graph_replays_matches_eager():
    mdmrg = _lib()
    dev = 'cuda:0'
    a, b = _context(mdmrg, 8), _context(mdmrg, 8)
    a.set_option(mdmrg.OPT_GRAPH, 1)
    _, ne = a.psi_layout()
    x = torch.from_numpy(si.random_vector(ne, 2)).to(dev)
    xa, xb = x.clone(), x.clone()
    ea, ra, na, ca = a.davidson(xa, tol=1e-9, max_iter=300)
    eb, rb, nb, cb = b.davidson(xb, tol=1e-9, max_iter=300)
    assert ca and cb
    assert abs(ea - eb) <= 1e-12 * abs(eb)
    assert a.stats()['graph64_launches'] >= 1
    a.close()
    b.close()
