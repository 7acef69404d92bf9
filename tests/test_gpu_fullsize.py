"""Full-size checks at the benchmark's shapes, where the explicit-Fock oracle
cannot run: properties that hold at any size.

Workloads: the Hubbard model on a 6x6 torus (t=1, U=4, 18 up + 18 down,
momentum basis, U(1)xU(1)) at bond dimension D=1024 -- the benchmarked
configuration, same kernels and launch shapes -- and the spinless 8x8 torus
(t=1, V=2, N=32, momentum basis with a seeded rotation inside degenerate
shells, dense two-body integrals) at a reduced D.

Checked on each:
* Hermiticity of H_eff: |<z,Hx> - <Hz,x>| <= 1e-12 |Hx||z|.
* The diagonal (a separate kernel) against <e_i|H e_i> from full products.
* FP32 split form against FP64: max |y32 - y64| <= 1e-5 max |y64|.
* Energy invariance under a lossless move of the two-site centre: psi is
  the product of the two random centre tensors, so its rank across the
  middle bond is at most that bond's dimension and decimation with D kept
  states discards nothing; after renormalisation and StVec the new psi
  represents the same state, so <psi|H|psi>/<psi|psi> must agree at the two
  bonds to rounding (a4 at two bonds, a6, a7 and a8 together).
"""
import numpy as np
import pytest

import seeded_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def log(msg):
    print(msg, flush=True)


def _lib():
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    return mdmrg


def _hubbard6x6(mdmrg):
    T, V = mdmrg.build_lattice(mdmrg.HUBBARD, mdmrg.MOMENTUM, 6, 6, 1.0, 4.0)
    return 36, True, (18, 18), T, V


def _spinless8x8_rotated(mdmrg):
    T, V = mdmrg.build_lattice(mdmrg.SPINLESS, mdmrg.MOMENTUM, 8, 8, 1.0, 2.0)
    R = si.shell_rotation(np.diag(T), 0)
    T, V = mdmrg.rotate_modes(R, T, V, False)
    return 64, False, (32, 0), T, V


CASES = {
    'hubbard_6x6_momentum_D1024': (_hubbard6x6, 1024, 16),
    'spinless_8x8_rotated_D512': (_spinless8x8_rotated, 512, 31),
}


def _two_site_psi(blocks, ne, bonds, tens, l, spinful):
    """psi(a,s1,s2,b) = sum_c A_l(a,s1,c) A_{l+1}(c,s2,b) in the library
    layout (sector c of the middle bond fixed by the quantum numbers)."""
    psi = np.zeros(ne)
    A, B = tens[l], tens[l + 1]
    mid = bonds[l + 1]
    for (a, s1, s2, b, off, m, n) in blocks:
        blk = np.zeros((m, n))
        for c in range(len(mid)):
            x, y = A.get((a, s1, c)), B.get((c, s2, b))
            if x is not None and y is not None:
                blk += x @ y
        psi[off:off + m * n] = blk.ravel()
    return psi


@pytest.mark.parametrize('name', list(CASES))
def test_fullsize_properties(name):
    mdmrg = _lib()
    make, D, l = CASES[name]
    n, spin, target, T, V = make(mdmrg)
    bonds = si.bond_profile(n, spin, target, D)
    tens = si.random_mps(bonds, spin, 1, l)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, V, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    log(f'[fullsize] {name}: environments at bond {l}')
    ctx.prepare_bond(l)
    blocks, ne = ctx.psi_layout()
    cost = ctx.heff_cost()
    log(f'[fullsize] {name}: |psi| = {ne}, {cost["n_terms"]} terms, {cost["flop"] / 1e12:.3f} TFLOP per product')
    hist = ctx.heff_histogram()
    assert abs(sum(hist.values()) - cost['flop']) <= 1e-9 * cost['flop']
    dev = 'cuda:0'
    x = torch.from_numpy(si.random_vector(ne, 3)).to(dev)
    z = torch.from_numpy(si.random_vector(ne, 4)).to(dev)
    hx, hz = torch.zeros_like(x), torch.zeros_like(x)
    ctx.heff_apply(x, hx)
    ctx.heff_apply(z, hz)
    lhs, rhs = float(torch.dot(z, hx)), float(torch.dot(hz, x))
    assert abs(lhs - rhs) <= 1e-12 * float(hx.norm()) * float(z.norm()), (lhs, rhs)
    # diagonal kernel vs full products on sampled unit vectors
    dg = torch.zeros_like(x)
    ctx.heff_diag(dg)
    e, he = torch.zeros_like(x), torch.zeros_like(x)
    for i in np.random.default_rng(5).choice(ne, 3, replace=False):
        e.zero_()
        e[int(i)] = 1.0
        ctx.heff_apply(e, he)
        assert abs(float(he[int(i)]) - float(dg[int(i)])) <= 1e-12 * float(he.abs().max())
    # FP32 split form
    h32 = torch.zeros_like(x)
    ctx.heff_apply(x, h32, prec=mdmrg.FP32)
    err32 = float((h32 - hx).abs().max() / hx.abs().max())
    log(f'[fullsize] {name}: FP32 vs FP64 max rel {err32:.2e}')
    assert err32 <= 1e-5
    # energy invariance under a lossless centre move
    psi = torch.from_numpy(_two_site_psi(blocks, ne, bonds, tens, l, spin)).to(dev)
    hp = torch.zeros_like(psi)
    ctx.heff_apply(psi, hp)
    e0 = float(torch.dot(psi, hp)) / float(torch.dot(psi, psi))
    trunc, _, _ = ctx.decimate(psi, sum(m for _, m in bonds[l + 1]), +1)
    assert trunc <= 1e-12
    ctx.renormalize(+1)
    _, ne2 = ctx.psi_layout()
    psi2 = torch.zeros(ne2, dtype=torch.float64, device=dev)
    ctx.stvec(psi, psi2)
    hp2 = torch.zeros_like(psi2)
    ctx.heff_apply(psi2, hp2)
    e1 = float(torch.dot(psi2, hp2)) / float(torch.dot(psi2, psi2))
    log(f'[fullsize] {name}: <H> at bond {l} = {e0:.14f}, at bond {l + 1} = {e1:.14f}')
    assert abs(e1 - e0) <= 1e-11 * max(1.0, abs(e0))
    ctx.close()


@pytest.mark.parametrize('name', list(CASES))
def test_fullsize_compressed_products_match_uncompressed(name):
    """The interpolative compression of the N^L x C^R products is exact to
    rounding: the product with and without it agree to 1e-12 (relative to
    max |H x|), and it never increases the number of products."""
    mdmrg = _lib()
    make, D, l = CASES[name]
    n, spin, target, T, V = make(mdmrg)
    bonds = si.bond_profile(n, spin, target, D)
    tens = si.random_mps(bonds, spin, 1, l)
    ys, terms = [], []
    for comp in (1, 0):
        ctx = mdmrg.Context(0)
        ctx.set_option(mdmrg.OPT_COMPRESS, comp)
        ctx.set_hamiltonian(n, spin, T, V, target)
        ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
        ctx.prepare_bond(l)
        _, ne = ctx.psi_layout()
        x = torch.from_numpy(si.random_vector(ne, 3)).to('cuda:0')
        y = torch.zeros_like(x)
        ctx.heff_apply(x, y)
        ys.append(y.cpu().numpy())
        terms.append(ctx.heff_cost()['n_terms'])
        ctx.close()
    log(f'[fullsize] {name}: products {terms[1]} -> {terms[0]} with compression')
    assert terms[0] <= terms[1]
    assert np.abs(ys[0] - ys[1]).max() <= 1e-12 * np.abs(ys[1]).max()
