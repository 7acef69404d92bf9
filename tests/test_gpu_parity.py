"""GPU parity of the library (through the C ABI) against the CPU oracle.

H_eff psi is compared element by element with the oracle's literal
projection P^T H P psi (Sec. II.A) on the same seeded MPS and vector; the
Davidson eigenvalue with the lowest eigenvalue of the same H_eff; full
two-site sweeps with exact diagonalisation.  Tolerances follow from FP64
arithmetic: elementwise |y - y_ref| <= 1e-12 * max|y_ref| (sums of O(10^3)
products of O(1) entries in double precision), energies 1e-12 relative.
"""
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import dmrg, ed
from oracle import integrals as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip('torch')


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2311_14106_amd import mdmrg
    return mdmrg


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to('cuda:0')


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def randspin(n, seed):
    rng = np.random.default_rng(seed)
    t = rng.standard_normal((n, n))
    t = t + t.T
    v = rng.standard_normal((n,) * 4)
    v = v + v.transpose(3, 2, 1, 0)
    T = np.kron(t, np.eye(2))
    W = np.zeros((2 * n,) * 4)
    for s in (0, 1):
        for u in (0, 1):
            W[s::2, u::2, u::2, s::2] = v
    return T, W


def randless(n, seed):
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((n, n))
    T = T + T.T
    W = rng.standard_normal((n,) * 4)
    W = W + W.transpose(3, 2, 1, 0)
    return T, W


CASES = {
    # name: (builder, n_sites, spin_half, target, D, bonds to test)
    'spinless_4x4_real_D64': (lambda: I.spinless_real_space(4, 4, 1.0, 1.0), 16, False, (8, 0), 64, [0, 3, 7, 13]),
    'spinless_4x5_real_D300': (lambda: I.spinless_real_space(4, 5, 1.0, 1.0), 20, False, (10, 0), 300, [9]),
    'hubbard_3x3_momentum_D64': (lambda: I.hubbard_momentum(3, 3, 1.0, 4.0), 9, True, (4, 4), 64, [1, 3, 6]),
    'spinless_dense_random_8': (lambda: randless(8, 3), 8, False, (4, 0), 40, [0, 2, 3, 5]),
    'spinful_dense_random_5': (lambda: randspin(5, 4), 5, True, (3, 2), 40, [0, 1, 2, 3]),
    'spinless_4x4_rotated_D128': (lambda: I.rotate(*I.spinless_real_space(4, 4, 1.0, 1.0),
                                                    si.random_orthogonal(16, 0)), 16, False, (8, 0), 128, [7]),
}


@pytest.mark.parametrize('name', list(CASES))
def test_heff_and_diag_match_oracle(name):
    mdmrg = _gpu()
    build, n, spin, target, D, ls = CASES[name]
    T, W = build()
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, D)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    for l in ls:
        log(f'[heff parity] {name} bond {l}')
        tens = si.random_mps(bonds, spin, 10 + l, l)
        mps = dmrg.MPS(ch, bonds, tens)
        prob = dmrg.TwoSiteProblem(mps, l)
        ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
        ctx.prepare_bond(l)
        blocks, ne = ctx.psi_layout()
        assert ne == prob.dim
        assert blocks == list(prob.layout)      # integer tables: bit-exact
        x = si.random_vector(ne, 100 + l)
        y_ref = prob.matvec(x)
        xd = to_dev(x)
        yd = torch.zeros(ne, dtype=torch.float64, device='cuda:0')
        ctx.heff_apply(xd, yd)
        y = yd.cpu().numpy()
        assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max(), name
        # diagonal on sampled entries
        dd = torch.zeros(ne, dtype=torch.float64, device='cuda:0')
        ctx.heff_diag(dd)
        d = dd.cpu().numpy()
        for i in np.random.default_rng(l).choice(ne, min(ne, 12), replace=False):
            e = np.zeros(ne)
            e[i] = 1.0
            assert abs(prob.matvec(e)[i] - d[i]) <= 1e-12 * max(1.0, abs(d[i]))
        # Hermiticity of the device operator
        z = si.random_vector(ne, 200 + l)
        hz = torch.zeros_like(yd)
        ctx.heff_apply(to_dev(z), hz)
        hz = hz.cpu().numpy()
        assert abs(x @ hz - z @ y) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(z)
        # the shape histogram partitions the algorithmic FLOP of the product
        cost, hist = ctx.heff_cost(), ctx.heff_histogram()
        assert abs(sum(hist.values()) - cost['flop']) <= 1e-9 * cost['flop']


@pytest.mark.parametrize('name,l', [('hubbard_3x3_momentum_D64', 3), ('spinless_4x4_real_D64', 7)])
def test_davidson_matches_lowest_eigenvalue(name, l):
    mdmrg = _gpu()
    build, n, spin, target, D, _ = CASES[name]
    T, W = build()
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, D)
    tens = si.random_mps(bonds, spin, 3, l)
    prob = dmrg.TwoSiteProblem(dmrg.MPS(ch, bonds, tens), l)
    e_ref, _ = prob.lowest(v0=si.random_vector(prob.dim, 1))
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    log(f'[davidson] {name} bond {l} dim {ne}')
    x = to_dev(si.random_vector(ne, 2))
    e, r, nmv, conv = ctx.davidson(x, tol=1e-9, max_iter=400)
    assert conv and r <= 1e-9
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    # returned vector is normalised and is an eigenvector
    xv = x.cpu().numpy()
    assert abs(np.linalg.norm(xv) - 1.0) < 1e-12
    assert np.linalg.norm(prob.matvec(xv) - e * xv) <= 2e-9


def _sweep(mdmrg, T, W, n, spin, target, D0, sched, nsw, tol=1e-9):
    bonds = si.bond_profile(n, spin, target, D0)
    tens = si.random_mps(bonds, spin, 1, 0)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    return ctx.sweep(nsw, sched, tol)


def test_sweeps_spinless_4x4_reach_exact_energy():
    mdmrg = _gpu()
    T, W = mdmrg.build_lattice(0, 0, 4, 4, 1.0, 1.0)
    e_ed = -7.2294974091395305   # tests/golden/ed_energies.json
    log('[sweep] spinless 4x4 D=64 (6 sweeps)')
    E64 = _sweep(mdmrg, T, W, 16, False, (8, 0), 16, [64], 6)
    # variational at D=64; truncated two-site DMRG on this near-degenerate
    # ground state (gap 5e-3) is path dependent at the 1e-4 level, so the
    # oracle's own D=64 result is matched to 2e-3
    e64_oracle = -7.215035031868164   # tests/golden/ed_energies.json
    assert E64[-1] >= e_ed - 1e-12 * abs(e_ed)
    assert abs(E64[-1] - e64_oracle) < 2e-3
    log('[sweep] spinless 4x4 D=256 (exact bond dimension at the centre)')
    E = _sweep(mdmrg, T, W, 16, False, (8, 0), 16, [64, 256], 4)
    assert abs(E[-1] - e_ed) <= 1e-12 * abs(e_ed)


def test_sweeps_hubbard_3x3_momentum_reach_exact_energy():
    mdmrg = _gpu()
    T, W = mdmrg.build_lattice(1, 1, 3, 3, 1.0, 4.0)
    e_ed = -9.364758521598883    # tests/golden/ed_energies.json
    log('[sweep] hubbard 3x3 momentum full D')
    E = _sweep(mdmrg, T, W, 9, True, (4, 4), 16, [64, 2000], 4)
    assert abs(E[-1] - e_ed) <= 1e-12 * abs(e_ed)


def test_decimation_matches_oracle():
    mdmrg = _gpu()
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    n, spin, target, l = 9, True, (4, 4), 3
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, 64)
    tens = si.random_mps(bonds, spin, 5, l)
    mps = dmrg.MPS(ch, bonds, tens)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = si.random_vector(ne, 8)
    x /= np.linalg.norm(x)
    for direction in (+1, -1):
        for D in (1, 5, 17, 40, 4096):   # D=1 keeps one state; 4096 keeps every state (no truncation)
            log(f'[decimate] dir {direction} D {D}')
            nb, _, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, D, direction)
            ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
            ctx.prepare_bond(l)
            t2, s2, h2 = ctx.decimate(to_dev(x), D, direction)
            assert abs(trunc - t2) <= 1e-12 and abs(svn - s2) <= 1e-12 and abs(shalf - h2) <= 1e-12
            if not tie:
                assert ctx.get_bond(l + 1) == nb      # kept sector dimensions: exact


@pytest.mark.parametrize('form,bound', [('FP32', 1e-5), ('BF16X3', 5e-4), ('BF16X6', 2e-5)])
def test_split_precision_heff_and_mixed_davidson(form, bound):
    """Split forms: the product error stays within the rounding of the form
    (FP32: |y32 - y| <= 1e-5 max|y|; 3xBF16, about 16 significant bits per
    operand and two GEMM phases: <= 5e-4 max|y|; 6xBF16, about 24 bits per
    operand: <= 2e-5 max|y|), the 3xBF16 product is less exact than the
    FP32 and 6xBF16 ones (it is a different arithmetic), and the
    mixed-precision Davidson (split products, then FP64 refinement) reaches
    the lowest FP64 eigenvalue of the oracle's H_eff to 1e-12 relative."""
    mdmrg = _gpu()
    prec = getattr(mdmrg, form)
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    n, spin, target, l = 9, True, (4, 4), 3
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, 64)
    tens = si.random_mps(bonds, spin, 3, l)
    prob = dmrg.TwoSiteProblem(dmrg.MPS(ch, bonds, tens), l)
    e_ref, _ = prob.lowest(v0=si.random_vector(prob.dim, 1))
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = si.random_vector(ne, 5)
    y_ref = prob.matvec(x)
    yd = torch.zeros(ne, dtype=torch.float64, device='cuda:0')
    ctx.heff_apply(to_dev(x), yd, prec=prec)
    err = np.abs(yd.cpu().numpy() - y_ref).max() / np.abs(y_ref).max()
    log(f'[split] {form} H_eff rel err {err:.2e}')
    assert 0 < err <= bound
    if form == 'BF16X3':
        ctx.heff_apply(to_dev(x), yd, prec=mdmrg.FP32)
        err32 = np.abs(yd.cpu().numpy() - y_ref).max() / np.abs(y_ref).max()
        assert err > 4 * err32
    if form == 'BF16X6':
        ctx.heff_apply(to_dev(x), yd, prec=mdmrg.BF16X3)
        err3 = np.abs(yd.cpu().numpy() - y_ref).max() / np.abs(y_ref).max()
        assert 4 * err < err3
    xd = to_dev(si.random_vector(ne, 2))
    e, r, n64, nsp, conv = ctx.davidson_mixed(xd, tol=1e-9, tol_split=1e-5, prec_split=prec)
    log(f'[split] mixed Davidson: FP64 products {n64}, {form} products {nsp}, E={e:.14f}')
    assert conv and nsp > 0 and r <= 1e-9
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)


def test_davidson_from_zero_start_vector():
    """A zero start vector is replaced by the library's seeded Gaussian
    vector; the solve still reaches the lowest eigenvalue of the oracle's
    H_eff."""
    mdmrg = _gpu()
    build, n, spin, target, D, _ = CASES['hubbard_3x3_momentum_D64']
    T, W = build()
    l = 4
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, D)
    tens = si.random_mps(bonds, spin, 3, l)
    prob = dmrg.TwoSiteProblem(dmrg.MPS(ch, bonds, tens), l)
    e_ref, _ = prob.lowest(v0=si.random_vector(prob.dim, 1))
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = torch.zeros(ne, dtype=torch.float64, device='cuda:0')
    e, r, nmv, conv = ctx.davidson(x, tol=1e-9, max_iter=400)
    assert conv and r <= 1e-9
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    assert abs(float(x.norm()) - 1.0) <= 1e-12


def test_memory_budget_fails_cleanly_and_context_recovers():
    """An allocation beyond the context's device-memory budget fails with
    ENOMEM (the failure is forced from the host with a small budget); with
    the default budget restored the same context prepares the bond and its
    H_eff product matches the oracle."""
    mdmrg = _gpu()
    build, n, spin, target, D, ls = CASES['spinless_4x5_real_D300']
    l = ls[0]
    T, W = build()
    ch = dmrg.Chain(T, W, n, spin, target)
    bonds = si.bond_profile(n, spin, target, D)
    tens = si.random_mps(bonds, spin, 10 + l, l)
    prob = dmrg.TwoSiteProblem(dmrg.MPS(ch, bonds, tens), l)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.set_option(mdmrg.OPT_MEMORY_BUDGET, 1 << 20)
    with pytest.raises(mdmrg.MdmrgError) as e:
        ctx.prepare_bond(l)
    assert e.value.code == mdmrg.ENOMEM and 'budget' in str(e.value)
    ctx.set_option(mdmrg.OPT_MEMORY_BUDGET, 0)
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = si.random_vector(ne, 100 + l)
    yd = torch.zeros(ne, dtype=torch.float64, device='cuda:0')
    ctx.heff_apply(to_dev(x), yd)
    y_ref = prob.matvec(x)
    assert np.abs(yd.cpu().numpy() - y_ref).max() <= 1e-12 * np.abs(y_ref).max()
    ctx.close()


def test_mps_export_round_trip_and_isometry_after_decimation():
    """mdmrg_get_mps returns exactly what mdmrg_set_mps loaded; after a
    decimation towards the right, the exported site l is a left isometry on
    the new bond (sum over left sector and site state of A^T A = 1 per right
    sector)."""
    mdmrg = _gpu()
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    n, spin, target, l = 9, True, (4, 4), 3
    bonds = si.bond_profile(n, spin, target, 64)
    tens = si.random_mps(bonds, spin, 5, l)
    flat = si.flatten_mps(bonds, tens, spin)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*flat)
    assert np.array_equal(ctx.get_mps(), flat[3])
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    ctx.decimate(to_dev(si.random_vector(ne, 9)), 30, +1)
    data = ctx.get_mps()
    nb = [ctx.get_bond(i) for i in range(n + 1)]
    d = 4 if spin else 2
    pos, gram = 0, {}
    for i in range(n):
        for (Ql, ml) in nb[i]:
            for s in range(d):
                q = si.local_qn(s, spin)
                for r, (Qr, mr) in enumerate(nb[i + 1]):
                    if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                        blk = data[pos:pos + ml * mr].reshape(ml, mr)
                        pos += ml * mr
                        if i == l:
                            gram[r] = gram.get(r, np.zeros((mr, mr))) + blk.T @ blk
    assert pos == len(data)
    assert sum(m for _, m in nb[l + 1]) == 30
    for r, g in gram.items():
        assert np.abs(g - np.eye(g.shape[0])).max() <= 1e-12, r
    ctx.close()
