"""Pins of the CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: closed
forms (free fermions, the Hubbard dimer), brute force on tiny inputs, basis
invariance of the spectrum (Sec. III.A: a unitary mode transformation with no
truncation leaves the spectrum intact), and isometry/variational properties
of the DMRG projection.
"""
import json
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import dmrg, ed
from oracle import integrals as I

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


# ---------------------------------------------------------------- integrals
@pytest.mark.parametrize('builder,args,spinful', [
    (I.spinless_real_space, (3, 3, 1.0, 1.0), False),
    (I.spinless_momentum, (3, 3, 1.0, 1.0), False),
    (I.hubbard_real_space, (3, 3, 1.0, 4.0), True),
    (I.hubbard_momentum, (3, 3, 1.0, 4.0), True),
])
def test_builders_hermitian(builder, args, spinful):
    T, W = builder(*args)
    assert I.is_hermitian(T, W)


def test_momentum_conservation_and_free_spectrum():
    Lx, Ly = 4, 4
    T, W = I.spinless_momentum(Lx, Ly, 1.0, 0.7)
    order, kint, eps = I.momentum_modes(Lx, Ly, 1.0)
    # T is diagonal with the band energies in ascending order
    assert np.allclose(T, np.diag(np.diag(T)))
    assert np.all(np.diff(np.diag(T)) >= -1e-12)
    # real-space T has the same single-particle spectrum
    Tr, _ = I.spinless_real_space(Lx, Ly, 1.0, 0.7)
    assert np.allclose(np.sort(np.linalg.eigvalsh(Tr)), np.sort(np.diag(T)), atol=1e-12)
    nz = np.argwhere(np.abs(W) > 1e-14)
    for (a, b, c, d) in nz:
        ka, kb, kc, kd = (kint[order[x]] for x in (a, b, c, d))
        assert np.all((ka + kb - kc - kd) % [Lx, Ly] == 0)


# ---------------------------------------------------------------------- ED
@pytest.mark.parametrize('N', [1, 2, 3, 4])
def test_pair_space_matches_brute_force(N):
    rng = np.random.default_rng(7 + N)
    nso = 6
    T = rng.standard_normal((nso, nso))
    T = T + T.T
    W = rng.standard_normal((nso,) * 4)
    W = W + W.transpose(3, 2, 1, 0)
    basis = ed.sector_basis(nso, N)
    x = rng.standard_normal(len(basis))
    y1 = ed.SectorHamiltonian(T, W, basis).matvec(x)
    y2 = ed.apply_terms_literal(T, W, basis, x)
    assert np.abs(y1 - y2).max() <= 1e-12 * max(1.0, np.abs(y2).max())


def test_free_fermion_closed_form_spinless():
    # V = 0: ground energy = sum of the N lowest single-particle energies
    T, W = I.spinless_real_space(4, 4, 1.0, 0.0)
    e = ed.ground_energy(T, W, 8)[0]
    assert abs(e - (-12.0)) < 1e-11
    assert abs(e - np.sort(np.linalg.eigvalsh(T))[:8].sum()) < 1e-11


def test_free_fermion_closed_form_hubbard():
    T, W = I.hubbard_real_space(3, 3, 1.0, 0.0)
    e = ed.ground_energy(T, W, 6, spinful=True, n_up=3)[0]
    eps = np.sort(np.linalg.eigvalsh(T[0::2, 0::2]))
    assert abs(e - 2 * eps[:3].sum()) < 1e-11


def test_hubbard_dimer_closed_form():
    # two sites, one bond, two electrons: E0 = U/2 - sqrt(U^2/4 + 4 t^2)
    t, U = 1.0, 3.7
    T = np.zeros((4, 4))
    for s in (0, 1):
        T[s, 2 + s] = T[2 + s, s] = -t
    W = np.zeros((4,) * 4)
    for i in range(2):
        W[2 * i, 2 * i + 1, 2 * i + 1, 2 * i] = U
    e = ed.ground_energy(T, W, 2, spinful=True, n_up=1)[0]
    assert abs(e - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-13


def test_spinless_two_particle_interaction():
    # 2 sites, 2 particles: the only state is |11>, energy V
    T = np.array([[0.0, -1.0], [-1.0, 0.0]])
    W = np.zeros((2,) * 4)
    W[0, 1, 1, 0] = 2.5
    assert abs(ed.ground_energy(T, W, 2)[0] - 2.5) < 1e-14


def test_momentum_equals_real_space():
    Tr, Wr = I.spinless_real_space(4, 4, 1.0, 1.0)
    Tk, Wk = I.spinless_momentum(4, 4, 1.0, 1.0)
    er = ed.ground_energy(Tr, Wr, 8)[0]
    ek = ed.ground_energy(Tk, Wk, 8)[0]
    assert abs(er - ek) < 1e-11
    Tr, Wr = I.hubbard_real_space(3, 3, 1.0, 4.0)
    Tk, Wk = I.hubbard_momentum(3, 3, 1.0, 4.0)
    er = ed.ground_energy(Tr, Wr, 8, True, 4)[0]
    ek = ed.ground_energy(Tk, Wk, 8, True, 4)[0]
    assert abs(er - ek) < 1e-11


def test_rotation_invariance():
    T, W = I.spinless_real_space(3, 3, 1.0, 1.3)
    R = si.random_orthogonal(9, 0)
    T2, W2 = I.rotate(T, W, R)
    assert I.is_hermitian(T2, W2)
    e1 = ed.ground_energy(T, W, 4, k=3)
    e2 = ed.ground_energy(T2, W2, 4, k=3)
    assert np.abs(e1 - e2).max() < 1e-11


def test_golden_ed_values():
    """Regression against values written by tests/golden/make_golden.py."""
    with open(os.path.join(GOLDEN, 'ed_energies.json')) as f:
        gold = json.load(f)
    T, W = I.spinless_real_space(4, 4, 1.0, 1.0)
    assert abs(ed.ground_energy(T, W, 8)[0] - gold['spinless_4x4_t1_V1_N8']) < 1e-10
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    assert abs(ed.ground_energy(T, W, 8, True, 4)[0] - gold['hubbard_3x3_t1_U4_4up4dn']) < 1e-10


# -------------------------------------------------------------------- DMRG
def _small_chain(spinful):
    if spinful:
        T, W = I.hubbard_momentum(3, 2, 1.0, 4.0)
        return dmrg.Chain(T, W, 6, True, (2, 2)), (T, W, 4, True, 2)
    T, W = I.spinless_real_space(3, 3, 1.0, 1.0)
    return dmrg.Chain(T, W, 9, False, (4, 0)), (T, W, 4, False, None)


@pytest.mark.parametrize('spinful', [False, True])
def test_dmrg_full_D_equals_ed(spinful):
    ch, (T, W, N, sf, nup) = _small_chain(spinful)
    e_ed = ed.ground_energy(T, W, N, sf, nup)[0]
    bonds = si.bond_profile(ch.n, spinful, ch.target, 8)
    mps = dmrg.MPS(ch, bonds, si.random_mps(bonds, spinful, 1, 0))
    E = dmrg.sweep_energy(ch, mps, [16, 4096], 3)
    assert abs(E[-1] - e_ed) <= 1e-11 * abs(e_ed)


@pytest.mark.parametrize('spinful', [False, True])
def test_projection_is_isometric_and_variational(spinful):
    ch, (T, W, N, sf, nup) = _small_chain(spinful)
    e_ed = ed.ground_energy(T, W, N, sf, nup)[0]
    bonds = si.bond_profile(ch.n, spinful, ch.target, 6)
    l = ch.n // 2 - 1
    mps = dmrg.MPS(ch, bonds, si.random_mps(bonds, spinful, 3, l))
    prob = dmrg.TwoSiteProblem(mps, l)
    x = si.random_vector(prob.dim, 4)
    y = si.random_vector(prob.dim, 5)
    # P^T P = 1
    assert np.abs(prob.from_full(prob.to_full(x)) - x).max() < 1e-12
    # Hermiticity of P^T H P
    hx, hy = prob.matvec(x), prob.matvec(y)
    assert abs(x @ hy - y @ hx) < 1e-12 * np.linalg.norm(hx) * np.linalg.norm(y)
    # variational: lowest eigenvalue of the projection >= exact
    e, v = prob.lowest(v0=x)
    assert e >= e_ed - 1e-12


def test_decimation_keeps_exact_state_and_reports_truncation():
    ch, _ = _small_chain(False)
    bonds = si.bond_profile(ch.n, False, ch.target, 8)
    l = 3
    mps = dmrg.MPS(ch, bonds, si.random_mps(bonds, False, 3, l))
    prob = dmrg.TwoSiteProblem(mps, l)
    x = si.random_vector(prob.dim, 9)
    x /= np.linalg.norm(x)
    full = prob.to_full(x)
    # keep everything: the state is reproduced after StVec
    nb, t, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, 10 ** 6, +1)
    assert trunc < 1e-14
    mps2 = dmrg.MPS(ch, mps.bonds, mps.A)
    mps2.bonds[l + 1] = nb
    mps2.A[l] = t
    prob2 = dmrg.TwoSiteProblem(mps2, l + 1)
    x2 = dmrg.start_vector(prob, x, prob2)
    assert np.abs(prob2.to_full(x2) - full).max() < 1e-12
    # truncating leaves a positive error below 1 and S_1/2 >= S_vN (the
    # exact values on known spectra are pinned in test_oracle_decimation.py)
    nb, t, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, 3, +1)
    assert 0.0 < trunc < 1.0
    assert shalf >= svn - 1e-12
