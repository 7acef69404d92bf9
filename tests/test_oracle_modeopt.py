"""Pins of the oracle's mode rotations of Fock-space states and the
half-Renyi entropy (oracle/modeopt.py; Sec. II.B mode transformation and
two-mode rotations lowering S_1/2).

* Energy invariance: for random integrals and a random orthogonal R, the
  state rotated on Fock space (the exponential of the one-body generator
  log R^T, built term by term) has under the rotated integrals of
  ``integrals.rotate`` the energy the original state has under the
  original ones -- spinless and spin-1/2 (same rotation for both spins).
  The two sides are independent implementations of one transformation.
* The rotation is unitary, R^T undoes R, and a quarter turn of modes i, j
  exchanges their occupations.
* S_1/2: zero for a product state, 2 ln(|cos a| + |sin a|) for the two-mode
  state cos a |10> + sin a |01> across the cut.
* The two-mode micro-iteration finds the angle that undoes a known
  entangling rotation of a product state, and S_1/2 returns to zero.
"""
import numpy as np
import pytest

from oracle import ed, integrals as I, modeopt as M


def _random_orthogonal(n, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize('spinful', [False, True])
def test_rotated_state_has_the_energy_of_the_rotated_integrals(spinful):
    rng = np.random.default_rng(7 + spinful)
    n = 3 if spinful else 6
    nso = 2 * n if spinful else n
    T = rng.standard_normal((n, n))
    T = T + T.T
    if spinful:
        Tso = np.kron(T, np.eye(2))
        W = np.zeros((nso,) * 4)
        for i in range(n):
            W[2 * i, 2 * i + 1, 2 * i + 1, 2 * i] = 4.0
        basis = ed.sector_basis(nso, 3, True, 2)
    else:
        Tso = T
        W = rng.standard_normal((nso,) * 4)
        W = W + W.transpose(3, 2, 1, 0)
        basis = ed.sector_basis(nso, 3)
    psi = rng.standard_normal(len(basis))
    psi /= np.linalg.norm(psi)
    e0 = psi @ ed.SectorHamiltonian(Tso, W, basis).matvec(psi)
    R = _random_orthogonal(n, rng)
    T2, W2 = I.rotate(Tso, W, R, spinful=spinful)
    psi2 = M.rotate_state(psi, basis, R, spinful=spinful)
    e1 = psi2 @ ed.SectorHamiltonian(T2, W2, basis).matvec(psi2)
    assert abs(np.linalg.norm(psi2) - 1.0) < 1e-12
    assert abs(e1 - e0) < 1e-12 * max(1.0, abs(e0))
    # the wrong direction (R instead of R^T in the generator) fails
    psi3 = M.rotate_state(psi, basis, R.T, spinful=spinful)
    assert abs(psi3 @ ed.SectorHamiltonian(T2, W2, basis).matvec(psi3) - e0) > 1e-6


def test_rotation_inverse_and_quarter_turn():
    rng = np.random.default_rng(3)
    n = 5
    basis = ed.sector_basis(n, 2)
    psi = rng.standard_normal(len(basis))
    psi /= np.linalg.norm(psi)
    R = _random_orthogonal(n, rng)
    back = M.rotate_state(M.rotate_state(psi, basis, R), basis, R.T)
    assert np.allclose(back, psi, atol=1e-12)
    # a quarter turn of modes 1 and 3 exchanges their occupations
    occ = lambda v, p: float(np.sum(v ** 2 * ((basis >> p) & 1)))
    q = M.rotate_state(psi, basis, M.givens(n, 1, 3, np.pi / 2))
    assert abs(occ(q, 1) - occ(psi, 3)) < 1e-12 and abs(occ(q, 3) - occ(psi, 1)) < 1e-12
    assert abs(occ(q, 0) - occ(psi, 0)) < 1e-12


def test_half_renyi_closed_forms():
    n = 4
    basis = list(ed.sector_basis(n, 1))
    psi = np.zeros(len(basis))
    psi[basis.index(0b0001)] = 1.0
    assert abs(M.half_renyi(psi, np.array(basis), 2)) < 1e-14
    for a in (0.1, 0.4, np.pi / 4, 1.2):
        psi = np.zeros(len(basis))
        psi[basis.index(0b0010)] = np.cos(a)   # mode 1 (left of the cut)
        psi[basis.index(0b0100)] = np.sin(a)   # mode 2 (right of the cut)
        want = 2.0 * np.log(abs(np.cos(a)) + abs(np.sin(a)))
        assert abs(M.half_renyi(psi, np.array(basis), 2) - want) < 1e-13


@pytest.mark.parametrize('theta0', [0.37, -0.9, 1.3])
def test_micro_iteration_undoes_a_known_rotation(theta0):
    n = 4
    basis = ed.sector_basis(n, 2)
    psi = np.zeros(len(basis))
    psi[list(basis).index(0b0101)] = 1.0       # modes 0 and 2 occupied: a product across the cut
    ent = M.rotate_state(psi, basis, M.givens(n, 1, 2, theta0))
    assert M.half_renyi(ent, basis, 2) > 0.05
    th, s = M.best_two_mode_angle(ent, basis, n, 1, 2, 2, np.linspace(-np.pi / 2, np.pi / 2, 37))
    # near its minimum S_1/2 = 2 ln(|cos d| + |sin d|) ~ 2|d| (a cusp), so the
    # minimiser's angle error d of order 1e-8 leaves S_1/2 of that order
    assert s < 1e-6
    # the minimiser is -theta0 modulo the quarter turns that keep the product form
    d = (th + theta0) / (np.pi / 2)
    assert abs(d - round(d)) < 1e-5
