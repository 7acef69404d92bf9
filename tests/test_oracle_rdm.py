"""Pins of the oracle's reduced density matrices and C_CDW (oracle/rdm.py;
Sec. II.B one-particle RDM, Sec. III.C RDMs and the CDW order parameter).

* The energy of Eq. (1) from the RDMs, sum T gamma + sum W Gamma, equals the
  exact eigenvalue of the state they come from: 4x4 spinless torus (t=1,
  V=1, 8 particles) and 3x3 Hubbard torus in the momentum basis (dense
  two-body integrals), both against the golden ED energies.
* gamma is Hermitian with trace N and eigenvalues in [0, 1]; the partial
  trace sum_q Gamma_pqqs = (N-1) gamma_ps.
* Free fermions (open chain, non-degenerate ground state): gamma is a
  projector of rank N and Gamma obeys Wick's theorem,
  Gamma_pqrs = gamma_ps gamma_qr - gamma_pr gamma_qs.
* C_CDW from the RDMs equals the expectation of (sum_i s_i n_i)^2 / N^2
  evaluated directly on the Fock amplitudes.
* A mistake planted in the oracle (annihilation without its Jordan-Wigner
  sign) breaks the energy identity.
"""
import json
import os

import numpy as np
import pytest

from oracle import ed, integrals as I, rdm

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'ed_energies.json')))


def _ground(T, W, n, spinful=False, n_up=None):
    basis = ed.sector_basis(T.shape[0], n, spinful, n_up)
    w, v = ed.SectorHamiltonian(T, W, basis).ground_state(k=1)
    psi = np.asarray(v).reshape(len(basis), -1)[:, 0]
    return float(np.atleast_1d(w)[0]), psi / np.linalg.norm(psi), basis


@pytest.fixture(scope='module')
def spinless44():
    T, W = I.spinless_real_space(4, 4, 1.0, 1.0)
    e, psi, basis = _ground(T, W, 8)
    g = rdm.one_rdm(psi, basis, 16)
    G = rdm.two_rdm(psi, basis, 16)
    return T, W, e, psi, basis, g, G


def test_energy_from_rdms_spinless_4x4(spinless44):
    T, W, e, psi, basis, g, G = spinless44
    assert abs(e - GOLDEN['spinless_4x4_t1_V1_N8']) < 1e-10
    assert abs(rdm.energy(T, W, g, G) - e) <= 1e-12 * abs(e)


def test_energy_from_rdms_hubbard_3x3_momentum():
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    e, psi, basis = _ground(T, W, 8, spinful=True, n_up=4)
    assert abs(e - GOLDEN['hubbard_3x3_t1_U4_4up4dn']) < 1e-10
    g = rdm.one_rdm(psi, basis, 18)
    G = rdm.two_rdm(psi, basis, 18)
    assert abs(rdm.energy(T, W, g, G) - e) <= 1e-12 * abs(e)
    # spin structure: no up-down coherence in gamma, 4 particles per spin
    assert np.abs(g[0::2, 1::2]).max() < 1e-12
    assert abs(np.trace(g[0::2, 0::2]) - 4) < 1e-12 and abs(np.trace(g[1::2, 1::2]) - 4) < 1e-12


def test_rdm_traces_and_bounds(spinless44):
    T, W, e, psi, basis, g, G = spinless44
    n = 8
    assert np.allclose(g, g.T, atol=1e-14)
    assert abs(np.trace(g) - n) < 1e-12
    w = np.linalg.eigvalsh(g)
    assert w.min() > -1e-12 and w.max() < 1 + 1e-12
    partial = np.einsum('pqqs->ps', G)
    assert np.allclose(partial, (n - 1) * g, atol=1e-12)
    # antisymmetry of Gamma in its creation and in its annihilation pair
    assert np.allclose(G, -G.transpose(1, 0, 2, 3), atol=1e-14)
    assert np.allclose(G, -G.transpose(0, 1, 3, 2), atol=1e-14)


def test_free_fermions_projector_and_wick():
    n_sites, n = 6, 3
    T = np.zeros((n_sites, n_sites))
    for i in range(n_sites - 1):
        T[i, i + 1] = T[i + 1, i] = -1.0
    W = np.zeros((n_sites,) * 4)
    e, psi, basis = _ground(T, W, n)
    g = rdm.one_rdm(psi, basis, n_sites)
    G = rdm.two_rdm(psi, basis, n_sites)
    # the ground energy is the sum of the n lowest single-particle levels
    eps = np.linalg.eigvalsh(T)
    assert abs(e - eps[:n].sum()) < 1e-12
    assert np.allclose(g @ g, g, atol=1e-12)
    assert np.allclose(np.linalg.eigvalsh(g), [0.0] * (n_sites - n) + [1.0] * n, atol=1e-12)
    wick = np.einsum('ps,qr->pqrs', g, g) - np.einsum('pr,qs->pqrs', g, g)
    assert np.allclose(G, wick, atol=1e-12)


def test_cdw_order_from_rdms_equals_direct(spinless44):
    T, W, e, psi, basis, g, G = spinless44
    s = rdm.checkerboard_signs(4, 4)
    assert sorted(set(s)) == [-1.0, 1.0] and s.sum() == 0
    # direct: (sum_i s_i n_i) is diagonal on the bitstrings
    m = np.array([sum(s[i] for i in range(16) if (f >> i) & 1) for f in basis])
    direct = float(np.sum(psi ** 2 * m ** 2)) / 8 ** 2
    assert abs(rdm.cdw_order(g, G, s) - direct) < 1e-13
    assert 0.0 <= direct <= 1.0


def test_planted_sign_mistake_breaks_the_energy_identity(spinless44, monkeypatch):
    T, W, e, psi, basis, g, G = spinless44

    def no_sign(psi_, basis_, p):
        occ = ((basis_ >> p) & 1).astype(bool)
        f = basis_[occ]
        return dict(zip((f ^ (np.int64(1) << np.int64(p))).tolist(), psi_[occ].tolist()))
    monkeypatch.setattr(rdm, '_annihilate', no_sign)
    g2 = rdm.one_rdm(psi, basis, 16)
    G2 = rdm.two_rdm(psi, basis, 16)
    assert abs(rdm.energy(T, W, g2, G2) - e) > 1e-3
