"""Pins of the oracle's one- and two-mode entropies, mutual information and
the ordering, active-space and reference choices taken from them
(oracle/mutual.py; Sec. II.B, the quantities computed after the last sweep).

* Every element of a one- or two-mode reduced density operator equals its
  definition <psi| (|b><a| (x) 1) |psi>, with |b><a| written as creation
  operators, the projector on the empty modes and annihilation operators,
  each applied one at a time with its Jordan-Wigner sign (brute force, no
  reordering sign) -- spinless and spin-1/2 random states, modes listed out
  of index order.
* Number conservation makes a one-mode operator diagonal: s_i is the
  Shannon entropy of the local occupation probabilities, summed directly
  from the amplitudes.
* Free fermions (Peschel): the reduced state of a Slater determinant is
  Gaussian, so s_ij = sum_k h(lambda_k) over the eigenvalues of gamma
  restricted to the spin-orbitals of i and j, h(x) = -x ln x -
  (1-x) ln(1-x).
* Closed forms: a product Fock state has no entropy; a particle shared by
  two modes (spinless, a JW string of occupied modes between them) and a
  singlet pair on two sites give I_ij = 2 ln 2 and nothing elsewhere.
* Invariants on the 4x4 spinless and 3x3 momentum Hubbard ground states:
  Tr_j rho_ij = rho_i, rho_ij positive with unit trace, and the Araki-Lieb
  bounds 0 <= I_ij <= 2 min(s_i, s_j).
* The natural modes of a Slater determinant turn it into one configuration:
  occupations 0 and 1, zero one-mode entropies and total correlation, and
  the HF reference picks that configuration.
* The Fiedler ordering of a weighted path graph whose modes are shuffled
  recovers the path, up to reversal, and attains the brute-force minimum of
  I_dist over all orderings; a mistake planted in the oracle's Laplacian
  (the wrong sign of the off-diagonal part) does not.
* DEAS order and HF reference on hand-made cases, I_tot and I_dist on a
  hand-made matrix.
* Dropping the reordering sign (a mistake planted in the oracle) fails the
  definition.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import ed, integrals as I, modeopt, mutual, rdm

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'ed_energies.json')))
LN2 = np.log(2.0)


# ---- brute-force operator application on {bitstring: amplitude} -----------
def _sign(f, p):
    return -1.0 if bin(f & ((1 << p) - 1)).count('1') & 1 else 1.0


def _cre(state, p):
    out = {}
    for f, a in state.items():
        if not (f >> p) & 1:
            g = f | (1 << p)
            out[g] = out.get(g, 0.0) + _sign(f, p) * a
    return out


def _ann(state, p):
    out = {}
    for f, a in state.items():
        if (f >> p) & 1:
            g = f ^ (1 << p)
            out[g] = out.get(g, 0.0) + _sign(f, p) * a
    return out


def _rdm_by_definition(psi, basis, modes, spinful):
    """rho[a, b] = <psi| C_b P C_a^+ |psi>, C_x = prod_{k ascending, x_k=1}
    a+_{q_k}, P = prod_k (1 - n_{q_k}) on the chosen spin-orbitals q."""
    q = [p for m in modes for p in mutual.mode_orbitals(m, spinful)]
    K = len(q)
    ket = {int(f): float(a) for f, a in zip(basis, psi)}
    rho = np.zeros((1 << K, 1 << K))
    for a in range(1 << K):
        for b in range(1 << K):
            s = dict(ket)
            for k in range(K):  # C_a^+ = ... a_{q_k2} a_{q_k1}: annihilate k ascending
                if (a >> k) & 1:
                    s = _ann(s, q[k])
            s = {f: v for f, v in s.items() if all(not (f >> p) & 1 for p in q)}  # P
            for k in reversed(range(K)):  # C_b: create k descending (k=0 leftmost)
                if (b >> k) & 1:
                    s = _cre(s, q[k])
            rho[a, b] = sum(ket.get(f, 0.0) * v for f, v in s.items())
    return rho


def _h(x):
    x = np.clip(x, 0.0, 1.0)
    out = np.zeros_like(x)
    m = (x > 0) & (x < 1)
    out[m] = -x[m] * np.log(x[m]) - (1 - x[m]) * np.log(1 - x[m])
    return out


def _ground(T, W, n, spinful=False, n_up=None):
    basis = ed.sector_basis(T.shape[0], n, spinful, n_up)
    w, v = ed.SectorHamiltonian(T, W, basis).ground_state(k=1)
    psi = np.asarray(v).reshape(len(basis), -1)[:, 0]
    return float(np.atleast_1d(w)[0]), psi / np.linalg.norm(psi), basis


def _random_state(nso, n, seed, spinful=False, n_up=None):
    basis = ed.sector_basis(nso, n, spinful, n_up)
    psi = np.random.default_rng(seed).standard_normal(len(basis))
    return psi / np.linalg.norm(psi), basis


@pytest.mark.parametrize('spinful,nso,n,n_up,modes', [
    (False, 7, 3, None, [5]), (False, 7, 3, None, [5, 1]), (False, 7, 4, None, [2, 6]),
    (True, 8, 4, 2, [2]), (True, 8, 4, 2, [3, 0]), (True, 8, 3, 2, [1, 2])])
def test_mode_rdm_equals_its_definition(spinful, nso, n, n_up, modes):
    psi, basis = _random_state(nso, n, 11 + nso + n, spinful, n_up)
    rho = mutual.mode_rdm(psi, basis, modes, spinful)
    ref = _rdm_by_definition(psi, basis, modes, spinful)
    assert np.allclose(rho, ref, atol=1e-14), np.abs(rho - ref).max()
    offdiag = np.count_nonzero(np.abs(ref - np.diag(np.diag(ref))) > 1e-6)
    # one mode: diagonal (number conservation); two modes: coherences that
    # carry the Jordan-Wigner signs
    assert offdiag == 0 if len(modes) == 1 else offdiag > 0


def test_one_mode_entropy_is_the_occupation_entropy():
    psi, basis = _random_state(8, 4, 5, True, 2)
    s = mutual.one_mode_entropies(psi, basis, 4, True)
    for i in range(4):
        c = ((basis >> (2 * i)) & 1) + 2 * ((basis >> (2 * i + 1)) & 1)
        p = np.array([np.sum(psi[c == k] ** 2) for k in range(4)])
        p = p[p > 0]
        assert abs(s[i] - float(-np.sum(p * np.log(p)))) < 1e-13


def _free_chain(n_sites, seed):
    rng = np.random.default_rng(seed)
    T = np.zeros((n_sites, n_sites))
    for i in range(n_sites - 1):
        T[i, i + 1] = T[i + 1, i] = -1.0 - 0.3 * rng.random()
    T += np.diag(0.2 * rng.standard_normal(n_sites))
    return T


def test_free_fermion_entropies_follow_peschel():
    # spinless: 6 modes, 3 particles
    T = _free_chain(6, 1)
    e, psi, basis = _ground(T, np.zeros((6,) * 4), 3)
    g = rdm.one_rdm(psi, basis, 6)
    S2 = mutual.two_mode_entropies(psi, basis, 6)
    for i in range(6):
        assert abs(S2[i, i] - _h(np.array([g[i, i]]))[0]) < 1e-12
        for j in range(i + 1, 6):
            lam = np.linalg.eigvalsh(g[np.ix_([i, j], [i, j])])
            assert abs(S2[i, j] - _h(lam).sum()) < 1e-12, (i, j)
    # spin-1/2: 4 sites, 2 up + 1 down, the same hopping for both spins
    T1 = _free_chain(4, 2)
    T2 = np.kron(T1, np.eye(2))
    e, psi, basis = _ground(T2, np.zeros((8,) * 4), 3, True, 2)
    eps = np.linalg.eigvalsh(T1)
    assert abs(e - (eps[:2].sum() + eps[0])) < 1e-12
    g = rdm.one_rdm(psi, basis, 8)
    S2 = mutual.two_mode_entropies(psi, basis, 4, True)
    for i in range(4):
        for j in range(i, 4):
            so = sorted(set(mutual.mode_orbitals(i, True) + mutual.mode_orbitals(j, True)))
            lam = np.linalg.eigvalsh(g[np.ix_(so, so)])
            assert abs(S2[i, j] - _h(lam).sum()) < 1e-12, (i, j)
    assert S2.max() > 0.5


def test_closed_forms_product_shared_particle_and_singlet():
    # product Fock state: nothing
    basis = np.array([0b1011001], dtype=np.int64)
    s = mutual.one_mode_entropies(np.ones(1), basis, 7)
    S2 = mutual.two_mode_entropies(np.ones(1), basis, 7)
    assert np.abs(s).max() < 1e-15 and np.abs(mutual.mutual_information(s, S2)).max() < 1e-15
    # one particle shared by modes 1 and 5 with modes 2 and 3 occupied
    # between them (a Jordan-Wigner string of length 2), mode 6 occupied
    f1, f2 = (1 << 1) | 0b1100 | (1 << 6), (1 << 5) | 0b1100 | (1 << 6)
    basis = np.array(sorted([f1, f2]), dtype=np.int64)
    psi = np.array([1.0, -1.0]) / np.sqrt(2)
    s = mutual.one_mode_entropies(psi, basis, 7)
    Imat = mutual.mutual_information(s, mutual.two_mode_entropies(psi, basis, 7))
    assert np.allclose(s, [0, LN2, 0, 0, 0, LN2, 0], atol=1e-14)
    ref = np.zeros((7, 7))
    ref[1, 5] = ref[5, 1] = 2 * LN2
    assert np.allclose(Imat, ref, atol=1e-14)
    # spin singlet of one electron on site 0 and one on site 2 (3 sites),
    # (a+_{0 up} a+_{2 dn} - a+_{0 dn} a+_{2 up}) |vac>
    fa, fb = (1 << 0) | (1 << 5), (1 << 1) | (1 << 4)
    basis = np.array(sorted([fa, fb]), dtype=np.int64)
    amp = {fa: 1.0, fb: -1.0}
    psi = np.array([amp[int(f)] for f in basis]) / np.sqrt(2)
    s = mutual.one_mode_entropies(psi, basis, 3, True)
    S2 = mutual.two_mode_entropies(psi, basis, 3, True)
    assert np.allclose(s, [LN2, 0, LN2], atol=1e-14)
    assert abs(S2[0, 2]) < 1e-14
    assert abs(mutual.mutual_information(s, S2)[0, 2] - 2 * LN2) < 1e-14


@pytest.fixture(scope='module')
def spinless44():
    T, W = I.spinless_real_space(4, 4, 1.0, 1.0)
    e, psi, basis = _ground(T, W, 8)
    assert abs(e - GOLDEN['spinless_4x4_t1_V1_N8']) < 1e-10
    return psi, basis


def _check_invariants(psi, basis, n, spinful, pairs):
    d = 4 if spinful else 2
    s = mutual.one_mode_entropies(psi, basis, n, spinful)
    for i, j in pairs:
        rho = mutual.mode_rdm(psi, basis, [i, j], spinful)
        assert abs(np.trace(rho) - 1) < 1e-12 and np.linalg.eigvalsh(rho).min() > -1e-13
        r4 = rho.reshape(d, d, d, d)  # [c_j, c_i, c_j', c_i']
        assert np.allclose(np.einsum('jajb->ab', r4), mutual.mode_rdm(psi, basis, [i], spinful), atol=1e-13)
        assert np.allclose(np.einsum('ajbj->ab', r4), mutual.mode_rdm(psi, basis, [j], spinful), atol=1e-13)
        sij = mutual.vn_entropy(rho)
        Iij = s[i] + s[j] - sij
        assert -1e-12 <= Iij <= 2 * min(s[i], s[j]) + 1e-12
    return s


def test_invariants_spinless_4x4(spinless44):
    psi, basis = spinless44
    s = _check_invariants(psi, basis, 16, False, [(0, 1), (0, 15), (3, 12), (7, 5)])
    # half filling of a translation-invariant torus: n_i = 1/2, s_i = ln 2
    assert np.allclose(s, LN2, atol=1e-10)


def test_invariants_hubbard_3x3_momentum():
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    e, psi, basis = _ground(T, W, 8, spinful=True, n_up=4)
    assert abs(e - GOLDEN['hubbard_3x3_t1_U4_4up4dn']) < 1e-10
    s = _check_invariants(psi, basis, 9, True, [(0, 1), (2, 7), (8, 4)])
    assert s.max() > 0.1


def test_natural_modes_disentangle_a_slater_determinant():
    T = _free_chain(6, 3)
    e, psi, basis = _ground(T, np.zeros((6,) * 4), 3)
    g = rdm.one_rdm(psi, basis, 6)
    lam, V = mutual.natural_orbitals(g)
    assert np.allclose(lam, [1, 1, 1, 0, 0, 0], atol=1e-12)
    s0 = mutual.one_mode_entropies(psi, basis, 6)
    assert mutual.total_correlation(s0) > 1.0
    psi2 = modeopt.rotate_state(psi, basis, V)
    s = mutual.one_mode_entropies(psi2, basis, 6)
    assert mutual.total_correlation(s) < 1e-10
    g2 = rdm.one_rdm(psi2, basis, 6)
    assert np.allclose(mutual.occupations(g2), [1, 1, 1, 0, 0, 0], atol=1e-12)
    f = mutual.hf_reference(g2, 3)
    assert f == 0b000111
    assert abs(abs(psi2[np.searchsorted(basis, f)]) - 1) < 1e-12


def _path(perm, w):
    n = len(perm)
    Imat = np.zeros((n, n))
    for k in range(n - 1):
        Imat[perm[k], perm[k + 1]] = Imat[perm[k + 1], perm[k]] = w[k]
    return Imat


def test_fiedler_recovers_a_shuffled_path():
    rng = np.random.default_rng(7)
    for trial in range(5):
        n = 7
        perm = rng.permutation(n)
        Imat = _path(perm, 0.2 + rng.random(n - 1))
        order = mutual.fiedler_order(Imat)
        assert list(order) in (list(perm), list(perm[::-1])), (trial, order, perm)
        best = min(mutual.correlation_distance(Imat, p) for p in itertools.permutations(range(n)))
        assert abs(mutual.correlation_distance(Imat, order) - best) < 1e-12
        assert best == pytest.approx(2 * Imat.sum() / 2)  # every edge at distance 1, both (i,j) and (j,i)


def test_planted_laplacian_sign_mistake_breaks_the_ordering(monkeypatch):
    monkeypatch.setattr(mutual, 'laplacian', lambda Imat: np.diag(Imat.sum(axis=1)) + Imat)
    rng = np.random.default_rng(7)
    misses = 0
    for trial in range(5):
        perm = rng.permutation(7)
        Imat = _path(perm, 0.2 + rng.random(6))
        try:
            order = mutual.fiedler_order(Imat)
        except ValueError:
            misses += 1
            continue
        misses += list(order) not in (list(perm), list(perm[::-1]))
    assert misses >= 3


def test_fiedler_refuses_a_disconnected_graph():
    Imat = np.zeros((4, 4))
    Imat[0, 1] = Imat[1, 0] = Imat[2, 3] = Imat[3, 2] = 1.0
    with pytest.raises(ValueError):
        mutual.fiedler_order(Imat)


def test_deas_order_hf_reference_and_sums():
    s = np.array([0.1, 0.7, 0.0, 0.7, 0.3])
    assert list(mutual.deas_order(s)) == [1, 3, 4, 0, 2]
    assert mutual.total_correlation(s) == pytest.approx(1.8)
    Imat = np.zeros((4, 4))
    Imat[0, 3] = Imat[3, 0] = 0.5
    Imat[1, 2] = Imat[2, 1] = 0.25
    # pairs at distance 3 and 1, both orientations: 2 * (0.5 * 9 + 0.25 * 1)
    assert mutual.correlation_distance(Imat) == pytest.approx(9.5)
    # the order (0, 3, 1, 2) puts both pairs next to each other
    assert mutual.correlation_distance(Imat, [0, 3, 1, 2]) == pytest.approx(1.5)
    # spin-1/2 reference: 2 up in the most occupied up spin-orbitals, 1 down
    g = np.diag([0.9, 0.2, 0.1, 0.8, 0.6, 0.3, 0.4, 0.05])
    f = mutual.hf_reference(g, 3, True, 2)
    assert f == (1 << 0) | (1 << 4) | (1 << 3)
    assert np.allclose(mutual.occupations(g, True), [1.1, 0.9, 0.9, 0.45])


def test_planted_reordering_sign_mistake_is_caught(monkeypatch):
    """Dropping the reordering sign (the Jordan-Wigner string between the
    chosen modes) changes two-mode coherences and fails the definition."""
    psi, basis = _random_state(8, 4, 31, True, 2)
    ref = _rdm_by_definition(psi, basis, [3, 0], True)
    monkeypatch.setattr(mutual, '_reorder_sign', lambda b, chosen: np.ones(len(b), dtype=np.int64))
    assert np.abs(mutual.mode_rdm(psi, basis, [3, 0], True) - ref).max() > 1e-3
