"""Oracle: reduced density matrices and the charge-density-wave order
parameter of an explicit Fock-space state.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For a state psi on the Fock bitstrings ``basis`` (conventions of ``ed``:
bit p set <=> spin-orbital p occupied, the state of bitstring f is
prod_{p ascending, f_p = 1} a+_p |vac>):

* the one-particle reduced density matrix (the orbital occupations and
  natural orbitals of Sec. II.B come from it)
      gamma_pq = <psi| a+_p a_q |psi> = (a_p psi) . (a_q psi);
* the two-particle reduced density matrix (Sec. III.C: 1- and 2-RDMs after
  the sweeps, and the order parameter measured from them)
      Gamma_pqrs = <psi| a+_p a+_q a_r a_s |psi> = (a_q a_p psi) . (a_r a_s psi),
  formed from the pair-annihilated vectors a_r a_s psi in the (N-2)-particle
  space, every operator applied with its Jordan-Wigner sign;
* the energy of Eq. (1) from them, sum_pq T_pq gamma_pq +
  sum_pqrs W_pqrs Gamma_pqrs (the two-body part is written, as in
  ``integrals``, as sum W_pqrs a+_p a+_q a_r a_s);
* the charge-density-wave order parameter C_CDW = <(sum_i s_i n_i)^2> / N^2
  with s_i = +1 on one sublattice and -1 on the other, from the RDMs via
  <n_i n_j> = Gamma_ijji + delta_ij gamma_ii.
"""
import itertools

import numpy as np

from .ed import popcount


def _annihilate(psi, basis, p):
    """(a_p psi) as a dict bitstring -> amplitude."""
    occ = ((basis >> p) & 1).astype(bool)
    f = basis[occ]
    sign = 1 - 2 * (popcount(f & ((np.int64(1) << np.int64(p)) - 1)) & 1)
    return dict(zip((f ^ (np.int64(1) << np.int64(p))).tolist(), (sign * psi[occ]).tolist()))


def _vectors(dicts):
    """Dense rows over the union of the bitstrings of a list of dicts."""
    keys = sorted(set().union(*dicts)) if dicts else []
    index = {k: i for i, k in enumerate(keys)}
    M = np.zeros((len(dicts), len(keys)))
    for r, d in enumerate(dicts):
        for k, v in d.items():
            M[r, index[k]] = v
    return M


def one_rdm(psi, basis, nso):
    """gamma_pq = <psi| a+_p a_q |psi>."""
    Y = _vectors([_annihilate(psi, basis, p) for p in range(nso)])
    return Y @ Y.T


def two_rdm(psi, basis, nso):
    """Gamma_pqrs = <psi| a+_p a+_q a_r a_s |psi> (dense nso^4 array)."""
    pairs = [(r, s) for r in range(nso) for s in range(nso) if r != s]
    dicts = []
    for r, s in pairs:  # a_r a_s psi: first a_s, then a_r
        d1 = _annihilate(psi, basis, s)
        if not d1:
            dicts.append({})
            continue
        keys = np.array(list(d1.keys()), dtype=np.int64)
        vals = np.array(list(d1.values()))
        dicts.append(_annihilate(vals, keys, r))
    Phi = _vectors(dicts)
    O = Phi @ Phi.T  # O[(r s), (r' s')] = (a_r a_s psi) . (a_r' a_s' psi)
    G = np.zeros((nso,) * 4)
    for a, (r, s) in enumerate(pairs):
        for b, (r2, s2) in enumerate(pairs):
            # <a+_p a+_q a_r2 a_s2> with (a_q a_p)^+ = a+_p a+_q: row pair (q, p) = (r, s)
            G[s, r, r2, s2] = O[a, b]
    return G


def energy(T, W, gamma, Gamma):
    """sum T_pq gamma_pq + sum W_pqrs Gamma_pqrs (Eq. (1))."""
    return float(np.sum(T * gamma) + np.sum(W * Gamma))


def density_correlation(gamma, Gamma):
    """<n_i n_j> = Gamma_ijji + delta_ij gamma_ii (spin-orbitals)."""
    nso = gamma.shape[0]
    nn = np.array([[Gamma[i, j, j, i] for j in range(nso)] for i in range(nso)])
    return nn + np.diag(np.diag(gamma))


def cdw_order(gamma, Gamma, signs):
    """C_CDW = <(sum_i s_i n_i)^2> / N^2, N = tr gamma."""
    s = np.asarray(signs, dtype=np.float64)
    n = float(np.trace(gamma))
    return float(s @ density_correlation(gamma, Gamma) @ s) / n ** 2


def checkerboard_signs(Lx, Ly, snake=True):
    """s_i = (-1)^(x+y) of the site at snake position i (``integrals``)."""
    from .integrals import snake_position
    s = np.zeros(Lx * Ly)
    for x, y in itertools.product(range(Lx), range(Ly)):
        s[snake_position(x, y, Lx) if snake else y * Lx + x] = (-1) ** (x + y)
    return s
