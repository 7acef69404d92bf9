"""Oracle: one- and two-mode entropies, mutual information and the
quantities taken from them at the end of the last sweep to set up the next
mode-transformation macro-iteration (Sec. II.B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A mode is a spatial orbital: spin-orbital i of a spinless model, the pair
(2i, 2i+1) of a spin-1/2 model (local dimension 2 or 4; conventions of
``ed``: bit p set <=> spin-orbital p occupied, the state of bitstring f is
prod_{p ascending, f_p = 1} a+_p |vac>).

* ``mode_rdm`` -- the reduced density operator of a list of modes.  Each
  basis state is rewritten with the spin-orbitals of the chosen modes first
  (in the order listed) and the others after them in ascending order; the
  reordering of its occupied creation operators costs the sign
  (-1)^(number of inversions).  Then psi = sum_{c,r} M[c,r] |c> (x) |r>
  over local configurations c of the chosen modes and r of the rest, and
  rho = M M^T.  Bit k of the local index c is the occupation of the k-th
  chosen spin-orbital, so for two modes (i, j) of local dimension d the
  index is c_i + d c_j.
* s_i and s_ij -- von Neumann entropies -Tr rho ln rho of the one- and
  two-mode operators; I_ij = s_i + s_j - s_ij (I_ii = 0);
  I_tot = sum_i s_i; I_dist = sum_{i,j} I_ij |pos(i) - pos(j)|^2 over the
  positions of the modes along the chain.
* the one-particle density matrix gamma_ij = <c+_j c_i> (real states: the
  symmetric gamma of ``rdm.one_rdm``), its eigenpairs (natural occupation
  numbers, descending, and natural modes) and the occupations <n_i>.
* ``fiedler_order`` -- the mode ordering from the Fiedler vector of the
  weighted graph with weights I_ij: the eigenvector of the second-smallest
  eigenvalue of the Laplacian L = diag(sum_j I_ij) - I, its entries sorted
  ascending.
* ``deas_order`` -- the complete-active-space vector of the DEAS warm-up:
  modes in order of decreasing one-mode entropy.
* ``hf_reference`` -- the Fock configuration that fills the most occupied
  spin-orbitals (per spin for spin-1/2 models).
"""
import numpy as np

from .ed import popcount


def mode_orbitals(m, spinful=False):
    """The spin-orbitals of mode m."""
    return [2 * m, 2 * m + 1] if spinful else [m]


def _reorder_sign(basis, chosen):
    """(-1)^inversions of moving the occupied spin-orbitals in `chosen` to the
    front (in that order), the rest keeping their ascending order."""
    basis = np.asarray(basis, dtype=np.int64)
    inv = np.zeros(len(basis), dtype=np.int64)
    chosen_mask = np.int64(0)
    for q in chosen:
        chosen_mask |= np.int64(1) << np.int64(q)
    rest = basis & ~chosen_mask
    for k, q in enumerate(chosen):
        occ = (basis >> np.int64(q)) & 1
        # rest spin-orbitals below q now follow it
        below = popcount(rest & ((np.int64(1) << np.int64(q)) - 1))
        # chosen spin-orbitals listed after q but lying below it
        later = 0
        for q2 in chosen[k + 1:]:
            if q2 < q:
                later = later + ((basis >> np.int64(q2)) & 1)
        inv += occ * (below + later)
    return 1 - 2 * (inv & 1)


def mode_rdm(psi, basis, modes, spinful=False):
    """Reduced density operator of the modes listed (module docstring)."""
    basis = np.asarray(basis, dtype=np.int64)
    chosen = [q for m in modes for q in mode_orbitals(m, spinful)]
    sign = _reorder_sign(basis, chosen)
    c = np.zeros(len(basis), dtype=np.int64)
    for k, q in enumerate(chosen):
        c |= ((basis >> np.int64(q)) & 1) << np.int64(k)
    chosen_mask = np.int64(0)
    for q in chosen:
        chosen_mask |= np.int64(1) << np.int64(q)
    rk, ri = np.unique(basis & ~chosen_mask, return_inverse=True)
    M = np.zeros((1 << len(chosen), len(rk)))
    M[c, ri] = sign * np.asarray(psi, dtype=np.float64)
    return M @ M.T


def vn_entropy(rho):
    """-Tr rho ln rho (eigenvalues below 1e-300 count as zero)."""
    w = np.linalg.eigvalsh(0.5 * (rho + rho.T))
    w = w[w > 1e-300]
    return float(-np.sum(w * np.log(w)))


def one_mode_entropies(psi, basis, n_modes, spinful=False):
    return np.array([vn_entropy(mode_rdm(psi, basis, [i], spinful)) for i in range(n_modes)])


def two_mode_entropies(psi, basis, n_modes, spinful=False):
    """s_ij for i != j (symmetric; the diagonal holds s_i)."""
    S = np.zeros((n_modes, n_modes))
    for i in range(n_modes):
        S[i, i] = vn_entropy(mode_rdm(psi, basis, [i], spinful))
        for j in range(i + 1, n_modes):
            S[i, j] = S[j, i] = vn_entropy(mode_rdm(psi, basis, [i, j], spinful))
    return S


def mutual_information(s, S2):
    """I_ij = s_i + s_j - s_ij, zero on the diagonal."""
    s = np.asarray(s, dtype=np.float64)
    I = s[:, None] + s[None, :] - S2
    np.fill_diagonal(I, 0.0)
    return I


def total_correlation(s):
    return float(np.sum(s))


def correlation_distance(I, order=None):
    """sum_{i,j} I_ij |pos(i) - pos(j)|^2, pos(order[k]) = k (default: the
    modes in index order)."""
    n = I.shape[0]
    pos = np.arange(n) if order is None else np.argsort(np.asarray(order))
    d = pos[:, None] - pos[None, :]
    return float(np.sum(I * d * d))


def natural_orbitals(gamma):
    """(occupation numbers descending, natural modes as columns)."""
    w, V = np.linalg.eigh(0.5 * (gamma + gamma.T))
    return w[::-1], V[:, ::-1]


def occupations(gamma, spinful=False):
    """<n_i> per mode (summed over spin for spin-1/2 models)."""
    d = np.diag(gamma)
    return d[0::2] + d[1::2] if spinful else d.copy()


def laplacian(I):
    return np.diag(I.sum(axis=1)) - I


def fiedler_order(I):
    """Modes sorted by their entries of the Fiedler vector.  The vector's
    sign is chosen so that it correlates non-negatively with the current
    positions (the new order reverses the old one no more than it must);
    ties keep index order.  Raises if the graph is disconnected (the second
    eigenvalue is zero and the vector is not defined)."""
    I = 0.5 * (I + I.T)
    w, V = np.linalg.eigh(laplacian(I))
    if w[1] <= 1e-12 * max(w[-1], 1e-300):
        raise ValueError('the mutual-information graph is disconnected')
    v = V[:, 1]
    if np.dot(v, np.arange(len(v)) - 0.5 * (len(v) - 1)) < 0:
        v = -v
    return np.argsort(v, kind='stable')


def deas_order(s):
    """Modes by decreasing one-mode entropy, ties in index order."""
    return np.argsort(-np.asarray(s, dtype=np.float64), kind='stable')


def hf_reference(gamma, n_elec, spinful=False, n_up=None):
    """Bitstring filling the n_elec most occupied spin-orbitals (spin-1/2:
    the n_up most occupied up and n_elec - n_up most occupied down ones);
    ties go to the lower index."""
    occ = np.diag(gamma)
    f = 0
    if spinful:
        for sigma, k in ((0, n_up), (1, n_elec - n_up)):
            so = np.arange(sigma, len(occ), 2)
            for p in so[np.argsort(-occ[so], kind='stable')[:k]]:
                f |= 1 << int(p)
    else:
        for p in np.argsort(-occ, kind='stable')[:n_elec]:
            f |= 1 << int(p)
    return f
