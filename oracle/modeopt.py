"""Oracle: mode rotations of an explicit Fock-space state and the half-Renyi
entropy they are chosen to lower (the mode optimisation of Sec. II.B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A real orthogonal mode transformation R (old modes c_a = sum_i R[a,i] d_i,
the convention of ``integrals.rotate``) maps the integrals to
T' = R^T T R and W'_ijkl = sum R_ai R_bj R_ck R_dl W_abcd.  On Fock space it
is U = exp(K), K = sum_ab kappa_ab a+_a a_b with kappa = log(R^T): since
exp(K) a+_p exp(-K) = sum_a a+_a (exp kappa)_ap, U H(T, W) U^+ = H(T', W'),
and the state psi of the old modes has the amplitudes U psi in the new
ones.  ``rotate_state`` applies U to a state of a particle-number sector
(the generator built term by term with Jordan-Wigner signs, its exponential
applied by scipy's ``expm_multiply``).

``half_renyi`` is S_1/2 = 2 ln sum_k sqrt(p_k) of the bipartition (modes
< cut | modes >= cut), p_k the squared Schmidt coefficients (Sec. II.B:
the quantity the two-mode rotations minimise).  Left modes come first in
the bitstring order, so the Schmidt matrix is the amplitude array indexed
by (left bits, right bits) without signs.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ed import popcount


def _sign_below(f, p):
    return 1 - 2 * (popcount(f & ((np.int64(1) << np.int64(p)) - 1)) & 1)


def one_body_operator(kappa, basis):
    """Sparse matrix of sum_ab kappa_ab a+_a a_b on a sorted bitstring basis
    (a closed particle-number sector)."""
    basis = np.asarray(basis, dtype=np.int64)
    index = {int(f): k for k, f in enumerate(basis)}
    rows, cols, vals = [], [], []
    nso = kappa.shape[0]
    for a in range(nso):
        for b in range(nso):
            if kappa[a, b] == 0.0:
                continue
            occ_b = ((basis >> b) & 1).astype(bool)
            f = basis[occ_b]
            s1 = _sign_below(f, b)
            g = f ^ (np.int64(1) << np.int64(b))
            free_a = ((g >> a) & 1) == 0
            f, s1, g = f[free_a], s1[free_a], g[free_a]
            s2 = _sign_below(g, a)
            h = g | (np.int64(1) << np.int64(a))
            src = np.nonzero(occ_b)[0][free_a]
            rows += [index[int(x)] for x in h]
            cols += src.tolist()
            vals += (kappa[a, b] * s1 * s2).tolist()
    n = len(basis)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def rotate_state(psi, basis, R, spinful=False):
    """Amplitudes in the rotated modes (module docstring) of the state psi."""
    R = np.asarray(R, dtype=np.float64)
    kappa = np.real(sla.logm(R.T))
    kappa = 0.5 * (kappa - kappa.T)  # exactly antisymmetric
    if spinful:  # the same rotation for both spin components, no spin mixing
        kappa = np.kron(kappa, np.eye(2))
    K = one_body_operator(kappa, basis)
    return spla.expm_multiply(K, np.asarray(psi, dtype=np.float64))


def givens(n, i, j, theta):
    """Rotation by theta in the plane of modes i and j (n x n)."""
    R = np.eye(n)
    c, s = np.cos(theta), np.sin(theta)
    R[i, i] = R[j, j] = c
    R[i, j], R[j, i] = -s, s
    return R


def schmidt_weights(psi, basis, cut):
    """Squared Schmidt coefficients of the bipartition (spin-orbitals < cut |
    >= cut)."""
    basis = np.asarray(basis, dtype=np.int64)
    left = basis & ((np.int64(1) << np.int64(cut)) - 1)
    right = basis >> np.int64(cut)
    lk, li = np.unique(left, return_inverse=True)
    rk, ri = np.unique(right, return_inverse=True)
    M = np.zeros((len(lk), len(rk)))
    M[li, ri] = psi
    s = np.linalg.svd(M, compute_uv=False)
    return s ** 2 / np.sum(s ** 2)


def half_renyi(psi, basis, cut):
    """S_1/2 = 2 ln sum_k sqrt(p_k) of the bipartition at spin-orbital cut."""
    p = schmidt_weights(psi, basis, cut)
    return float(2.0 * np.log(np.sum(np.sqrt(np.clip(p, 0.0, None)))))


def best_two_mode_angle(psi, basis, n_modes, i, j, cut, thetas, spinful=False):
    """The two-mode micro-iteration: the angle of the (i, j) rotation that
    minimises S_1/2 at `cut`, from a scan of the grid `thetas` refined by a
    bounded scalar minimisation within one grid step of the best point;
    returns (theta, S_1/2)."""
    from scipy.optimize import minimize_scalar

    def f(th):
        return half_renyi(rotate_state(psi, basis, givens(n_modes, i, j, th), spinful), basis, cut)
    thetas = np.asarray(thetas, dtype=np.float64)
    vals = [f(th) for th in thetas]
    k = int(np.argmin(vals))
    step = float(np.max(np.diff(thetas))) if len(thetas) > 1 else 0.0
    if step > 0.0:
        r = minimize_scalar(f, bounds=(thetas[k] - step, thetas[k] + step), method='bounded',
                            options={'xatol': 1e-10})
        if r.fun < vals[k]:
            return float(r.x), float(r.fun)
    return float(thetas[k]), float(vals[k])
