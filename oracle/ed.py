"""Oracle: exact diagonalisation of Eq. (1) in a fixed particle-number sector.

Fock states are bitstrings; bit p set <=> spin-orbital p occupied.  The state
of bitstring f is  prod_{p ascending, f_p = 1} a+_p |vac>,  so applying a_p or
a+_p picks up (-1)^(number of occupied spin-orbitals q < p) (Jordan-Wigner).

Two independent ways of applying H are provided:

* ``apply_terms_literal`` -- every term of Eq. (1) applied to every bitstring
  one operator at a time, right to left (brute force; tiny systems only);
* ``SectorHamiltonian``  -- the same operator written through the
  intermediate (N-1)- and (N-2)-particle spaces:
      H_1 = sum_pq T_pq a+_p a_q = A1^T (T (x) 1) A1,     A1 = [a_q]_q
      H_2 = - E^T (G (x) 1) E,   E = [a_r a_s]_{r<s},
      G[pq,rs] = V_pqrs - V_qprs - V_pqsr + V_qpsr   (p<q, r<s)
  which is what the DMRG oracle uses because it is fast.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


def sector_basis(nso, n_elec, spinful=False, n_up=None):
    """Sorted bitstrings with ``n_elec`` particles (and ``n_up`` up-spins).

    For spin-1/2 models spin-orbital p = 2*mode + sigma, sigma = 0 is up.
    """
    states = []
    for occ in itertools.combinations(range(nso), n_elec):
        if spinful and n_up is not None:
            if sum(1 for p in occ if p % 2 == 0) != n_up:
                continue
        states.append(sum(1 << p for p in occ))
    return np.array(sorted(states), dtype=np.int64)


def _sign_below(f, p):
    """(-1)^(number of set bits of f strictly below bit p), vectorised."""
    mask = (np.int64(1) << np.int64(p)) - 1
    return 1 - 2 * (popcount(f & mask) & 1)


def apply_terms_literal(T, W, basis, x):
    """Brute force: apply every term of Eq. (1) to every basis state.

    Each operator string is applied right to left, one elementary operator at
    a time, with its Jordan-Wigner sign.  O(nso^4 * dim): tiny systems only.
    """
    index = {int(f): i for i, f in enumerate(basis)}
    y = np.zeros_like(x)
    nso = T.shape[0]

    def apply_string(ops, coef):
        for i, f0 in enumerate(basis):
            f = int(f0)
            amp = coef * x[i]
            ok = True
            for (p, dag) in reversed(ops):
                occ = (f >> p) & 1
                if dag == occ:          # a+ on occupied or a on empty
                    ok = False
                    break
                below = bin(f & ((1 << p) - 1)).count('1')
                if below & 1:
                    amp = -amp
                f ^= (1 << p)
            if ok and f in index:
                y[index[f]] += amp

    for p in range(nso):
        for q in range(nso):
            if T[p, q] != 0.0:
                apply_string([(p, 1), (q, 0)], T[p, q])
    nz = np.argwhere(W != 0.0)
    for (p, q, r, s) in nz:
        apply_string([(p, 1), (q, 1), (r, 0), (s, 0)], W[p, q, r, s])
    return y


def antisymmetrised_pairs(W):
    """G[pq, rs] for p<q, r<s (pair index in itertools.combinations order)."""
    nso = W.shape[0]
    pairs = list(itertools.combinations(range(nso), 2))
    P = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    p, q = P[:, 0], P[:, 1]
    G = (W[p[:, None], q[:, None], p[None, :], q[None, :]]
         - W[q[:, None], p[:, None], p[None, :], q[None, :]]
         - W[p[:, None], q[:, None], q[None, :], p[None, :]]
         + W[q[:, None], p[:, None], q[None, :], p[None, :]])
    return P, G


class SectorHamiltonian:
    """H of Eq. (1) restricted to a sorted list of bitstrings ``basis``.

    Builds the sparse maps A1 (single annihilation) and E (pair annihilation
    a_r a_s, r<s) from the sector into the full (N-1)/(N-2)-particle spaces.
    """

    def __init__(self, T, W, basis):
        self.T = np.asarray(T, dtype=np.float64)
        self.basis = np.asarray(basis, dtype=np.int64)
        nso = self.T.shape[0]
        self.nso = nso
        dim = len(self.basis)
        # --- single annihilation a_q ------------------------------------
        rows, cols, vals, inter = [], [], [], {}
        for q in range(nso):
            occ = (self.basis >> q) & 1
            idx = np.nonzero(occ)[0]
            f2 = self.basis[idx] ^ (np.int64(1) << np.int64(q))
            sg = _sign_below(self.basis[idx], q)
            rows.append(np.full(len(idx), q)), cols.append(idx)
            vals.append(sg.astype(np.float64)), inter.setdefault('f', []).append(f2)
        f1 = np.concatenate(inter['f']) if inter else np.zeros(0, np.int64)
        uniq1, inv1 = np.unique(f1, return_inverse=True)
        self.n1 = len(uniq1)
        qrow = np.concatenate(rows)
        self.A1 = sp.csr_matrix((np.concatenate(vals), (qrow * self.n1 + inv1, np.concatenate(cols))),
                                shape=(nso * self.n1, dim))
        # --- pair annihilation a_r a_s (first a_s, then a_r), r < s ---------
        P, G = antisymmetrised_pairs(W)
        self.G = G
        keep = np.nonzero(np.abs(G).max(axis=1, initial=0.0) + np.abs(G).max(axis=0, initial=0.0) > 0)[0]
        self.keep = keep
        rows, cols, vals, f2s = [], [], [], []
        for kk, pi in enumerate(keep):
            r, s = P[pi]
            occ = ((self.basis >> r) & 1) & ((self.basis >> s) & 1)
            idx = np.nonzero(occ)[0]
            f = self.basis[idx]
            sg = _sign_below(f, s)
            f = f ^ (np.int64(1) << np.int64(s))
            sg = sg * _sign_below(f, r)
            f = f ^ (np.int64(1) << np.int64(r))
            rows.append(np.full(len(idx), kk)), cols.append(idx), vals.append(sg.astype(np.float64))
            f2s.append(f)
        if keep.size:
            f2 = np.concatenate(f2s)
            uniq2, inv2 = np.unique(f2, return_inverse=True)
            self.n2 = len(uniq2)
            prow = np.concatenate(rows)
            self.E = sp.csr_matrix((np.concatenate(vals), (prow * self.n2 + inv2, np.concatenate(cols))),
                                   shape=(len(keep) * self.n2, dim))
            self.Gk = G[np.ix_(keep, keep)]
        else:
            self.E = None
        self.dim = dim

    def matvec(self, x):
        x = np.asarray(x, dtype=np.float64)
        z = (self.A1 @ x).reshape(self.nso, self.n1)
        y = self.A1.T @ (self.T @ z).ravel()
        if self.E is not None:
            z2 = (self.E @ x).reshape(len(self.keep), self.n2)
            y = y - self.E.T @ (self.Gk @ z2).ravel()
        return y

    def ground_state(self, tol=1e-14, k=1):
        if self.dim <= 400:
            H = np.column_stack([self.matvec(e) for e in np.eye(self.dim)])
            w, v = np.linalg.eigh(0.5 * (H + H.T))
            return w[:k], v[:, :k]
        op = spla.LinearOperator((self.dim, self.dim), matvec=self.matvec, dtype=np.float64)
        rng = np.random.default_rng(12345)
        w, v = spla.eigsh(op, k=k, which='SA', tol=tol, v0=rng.standard_normal(self.dim), ncv=max(20, 2 * k + 10))
        order = np.argsort(w)
        return w[order], v[:, order]


def ground_energy(T, W, n_elec, spinful=False, n_up=None, k=1):
    nso = T.shape[0]
    basis = sector_basis(nso, n_elec, spinful, n_up)
    w, _ = SectorHamiltonian(T, W, basis).ground_state(k=k)
    return w
