"""Oracle: two-site DMRG with explicit Fock-space block bases (Sec. II.A).

The MPS of Eq. (4) is stored as quantum-number blocked site tensors.  Every
renormalised block state is kept as an explicit vector over the block's Fock
bitstrings, so the effective Hamiltonian is never assembled from renormalised
operators: its product with a two-site wave function is, literally,

    H_eff psi = P^T H P psi,

with P the isometry from the (left block, site, site, right block) product
basis into the fixed-particle-number Fock sector and H applied by ``ed``.
This costs 2^(spin-orbitals) memory and is only meant for small lattices.

Conventions shared with the library only through the exchange format
(documented in ``include/mdmrg.h``):

* bond i sits between site i-1 and site i; its sectors are labelled by the
  quantum numbers of sites [0, i) ("left labels"): (N, 0) for spinless
  fermions, (N_up, N_down) for spin-1/2 fermions, sorted ascending;
* site tensor i has blocks (l, s, r) with Q_r = Q_l + q(s), each a dense
  m_l x m_r matrix; local state s has bit sigma set when spin-orbital
  (site, sigma) is occupied;
* a two-site wave function at bond (l, l+1) has blocks (a, s1, s2, b),
  a a sector of bond l, b of bond l+2, with Q_a + q(s1) + q(s2) = Q_b,
  ordered lexicographically by (a, s1, s2, b); each block m_a x m_b,
  row-major, packed without padding.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import ed


class Chain:
    """Problem definition: sites, local dimension and the target sector."""

    def __init__(self, T, W, n_sites, spinful, target):
        self.T = np.asarray(T, dtype=np.float64)
        self.W = np.asarray(W, dtype=np.float64)
        self.n = n_sites
        self.ns = 2 if spinful else 1
        self.d = 1 << self.ns
        self.spinful = spinful
        self.target = tuple(target)
        assert self.T.shape[0] == self.ns * n_sites
        self._H = None
        self._basis = None

    def q(self, s):
        """Quantum numbers carried by local state s."""
        if self.spinful:
            return ((s >> 0) & 1, (s >> 1) & 1)
        return (s & 1, 0)

    def qn_of_bits(self, f, nbits):
        """Quantum numbers of a bitstring over ``nbits`` spin-orbitals."""
        if self.spinful:
            up = sum((f >> p) & 1 for p in range(0, nbits, 2))
            dn = sum((f >> p) & 1 for p in range(1, nbits, 2))
            return (up, dn)
        return (bin(f).count('1'), 0)

    def hamiltonian(self):
        if self._H is None:
            nso = self.T.shape[0]
            N = self.target[0] + self.target[1] if self.spinful else self.target[0]
            self._basis = ed.sector_basis(nso, N, self.spinful, self.target[0] if self.spinful else None)
            self._H = ed.SectorHamiltonian(self.T, self.W, self._basis)
        return self._H, self._basis


def add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def sub(a, b):
    return (a[0] - b[0], a[1] - b[1])


class MPS:
    """Block-sparse MPS: ``bonds[i]`` = list of (qn, dim); ``A[i]`` = dict."""

    def __init__(self, chain, bonds, tensors):
        self.chain = chain
        self.bonds = [list(b) for b in bonds]
        self.A = [dict(t) for t in tensors]

    def sector_index(self, i):
        return {qn: k for k, (qn, _) in enumerate(self.bonds[i])}


# --------------------------------------------------------------------------
# explicit block bases
# --------------------------------------------------------------------------

def left_basis(mps, i):
    """Explicit basis of the left block at bond i (sites [0, i)).

    Returns a list over the sectors of bond i of (bitstrings, matrix), the
    matrix having one row per bitstring (ascending) and one column per
    renormalised state.
    """
    ch = mps.chain
    # bond 0: vacuum
    cur = [(np.array([0], dtype=np.int64), np.ones((1, 1)))]
    for site in range(i):
        nxt = []
        sidx_l = mps.bonds[site]
        for r, (qr, mr) in enumerate(mps.bonds[site + 1]):
            rows_f, rows_M = [], []
            for l, (ql, ml) in enumerate(sidx_l):
                for s in range(ch.d):
                    if add(ql, ch.q(s)) != qr:
                        continue
                    blk = mps.A[site].get((l, s, r))
                    if blk is None:
                        continue
                    f, M = cur[l]
                    rows_f.append(f | (np.int64(s) << np.int64(ch.ns * site)))
                    rows_M.append(M @ blk)
            if rows_f:
                f = np.concatenate(rows_f)
                M = np.vstack(rows_M)
                order = np.argsort(f)
                nxt.append((f[order], M[order]))
            else:
                nxt.append((np.zeros(0, dtype=np.int64), np.zeros((0, mr))))
        cur = nxt
    return cur


def right_basis(mps, i):
    """Explicit basis of the right block at bond i (sites [i, n)).

    Bitstrings are relative to the block (bit 0 = first spin-orbital of site
    i).  Returned per sector of bond i (left labels).
    """
    ch = mps.chain
    n = ch.n
    cur = [(np.array([0], dtype=np.int64), np.ones((1, 1)))]  # bond n
    for site in range(n - 1, i - 1, -1):
        nxt = []
        for l, (ql, ml) in enumerate(mps.bonds[site]):
            rows_f, rows_M = [], []
            for s in range(ch.d):
                for r, (qr, mr) in enumerate(mps.bonds[site + 1]):
                    if add(ql, ch.q(s)) != qr:
                        continue
                    blk = mps.A[site].get((l, s, r))
                    if blk is None:
                        continue
                    f, M = cur[r]
                    rows_f.append(np.int64(s) | (f << np.int64(ch.ns)))
                    rows_M.append(M @ blk.T)
            if rows_f:
                f = np.concatenate(rows_f)
                M = np.vstack(rows_M)
                order = np.argsort(f)
                nxt.append((f[order], M[order]))
            else:
                nxt.append((np.zeros(0, dtype=np.int64), np.zeros((0, ml))))
        cur = nxt
    return cur


# --------------------------------------------------------------------------
# two-site wave function layout and H_eff psi
# --------------------------------------------------------------------------

def psi_layout(mps, l):
    """Blocks (a, s1, s2, b, offset, m_a, m_b) of the two-site vector."""
    ch = mps.chain
    out = []
    off = 0
    for a, (qa, ma) in enumerate(mps.bonds[l]):
        for s1 in range(ch.d):
            for s2 in range(ch.d):
                q = add(add(qa, ch.q(s1)), ch.q(s2))
                for b, (qb, mb) in enumerate(mps.bonds[l + 2]):
                    if qb == q and ma > 0 and mb > 0:
                        out.append((a, s1, s2, b, off, ma, mb))
                        off += ma * mb
    return out, off


class TwoSiteProblem:
    """H_eff at bond (l, l+1) as the projection P^T H P."""

    def __init__(self, mps, l):
        self.mps = mps
        self.l = l
        ch = mps.chain
        self.H, self.basis = ch.hamiltonian()
        self.layout, self.dim = psi_layout(mps, l)
        self.LB = left_basis(mps, l)
        self.RB = right_basis(mps, l + 2)
        self.pos = []
        shift1 = np.int64(ch.ns * l)
        shift2 = np.int64(ch.ns * (l + 1))
        shiftR = np.int64(ch.ns * (l + 2))
        for (a, s1, s2, b, off, ma, mb) in self.layout:
            fL = self.LB[a][0]
            fR = self.RB[b][0]
            g = (fL[:, None] | (np.int64(s1) << shift1) | (np.int64(s2) << shift2)
                 | (fR[None, :] << shiftR))
            p = np.searchsorted(self.basis, g)
            assert np.all(self.basis[np.minimum(p, len(self.basis) - 1)] == g)
            self.pos.append(p)

    def to_full(self, x):
        full = np.zeros(len(self.basis))
        for (a, s1, s2, b, off, ma, mb), p in zip(self.layout, self.pos):
            blk = x[off:off + ma * mb].reshape(ma, mb)
            full[p] = self.LB[a][1] @ blk @ self.RB[b][1].T
        return full

    def from_full(self, full):
        y = np.zeros(self.dim)
        for (a, s1, s2, b, off, ma, mb), p in zip(self.layout, self.pos):
            y[off:off + ma * mb] = (self.LB[a][1].T @ full[p] @ self.RB[b][1]).ravel()
        return y

    def matvec(self, x):
        return self.from_full(self.H.matvec(self.to_full(x)))

    def lowest(self, v0=None, tol=1e-13):
        """Lowest eigenpair of H_eff (plain definition: dense or Lanczos)."""
        if self.dim <= 600:
            Hd = np.column_stack([self.matvec(e) for e in np.eye(self.dim)])
            w, v = np.linalg.eigh(0.5 * (Hd + Hd.T))
            return w[0], v[:, 0]
        op = spla.LinearOperator((self.dim, self.dim), matvec=self.matvec, dtype=np.float64)
        w, v = spla.eigsh(op, k=1, which='SA', tol=tol, v0=v0, ncv=min(self.dim - 1, 40))
        return w[0], v[:, 0]


# --------------------------------------------------------------------------
# decimation, renormalisation of the MPS, start vector
# --------------------------------------------------------------------------

def decimate(mps, l, x, D, direction, tie_tol=1e-10):
    """Reduced-density-matrix truncation of the two-site vector (Diag_D).

    direction +1: rho of the left enlarged block (bond l+1 basis, left
    canonical A_l); direction -1: rho of the right enlarged block (right
    canonical tensor at site l+1).  Keeps exactly min(D, rank-dimension)
    states, ranked by eigenvalue with ties broken by (sector label, index).
    Returns (new bond list, new site tensor, truncation error, S_vN, S_1/2,
    tie flag).
    """
    ch = mps.chain
    layout, _ = psi_layout(mps, l)
    # rho is the density matrix of the normalised state (trace 1), so that
    # the weights, the truncation error and the entropies do not depend on
    # the scale of x
    norm2 = float(np.dot(x, x))
    assert norm2 > 0.0, 'decimate: zero vector'
    rows = {}   # sector -> list of row keys
    cols = {}
    blocks = []
    for (a, s1, s2, b, off, ma, mb) in layout:
        blk = x[off:off + ma * mb].reshape(ma, mb)
        if direction > 0:
            Q = add(mps.bonds[l][a][0], ch.q(s1))
            rk, ck = (a, s1), (s2, b)
        else:
            Q = sub(mps.bonds[l + 2][b][0], ch.q(s2))
            rk, ck = (s2, b), (a, s1)
            blk = blk.T
        rows.setdefault(Q, [])
        cols.setdefault(Q, [])
        if rk not in rows[Q]:
            rows[Q].append(rk)
        if ck not in cols[Q]:
            cols[Q].append(ck)
        blocks.append((Q, rk, ck, blk))
    evals = []
    vecs = {}
    row_dims = {}
    for Q in sorted(rows):
        rows[Q].sort()
        cols[Q].sort()
        if direction > 0:
            rd = [mps.bonds[l][a][1] for (a, s1) in rows[Q]]
            cd = [mps.bonds[l + 2][b][1] for (s2, b) in cols[Q]]
        else:
            rd = [mps.bonds[l + 2][b][1] for (s2, b) in rows[Q]]
            cd = [mps.bonds[l][a][1] for (a, s1) in cols[Q]]
        ro = np.concatenate([[0], np.cumsum(rd)])
        co = np.concatenate([[0], np.cumsum(cd)])
        M = np.zeros((ro[-1], co[-1]))
        for (QQ, rk, ck, blk) in blocks:
            if QQ != Q:
                continue
            i = rows[Q].index(rk)
            j = cols[Q].index(ck)
            M[ro[i]:ro[i + 1], co[j]:co[j + 1]] = blk
        rho = M @ M.T / norm2
        w, v = np.linalg.eigh(rho)
        w = w[::-1]
        v = v[:, ::-1]
        vecs[Q] = v
        row_dims[Q] = (ro, rd)
        for k, lam in enumerate(w):
            evals.append((-lam, Q, k))
    evals.sort()
    keep = evals[:D]
    tie = (len(evals) > D and
           abs(evals[D][0] - evals[D - 1][0]) < tie_tol * max(-evals[D - 1][0], 1e-300))
    lam_all = np.array([-e[0] for e in evals])
    lam_keep = np.array([-e[0] for e in keep])
    trunc = max(0.0, 1.0 - lam_keep.sum())
    # entropies over the numerical rank: eigenvalues at the rounding level
    # (|lambda| <~ 1e-16) would enter sqrt() as ~1e-8 noise
    p = lam_all[lam_all > 1e-14]
    s_vn = float(-(p * np.log(p)).sum())
    s_half = float(2.0 * np.log(np.sqrt(p).sum()))
    count = {}
    for (_, Q, k) in keep:
        count[Q] = count.get(Q, 0) + 1
    new_bond = [(Q, count[Q]) for Q in sorted(count)]
    newidx = {Q: i for i, (Q, _) in enumerate(new_bond)}
    tensor = {}
    for Q, kcount in count.items():
        ks = sorted(k for (_, QQ, k) in keep if QQ == Q)
        U = vecs[Q][:, ks]
        ro, rd = row_dims[Q]
        for i, rk in enumerate(rows[Q]):
            piece = U[ro[i]:ro[i + 1], :]
            if direction > 0:
                a, s1 = rk
                tensor[(a, s1, newidx[Q])] = piece.copy()
            else:
                s2, b = rk
                tensor[(newidx[Q], s2, b)] = piece.T.copy()
    return new_bond, tensor, trunc, s_vn, s_half, bool(tie)


def start_vector(prob_old, x, prob_new):
    """Wave-function transformation to the next bond (StVec).

    Plain definition: psi' = P'^T P psi, with P the old and P' the new
    isometry into the Fock sector.  When the new basis spans the truncated
    state this is the exact representation of that state at the next bond.
    """
    return prob_new.from_full(prob_old.to_full(x))


def sweep_energy(chain, mps, D_schedule, n_sweeps, rng_seed=3, verbose=False):
    """Full two-site sweeps; returns the list of energies per optimisation.

    Each optimisation uses the lowest eigenpair of H_eff (plain definition)
    from a seeded random start vector.
    """
    rng = np.random.default_rng(rng_seed)
    n = chain.n
    energies = []
    for sw in range(n_sweeps):
        D = D_schedule[min(sw, len(D_schedule) - 1)]
        for l in list(range(0, n - 2)):
            prob = TwoSiteProblem(mps, l)
            e, v = prob.lowest(v0=rng.standard_normal(prob.dim))
            energies.append(e)
            nb, t, *_ = decimate(mps, l, v, D, +1)
            mps.bonds[l + 1] = nb
            mps.A[l] = t
        for l in list(range(n - 2, 0, -1)):
            prob = TwoSiteProblem(mps, l)
            e, v = prob.lowest(v0=rng.standard_normal(prob.dim))
            energies.append(e)
            nb, t, *_ = decimate(mps, l, v, D, -1)
            mps.bonds[l + 1] = nb
            mps.A[l + 1] = t
        if verbose:
            print('sweep', sw, 'D', D, 'E', energies[-1])
    return energies
