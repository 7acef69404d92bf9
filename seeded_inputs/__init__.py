"""Seeded synthetic inputs shared by the oracle-side tests and the library.

This module holds NO arithmetic of the method: it only draws random numbers
and arranges them into the exchange layouts that both sides accept
(sector dimension profiles, random isometric MPS site tensors, random
vectors, random orthogonal mode rotations).  Everything is a pure function of
its arguments and a numpy ``default_rng`` seed.

Quantum-number convention of the exchange format: spinless fermions carry
(N, 0); spin-1/2 fermions carry (N_up, N_down); local state s of a spin-1/2
site has bit 0 = up occupied, bit 1 = down occupied.  Bond i is labelled by
the quantum numbers of sites [0, i).
"""
from math import comb

import numpy as np


def local_qn(s, spinful):
    if spinful:
        return (s & 1, (s >> 1) & 1)
    return (s & 1, 0)


def _count_left(i, Q, spinful):
    """Number of Fock states of i sites with quantum numbers Q."""
    if spinful:
        u, d = Q
        if u < 0 or d < 0 or u > i or d > i:
            return 0
        return comb(i, u) * comb(i, d)
    N = Q[0]
    if N < 0 or N > i or Q[1] != 0:
        return 0
    return comb(i, N)


def bond_profile(n_sites, spinful, target, D, weight_power=1.0):
    """Sector dimensions per bond for a bond dimension D.

    The largest possible dimension of sector Q at bond i is
    min(#states of the left part with Q, #states of the right part with
    target - Q).  When the sum exceeds D, dimensions are scaled down in
    proportion to (that maximum)**weight_power, then made consistent so that
    every site tensor can be left- and right-isometric.
    Returns ``bonds``: list over bonds 0..n of [(qn, dim), ...].
    """
    target = tuple(target)
    bonds = []
    for i in range(n_sites + 1):
        cand = {}
        if spinful:
            qs = [(u, dd) for u in range(i + 1) for dd in range(i + 1)]
        else:
            qs = [(N, 0) for N in range(i + 1)]
        for Q in qs:
            right = (target[0] - Q[0], target[1] - Q[1])
            m = min(_count_left(i, Q, spinful), _count_left(n_sites - i, right, spinful))
            if m > 0:
                cand[Q] = m
        tot = sum(cand.values())
        if tot > D:
            w = {Q: float(m) ** weight_power for Q, m in cand.items()}
            wt = sum(w.values())
            cand = {Q: min(cand[Q], int(np.floor(D * w[Q] / wt))) for Q in cand}
            # hand out the remainder to the largest weights
            rem = D - sum(cand.values())
            for Q in sorted(cand, key=lambda q: (-w[q], q)):
                if rem <= 0:
                    break
                full = _count_left(i, Q, spinful)
                if cand[Q] < full:
                    cand[Q] += 1
                    rem -= 1
        bonds.append({Q: m for Q, m in cand.items() if m > 0})
    return _consistent(bonds, n_sites, spinful)


def _consistent(bonds, n_sites, spinful):
    """Shrink dimensions until every site tensor can be left and right
    isometric (rows >= columns both ways)."""
    d = 4 if spinful else 2
    changed = True
    while changed:
        changed = False
        for i in range(n_sites):
            L, R = bonds[i], bonds[i + 1]
            for Qr in list(R):
                avail = sum(L.get((Qr[0] - local_qn(s, spinful)[0], Qr[1] - local_qn(s, spinful)[1]), 0)
                            for s in range(d))
                if R[Qr] > avail:
                    R[Qr] = avail
                    changed = True
                if R[Qr] == 0:
                    del R[Qr]
        for i in range(n_sites - 1, -1, -1):
            L, R = bonds[i], bonds[i + 1]
            for Ql in list(L):
                avail = sum(R.get((Ql[0] + local_qn(s, spinful)[0], Ql[1] + local_qn(s, spinful)[1]), 0)
                            for s in range(d))
                if L[Ql] > avail:
                    L[Ql] = avail
                    changed = True
                if L[Ql] == 0:
                    del L[Ql]
    return [sorted(b.items()) for b in bonds]


def scale_profile(bonds_small, n_sites, spinful, target, D):
    """Scale a recorded sector-dimension profile (list of [(qn, dim)] per
    bond, e.g. from a short low-D run) to bond dimension D: every sector
    keeps its share of the bond, capped by the largest possible dimension
    (the smaller Fock count of the two sides), then made consistent."""
    target = tuple(target)
    out = []
    for i, b in enumerate(bonds_small):
        tot = sum(m for _, m in b)
        nb = {}
        for Q, m in b:
            right = (target[0] - Q[0], target[1] - Q[1])
            cap = min(_count_left(i, Q, spinful), _count_left(n_sites - i, right, spinful))
            nb[tuple(Q)] = max(1, min(cap, int(round(m * D / max(tot, 1)))))
        # trim to D (largest first keeps the shape)
        while sum(nb.values()) > D:
            Q = max(nb, key=lambda q: (nb[q], q))
            nb[Q] -= 1
            if nb[Q] == 0:
                del nb[Q]
        out.append(nb)
    return _consistent(out, n_sites, spinful)


def random_mps(bonds, spinful, seed, center):
    """Random MPS: sites < center left-isometric, sites > center+1
    right-isometric, sites center and center+1 random Gaussian.

    Returns a list of dicts {(l, s, r): block}.
    """
    rng = np.random.default_rng(seed)
    n = len(bonds) - 1
    d = 4 if spinful else 2
    tensors = []
    for i in range(n):
        Lb, Rb = bonds[i], bonds[i + 1]
        t = {}
        if i < center:
            for r, (Qr, mr) in enumerate(Rb):
                rows = []
                for l, (Ql, ml) in enumerate(Lb):
                    for s in range(d):
                        q = local_qn(s, spinful)
                        if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                            rows.append((l, s, ml))
                M = sum(m for *_, m in rows)
                Q, _ = np.linalg.qr(rng.standard_normal((M, mr)))
                off = 0
                for (l, s, ml) in rows:
                    t[(l, s, r)] = Q[off:off + ml, :].copy()
                    off += ml
        elif i > center + 1:
            for l, (Ql, ml) in enumerate(Lb):
                cols = []
                for s in range(d):
                    q = local_qn(s, spinful)
                    for r, (Qr, mr) in enumerate(Rb):
                        if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                            cols.append((s, r, mr))
                M = sum(m for *_, m in cols)
                Q, _ = np.linalg.qr(rng.standard_normal((M, ml)))
                off = 0
                for (s, r, mr) in cols:
                    t[(l, s, r)] = Q[off:off + mr, :].T.copy()
                    off += mr
        else:
            for l, (Ql, ml) in enumerate(Lb):
                for s in range(d):
                    q = local_qn(s, spinful)
                    for r, (Qr, mr) in enumerate(Rb):
                        if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                            t[(l, s, r)] = rng.standard_normal((ml, mr))
        tensors.append(t)
    return tensors


def flatten_mps(bonds, tensors, spinful):
    """Exchange arrays: (n_sect[n+1], sect_qn[2*total], sect_dim[total], data).

    ``data`` concatenates, site by site, the blocks (l, s, r) in
    lexicographic order, each row-major.
    """
    d = 4 if spinful else 2
    n_sect = np.array([len(b) for b in bonds], dtype=np.int32)
    sect_qn = np.array([q for b in bonds for (Q, m) in b for q in Q], dtype=np.int32)
    sect_dim = np.array([m for b in bonds for (Q, m) in b], dtype=np.int32)
    chunks = []
    for i, t in enumerate(tensors):
        for l, (Ql, ml) in enumerate(bonds[i]):
            for s in range(d):
                q = local_qn(s, spinful)
                for r, (Qr, mr) in enumerate(bonds[i + 1]):
                    if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                        blk = t.get((l, s, r))
                        if blk is None:
                            blk = np.zeros((ml, mr))
                        chunks.append(np.ascontiguousarray(blk, dtype=np.float64).ravel())
    data = np.concatenate(chunks) if chunks else np.zeros(0)
    return n_sect, sect_qn, sect_dim, data


def random_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def random_orthogonal(n, seed):
    """Haar-like random orthogonal n x n matrix (QR of a Gaussian)."""
    rng = np.random.default_rng(seed)
    Q, Rm = np.linalg.qr(rng.standard_normal((n, n)))
    return Q * np.sign(np.diag(Rm))[None, :]


def shell_rotation(eps_chain, seed, angle=0.1, tol=1e-12):
    """Seeded rotation within degenerate single-particle shells.

    ``eps_chain`` are the mode energies in chain order.  For each maximal run
    of modes with |delta eps| < tol and size >= 2, an antisymmetric Gaussian
    X is scaled to spectral norm ``angle`` and R = expm(X) is placed on that
    block.  Returns the n x n orthogonal matrix.
    """
    from scipy.linalg import expm
    rng = np.random.default_rng(seed)
    eps = np.asarray(eps_chain)
    n = len(eps)
    R = np.eye(n)
    groups = {}
    for i in range(n):
        key = None
        for k in groups:
            if abs(eps[groups[k][0]] - eps[i]) < tol:
                key = k
                break
        if key is None:
            groups[len(groups)] = [i]
        else:
            groups[key].append(i)
    for idx in groups.values():
        if len(idx) < 2:
            continue
        G = rng.standard_normal((len(idx), len(idx)))
        X = G - G.T
        X *= angle / np.linalg.norm(X, 2)
        R[np.ix_(idx, idx)] = expm(X)
    return R
