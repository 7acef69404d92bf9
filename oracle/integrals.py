"""Oracle: one- and two-body parameters T, V of Eq. (1) for the lattice models.

Conventions (all FP64, dense, literal sums of Eq. (1), no implied 1/2):

    H = sum_pq T[p,q] a+_p a_q + sum_pqrs V[p,q,r,s] a+_p a+_q a_r a_s

``p`` is a spin-orbital index.  Spinless models have one spin-orbital per
mode.  Spin-1/2 models use ``p = 2*mode + sigma`` with sigma = 0 (up),
1 (down), i.e. the local basis of Eq. (4) ordered up-bit first.

Lattice (Sec. II.A, torus geometry): site (x, y) with 0 <= x < Lx,
0 <= y < Ly; chain position of a site is the row-major snake
``y*Lx + (x if y even else Lx-1-x)``.  Nearest-neighbour bonds
(x,y)-(x+1,y) and (x,y)-(x,y+1) with periodic wrap, each counted once.

Hopping sign: the hopping enters as ``-t`` (Eq. (2)/(3) print ``+t``; on
bipartite tori with nearest-neighbour hopping the two are related by a gauge
transformation and give identical spectra).  The on-site Hubbard term of
Eq. (2) is read as ``U sum_i n_i,up n_i,down``.

Momentum basis: plane-wave modes k = (2 pi a / Lx, 2 pi b / Ly), mode label
b*Lx + a, ordered along the chain by single-particle energy
eps_k = -2t (cos kx + cos ky) ascending, ties by mode label.

Mode transformation (Sec. II.B): old modes c_a = sum_i R[a,i] d_i with R real
orthogonal; the parameters transform as T' = R^T T R and
V'[i,j,k,l] = sum R[a,i] R[b,j] R[c,k] R[d,l] V[a,b,c,d].
"""
import numpy as np


def snake_position(x, y, Lx):
    """Chain position of lattice site (x, y) in the row-major snake order."""
    return y * Lx + (x if y % 2 == 0 else Lx - 1 - x)


def torus_bonds(Lx, Ly):
    """Nearest-neighbour bonds of an Lx x Ly torus, each listed once.

    A direction of extent 1 contributes no bond (no self-loops).
    """
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            for nb in (((x + 1) % Lx, y), (x, (y + 1) % Ly)):
                if nb != (x, y):
                    bonds.append(((x, y), nb))
    return bonds


def spinless_real_space(Lx, Ly, t, V):
    """Eq. (3) with t' = 0 on the torus, snake order.  Returns (T, V4)."""
    n = Lx * Ly
    T = np.zeros((n, n))
    W = np.zeros((n, n, n, n))
    for a, b in torus_bonds(Lx, Ly):
        i = snake_position(*a, Lx)
        j = snake_position(*b, Lx)
        T[i, j] += -t
        T[j, i] += -t
        # n_i n_j = a+_i a+_j a_j a_i
        W[i, j, j, i] += V
    return T, W


def hubbard_real_space(Lx, Ly, t, U):
    """Eq. (2) on the torus, snake order, spin-orbital p = 2*site + sigma."""
    n = Lx * Ly
    nso = 2 * n
    T = np.zeros((nso, nso))
    W = np.zeros((nso, nso, nso, nso))
    for a, b in torus_bonds(Lx, Ly):
        i = snake_position(*a, Lx)
        j = snake_position(*b, Lx)
        for s in (0, 1):
            T[2 * i + s, 2 * j + s] += -t
            T[2 * j + s, 2 * i + s] += -t
    for i in range(n):
        up, dn = 2 * i, 2 * i + 1
        # n_up n_dn = a+_up a+_dn a_dn a_up
        W[up, dn, dn, up] += U
    return T, W


def momentum_modes(Lx, Ly, t):
    """Return (chain order of mode labels, k-vectors, eps) for the torus.

    ``order[c]`` is the mode label placed at chain position c.
    """
    labels = np.arange(Lx * Ly)
    ka = 2.0 * np.pi * (labels % Lx) / Lx
    kb = 2.0 * np.pi * (labels // Lx) / Ly
    eps = -2.0 * t * (np.cos(ka) + np.cos(kb))
    # ascending energy, ties by label; round to suppress cos() noise
    key = np.round(eps, 12)
    order = np.array(sorted(labels, key=lambda m: (key[m], m)))
    return order, np.stack([labels % Lx, labels // Lx], axis=1), eps


def spinless_momentum(Lx, Ly, t, V):
    """Eq. (3) (t'=0) Fourier transformed to plane-wave modes.

    V[k1,k2,k3,k4] = (V/N) (cos qx + cos qy) delta(k1+k2 = k3+k4), q = k3-k2
    (the real form obtained by symmetrising over the relabelling of the two
    particles, which leaves the operator sum unchanged).
    """
    n = Lx * Ly
    order, kint, eps = momentum_modes(Lx, Ly, t)
    T = np.diag(eps[order])
    W = np.zeros((n, n, n, n))
    pos = np.empty(n, dtype=int)
    pos[order] = np.arange(n)
    for m1 in range(n):
        for m2 in range(n):
            for m3 in range(n):
                # k4 = k1 + k2 - k3
                ax = (kint[m1, 0] + kint[m2, 0] - kint[m3, 0]) % Lx
                by = (kint[m1, 1] + kint[m2, 1] - kint[m3, 1]) % Ly
                m4 = by * Lx + ax
                qx = 2.0 * np.pi * (kint[m3, 0] - kint[m2, 0]) / Lx
                qy = 2.0 * np.pi * (kint[m3, 1] - kint[m2, 1]) / Ly
                W[pos[m1], pos[m2], pos[m3], pos[m4]] += V / n * (np.cos(qx) + np.cos(qy))
    return T, W


def hubbard_momentum(Lx, Ly, t, U):
    """Eq. (2) in plane-wave modes; spin-orbital p = 2*chainpos + sigma.

    V[(k1 up),(k2 dn),(k3 dn),(k4 up)] = U/N delta(k1+k2 = k3+k4).
    """
    n = Lx * Ly
    nso = 2 * n
    order, kint, eps = momentum_modes(Lx, Ly, t)
    pos = np.empty(n, dtype=int)
    pos[order] = np.arange(n)
    T = np.zeros((nso, nso))
    for m in range(n):
        for s in (0, 1):
            T[2 * pos[m] + s, 2 * pos[m] + s] = eps[m]
    W = np.zeros((nso, nso, nso, nso))
    for m1 in range(n):
        for m2 in range(n):
            for m3 in range(n):
                ax = (kint[m1, 0] + kint[m2, 0] - kint[m3, 0]) % Lx
                by = (kint[m1, 1] + kint[m2, 1] - kint[m3, 1]) % Ly
                m4 = by * Lx + ax
                W[2 * pos[m1], 2 * pos[m2] + 1, 2 * pos[m3] + 1, 2 * pos[m4]] += U / n
    return T, W


def rotate(T, W, R, spinful=False):
    """Mode transformation on the parameters (Sec. II.B).

    ``R`` acts on modes (n x n, real orthogonal), c_a = sum_i R[a,i] d_i.
    For spin-1/2 models the same R is used for both spin components.
    """
    if spinful:
        R = np.kron(R, np.eye(2))
    T2 = R.T @ T @ R
    W2 = np.einsum('ai,bj,ck,dl,abcd->ijkl', R, R, R, R, W, optimize=True)
    return T2, W2


def is_hermitian(T, W, tol=1e-12):
    """Hermiticity of Eq. (1) for real parameters: T = T^T, V_pqrs = V_srqp."""
    scale = max(1.0, np.abs(T).max(initial=0.0), np.abs(W).max(initial=0.0))
    return (np.abs(T - T.T).max(initial=0.0) <= tol * scale and
            np.abs(W - W.transpose(3, 2, 1, 0)).max(initial=0.0) <= tol * scale)
