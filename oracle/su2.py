"""Oracle: SU(2) coupling coefficients and spin-adapted reduced operators.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The spin-adapted form of the method (Sec. IV: the bond dimension counts
renormalised SU(2) multiplets, and products of block operators carry
Clebsch-Gordan / 6j recoupling factors) needs two exact ingredients, written
out here from their textbook definitions:

* Clebsch-Gordan coefficients <j1 m1 j2 m2 | J M> by the Racah formula;
* Wigner 6j symbols {j1 j2 j3; j4 j5 j6} by the Racah formula.

Both are evaluated in exact rational arithmetic: each is sign * sqrt(q) with
q a Fraction (a rational prefactor under the square root times the square of
a rational alternating sum), converted to FP64 only at the end.  Angular
momenta are passed as twice their value (integers), so j = 1/2 is ``1``.

On top of them, for explicit Fock-space blocks of spin-1/2 fermions:

* ``multiplet_basis``: the states of a block grouped into SU(2) multiplets
  |N, S, M, alpha>, built from highest-weight states (eigenvectors of S^2 at
  M = S) by the lowering operator, Condon-Shortley phases;
* ``reduced_element``: the Wigner-Eckart reduced matrix element of a tensor
  operator between two multiplets, in the convention
      <S' M' a'| T^k_q |S M a> = <S M k q | S' M'> <S' a'||T^k||S a> / sqrt(2S'+1);
* ``coupled_reduced``: the reduced matrix element of the coupled product
  [A^k1 x B^k2]^k from those of A and B through one 6j symbol (the
  recoupling a spin-adapted renormalisation applies to composite operators).

* ``ninej``, ``reduced_matrix``, ``singlet_product_factor`` and
  ``two_block_singlet_hubbard``: the spin-adapted superblock Hamiltonian of
  a Hubbard model on two blocks (the structure a spin-adapted DMRG step
  diagonalises), built from the blocks' multiplets, reduced creation and
  annihilation operators and the two-block singlet recoupling.

Tests check these against orthogonality sums, closed forms, brute-force
diagonalisation of S^2, the matrix elements of the plain Fock-space
operators and the exact ground energies of the plain Fock-space
diagonalisation (``tests/test_oracle_su2.py``).
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, sqrt

import numpy as np


def _f(n):
    """n! for a non-negative integer n (given as a Python int)."""
    if n < 0:
        raise ValueError('negative factorial')
    return factorial(n)


def _half(t):
    """Integer value of t/2 (t even) -- used for sums of angular momenta."""
    assert t % 2 == 0, 'half-integer where an integer is required'
    return t // 2


class Root:
    """sign * sqrt(q), q a non-negative Fraction: an exact coupling coefficient."""

    def __init__(self, sign, q):
        self.sign = 0 if q == 0 else (1 if sign > 0 else -1)
        self.q = Fraction(q)

    def __float__(self):
        return self.sign * sqrt(float(self.q)) if self.q else 0.0

    def __eq__(self, other):
        return self.sign == other.sign and self.q == other.q

    def __repr__(self):
        return f'Root({self.sign:+d} sqrt({self.q}))'


def triangle(ta, tb, tc):
    """|a-b| <= c <= a+b with a+b+c integer (twice-values)."""
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


def _delta2(ta, tb, tc):
    """Squared triangle coefficient (a+b-c)!(a-b+c)!(-a+b+c)!/(a+b+c+1)!."""
    return Fraction(_f(_half(ta + tb - tc)) * _f(_half(ta - tb + tc)) * _f(_half(-ta + tb + tc)),
                    _f(_half(ta + tb + tc) + 1))


def cg(tj1, tm1, tj2, tm2, tJ, tM):
    """<j1 m1 j2 m2 | J M> (Racah formula, Condon-Shortley phase), exact."""
    if tm1 + tm2 != tM or not triangle(tj1, tj2, tJ):
        return Root(0, 0)
    for tj, tm in ((tj1, tm1), (tj2, tm2), (tJ, tM)):
        if abs(tm) > tj or (tj + tm) % 2:
            return Root(0, 0)
    pre = Fraction(tJ + 1) * _delta2(tj1, tj2, tJ)
    pre *= (_f(_half(tJ + tM)) * _f(_half(tJ - tM)) * _f(_half(tj1 - tm1)) * _f(_half(tj1 + tm1)) *
            _f(_half(tj2 - tm2)) * _f(_half(tj2 + tm2)))
    s = Fraction(0)
    for k in range(0, _half(tj1 + tj2 - tJ) + 1):
        args = (k, _half(tj1 + tj2 - tJ) - k, _half(tj1 - tm1) - k, _half(tj2 + tm2) - k,
                _half(tJ - tj2 + tm1) + k, _half(tJ - tj1 - tm2) + k)
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= _f(a)
        s += Fraction((-1) ** k, den)
    return Root(1 if s > 0 else -1, pre * s * s)


def sixj(tj1, tj2, tj3, tj4, tj5, tj6):
    """Wigner 6j symbol {j1 j2 j3; j4 j5 j6} (Racah formula), exact."""
    tri = ((tj1, tj2, tj3), (tj1, tj5, tj6), (tj4, tj2, tj6), (tj4, tj5, tj3))
    if not all(triangle(*t) for t in tri):
        return Root(0, 0)
    pre = Fraction(1)
    for t in tri:
        pre *= _delta2(*t)
    a = [_half(sum(t)) for t in tri]  # the four triad sums
    b = [_half(tj1 + tj2 + tj4 + tj5), _half(tj2 + tj3 + tj5 + tj6), _half(tj3 + tj1 + tj6 + tj4)]
    s = Fraction(0)
    for t in range(max(a), min(b) + 1):
        den = 1
        for x in a:
            den *= _f(t - x)
        for y in b:
            den *= _f(y - t)
        s += Fraction((-1) ** t * _f(t + 1), den)
    return Root(1 if s > 0 else -1, pre * s * s)


# ------------------------------------------------ spin-1/2 fermion blocks
# A block of n_sites sites has 2 n_sites spin-orbitals p = 2*site + sigma
# (sigma 0 = up); its states are Fock bitstrings, the state of bitstring f
# being prod_{p ascending, f_p = 1} a+_p |vac> (as in ``ed``).

def fock_op(n_so, ops):
    """Dense matrix of a product of elementary operators on all 2^n_so
    bitstrings: ops = [(p, dagger), ...] applied right to left."""
    dim = 1 << n_so
    M = np.zeros((dim, dim))
    for f in range(dim):
        g, sign = f, 1.0
        ok = True
        for p, dag in reversed(ops):
            occ = (g >> p) & 1
            if occ == dag:
                ok = False
                break
            if bin(g & ((1 << p) - 1)).count('1') % 2:
                sign = -sign
            g ^= 1 << p
        if ok:
            M[g, f] += sign
    return M


def spin_ops(n_sites):
    """S_z, S_+ and S^2 of a block of n_sites spin-1/2 fermion sites."""
    n_so = 2 * n_sites
    Sz = np.zeros((1 << n_so, 1 << n_so))
    Sp = np.zeros_like(Sz)
    for i in range(n_sites):
        up, dn = 2 * i, 2 * i + 1
        Sz += 0.5 * (fock_op(n_so, [(up, 1), (up, 0)]) - fock_op(n_so, [(dn, 1), (dn, 0)]))
        Sp += fock_op(n_so, [(up, 1), (dn, 0)])
    S2 = Sp.T @ Sp + Sz @ Sz + Sz
    return Sz, Sp, S2


def multiplet_basis(n_sites, tol=1e-10):
    """Orthonormal basis of the block's Fock space in SU(2) multiplets.

    Returns a list of multiplets (N, tS, vectors) where vectors[:, k] is the
    state with tM = tS - 2k (k = 0 .. tS), obtained from the highest-weight
    state by S_- and normalisation (Condon-Shortley: positive S_- matrix
    elements).  Highest-weight states are eigenvectors of S^2 in the
    (N, M = S) sector; degenerate ones are orthonormalised by eigh."""
    n_so = 2 * n_sites
    Sz, Sp, S2 = spin_ops(n_sites)
    Sm = Sp.T
    dim = 1 << n_so
    nbits = np.array([bin(f).count('1') for f in range(dim)])
    tmz = np.rint(2 * np.diag(Sz)).astype(int)
    out = []
    for N in range(n_so + 1):
        for tS in range(N % 2, min(N, n_so - N) + 1, 2):
            idx = np.where((nbits == N) & (tmz == tS))[0]
            if len(idx) == 0:
                continue
            sub = S2[np.ix_(idx, idx)]
            w, U = np.linalg.eigh(sub)
            target = 0.25 * tS * (tS + 2)
            sel = np.abs(w - target) < tol
            for u in U[:, sel].T:
                v = np.zeros(dim)
                v[idx] = u
                # fix the sign of each highest-weight state: first nonzero component positive
                nz = np.flatnonzero(np.abs(v) > tol)
                if v[nz[0]] < 0:
                    v = -v
                vecs = [v]
                for _ in range(tS):
                    v = Sm @ v
                    v = v / np.linalg.norm(v)
                    vecs.append(v)
                out.append((N, tS, np.array(vecs).T))
    return out


def reduced_element(mults, comps, tk, a, b, tol=1e-10):
    """<a||T^k||b> for a tensor operator given by its components
    comps[tq] (dense Fock matrices, tq = -tk..tk step 2) between multiplets
    a = (N', tS', V') and b = (N, tS, V) of ``multiplet_basis``, in the
    convention of the module docstring.  Raises AssertionError unless every
    component matrix element equals CG x reduced / sqrt(2S'+1) (the
    Wigner-Eckart theorem), i.e. unless comps really is a rank-k tensor
    between these multiplets.  Returns 0.0 when no CG coefficient connects
    them."""
    _, tSa, Va = a
    _, tSb, Vb = b
    red = None
    pairs = []
    for tq, T in comps.items():
        for kb in range(tSb + 1):
            tMb = tSb - 2 * kb
            for ka in range(tSa + 1):
                tMa = tSa - 2 * ka
                c = float(cg(tSb, tMb, tk, tq, tSa, tMa))
                me = Va[:, ka] @ T @ Vb[:, kb]
                pairs.append((c, me))
                if c != 0.0 and red is None:
                    red = me * sqrt(tSa + 1) / c
    if red is None:
        for c, me in pairs:
            assert abs(me) < tol
        return 0.0
    for c, me in pairs:
        assert abs(me - c * red / sqrt(tSa + 1)) < tol * max(1.0, abs(red)), (me, c, red)
    return red


def coupled_components(A, tk1, B, tk2, tk):
    """Components of [A^k1 x B^k2]^k_q = sum <k1 q1 k2 q2|k q> A_q1 B_q2."""
    out = {}
    for tq in range(-tk, tk + 1, 2):
        M = 0.0
        for tq1 in range(-tk1, tk1 + 1, 2):
            tq2 = tq - tq1
            if abs(tq2) > tk2:
                continue
            c = float(cg(tk1, tq1, tk2, tq2, tk, tq))
            if c:
                M = M + c * (A[tq1] @ B[tq2])
        out[tq] = M
    return out


def coupled_reduced(redA, redB, tk1, tk2, tk, a, b, mults):
    """<a||[A^k1 x B^k2]^k||b> from the reduced elements of A and B by the
    product rule (Edmonds, Angular Momentum in Quantum Mechanics, 7.1.1):

        <a||[A x B]^k||b> = (-1)^(k + S_a + S_b) sqrt(2k+1)
                            sum_c {k1 k2 k; S_b S_a S_c} <a||A||c> <c||B||b>,

    a sum over all intermediate multiplets c.  The convention of this module
    differs from Edmonds' reduced elements by (-1)^(2k) per operator, and
    (-1)^(2(k1+k2+k)) = 1, so the rule holds unchanged.  redA(a, c) and
    redB(c, b) are callables."""
    _, tSa, _ = a
    _, tSb, _ = b
    if not triangle(tSb, tk, tSa):
        return 0.0  # no rank-k operator connects S_b to S_a
    ph = (-1) ** _half(tk + tSa + tSb)
    tot = 0.0
    for c in mults:
        _, tSc, _ = c
        six = sixj(tk1, tk2, tk, tSb, tSa, tSc)
        if six.sign == 0:
            continue
        tot += ph * sqrt(tk + 1) * float(six) * redA(a, c) * redB(c, b)
    return tot


def ninej(ta, tb, tc, td, te, tf, tg, th, ti):
    """Wigner 9j symbol {a b c; d e f; g h i} from the sum over products of
    three 6j symbols (Edmonds 6.4.3):
        sum_x (-1)^(2x) (2x+1) {a b c; f i x} {d e f; b x h} {g h i; x a d};
    exact 6j factors, the sum in FP64."""
    lo = max(abs(ta - ti), abs(th - td), abs(tb - tf))
    hi = min(ta + ti, th + td, tb + tf)
    tot = 0.0
    for tx in range(lo, hi + 1, 2):
        s1 = sixj(ta, tb, tc, tf, ti, tx)
        s2 = sixj(td, te, tf, tb, tx, th)
        s3 = sixj(tg, th, ti, tx, ta, td)
        if s1.sign == 0 or s2.sign == 0 or s3.sign == 0:
            continue
        tot += (-1) ** tx * (tx + 1) * float(s1) * float(s2) * float(s3)
    return tot


@lru_cache(maxsize=None)
def cg_float(tj1, tm1, tj2, tm2, tJ, tM):
    """float(cg(...)), memoised."""
    return float(cg(tj1, tm1, tj2, tm2, tJ, tM))


def reduced_matrix(bra, ket, comps, tk, dN=None):
    """<a||T^k||b> for every multiplet a of `bra` and b of `ket` (lists of
    ``multiplet_basis``), from one component each: the bra at its top weight
    M' = S' and the first component q with a nonzero Clebsch-Gordan
    coefficient (the Wigner-Eckart theorem, pinned on small blocks by
    ``reduced_element``, makes the choice irrelevant).  comps[tq] are dense
    Fock matrices of the block; dN, if given, is the change of particle
    number the operator makes (other pairs are zero and skipped)."""
    R = np.zeros((len(bra), len(ket)))
    for ib, (Nb, tSb, Vb) in enumerate(ket):
        for ia, (Na, tSa, Va) in enumerate(bra):
            if not triangle(tSb, tk, tSa) or (dN is not None and Na - Nb != dN):
                continue
            for tq in range(-tk, tk + 1, 2):
                tMb = tSa - tq
                if abs(tMb) > tSb or (tSb - tMb) % 2:
                    continue
                c = cg_float(tSb, tMb, tk, tq, tSa, tSa)
                if c == 0.0:
                    continue
                me = Va[:, 0] @ (comps[tq] @ Vb[:, (tSb - tMb) // 2])
                R[ia, ib] = me * sqrt(tSa + 1) / c
                break
    return R


def singlet_product_factor(tSp, tS, tk):
    """Matrix element of [X^k (block 1) x Y^k (block 2)]^0 between the total
    singlets |(S' S')0> and |(S S)0> of two blocks, per unit reduced elements
    <S'||X||S> <S'||Y||S> (the convention of the module docstring), by the
    explicit sum over magnetic quantum numbers of the Clebsch-Gordan
    couplings: the two-block recoupling coefficient of a spin-adapted
    superblock Hamiltonian."""
    tot = 0.0
    for tM in range(-tS, tS + 1, 2):
        c0 = float(cg(tS, tM, tS, -tM, 0, 0))
        for tq in range(-tk, tk + 1, 2):
            tMp = tM + tq
            if abs(tMp) > tSp:
                continue
            tot += (c0 * float(cg(tSp, tMp, tSp, -tMp, 0, 0)) * float(cg(tk, tq, tk, -tq, 0, 0)) *
                    float(cg(tS, tM, tk, tq, tSp, tMp)) * float(cg(tS, -tM, tk, -tq, tSp, -tMp)) / (tSp + 1))
    return tot


def _block_hubbard(Tsp, U):
    """Dense Fock matrix of a Hubbard block: hopping Tsp (sites x sites,
    spin-diagonal) and on-site U n_up n_dn; spin-orbital p = 2 site + sigma."""
    nb = Tsp.shape[0]
    nso = 2 * nb
    H = np.zeros((1 << nso, 1 << nso))
    for i in range(nb):
        for j in range(nb):
            if Tsp[i, j] != 0.0:
                for s in (0, 1):
                    H += Tsp[i, j] * fock_op(nso, [(2 * i + s, 1), (2 * j + s, 0)])
        H += U * fock_op(nso, [(2 * i, 1), (2 * i, 0), (2 * i + 1, 1), (2 * i + 1, 0)])
    return H


def two_block_singlet_hubbard(Tsp, U, n_left, n_elec):
    """Spin-adapted superblock Hamiltonian of a Hubbard model (spatial
    hopping Tsp, on-site U) on sites [0, n_left) + [n_left, n) in the basis of
    total singlets |(a b) S=0> of a left multiplet a and a right multiplet b
    (S_a = S_b, N_a + N_b = n_elec): the block Hamiltonians act within a
    block (scalars); a hopping t_ij across the blocks is
    sum_sigma c+_i,sigma c_j,sigma = -sqrt(2) [c+_i x c~_j]^0 (c~ the rank-1/2
    annihilator, components (c_dn, -c_up)), whose singlet matrix elements are
    (-1)^N_a F(S_a', S_a) <a'||c+_i||a> <b'||c~_j||b> with F the two-block
    recoupling factor (the fermion sign moves c~_j past the N_a electrons of
    the left block in the ket), plus its transpose.  Returns (H, basis)."""
    n = Tsp.shape[0]
    nL, nR = n_left, n - n_left
    mL, mR = multiplet_basis(nL), multiplet_basis(nR)
    basis = [(ia, ib) for ia, (Na, tSa, _) in enumerate(mL) for ib, (Nb, tSb, _) in enumerate(mR)
             if tSa == tSb and Na + Nb == n_elec]
    index = {p: k for k, p in enumerate(basis)}
    HL, HR = _block_hubbard(Tsp[:nL, :nL], U), _block_hubbard(Tsp[nL:, nL:], U)
    top = lambda m: np.array([v[:, 0] for _, _, v in m]).T  # top-weight vectors
    TL, TR = top(mL), top(mR)
    hL, hR = TL.T @ HL @ TL, TR.T @ HR @ TR  # scalar blocks: equal in every M
    # <a'||H_L||a> between multiplets of equal (N, S), times delta_b'b; same for R
    A = np.array([p[0] for p in basis])
    B = np.array([p[1] for p in basis])
    keyL = np.array([mL[a][0] * 1000 + mL[a][1] for a in A])
    keyR = np.array([mR[b][0] * 1000 + mR[b][1] for b in B])
    H = hL[np.ix_(A, A)] * ((B[:, None] == B[None, :]) & (keyL[:, None] == keyL[None, :]))
    H += hR[np.ix_(B, B)] * ((A[:, None] == A[None, :]) & (keyR[:, None] == keyR[None, :]))
    nsoL, nsoR = 2 * nL, 2 * nR
    F = {}
    Ys = {}
    for i in range(nL):
        if not np.any(Tsp[i, nL:]):
            continue
        Xc = reduced_matrix(mL, mL, {1: fock_op(nsoL, [(2 * i, 1)]), -1: fock_op(nsoL, [(2 * i + 1, 1)])}, 1,
                            dN=1)
        for j in range(nR):
            t = Tsp[i, nL + j]
            if t == 0.0:
                continue
            if j not in Ys:
                Ys[j] = reduced_matrix(mR, mR, {1: fock_op(nsoR, [(2 * j + 1, 0)]),
                                                -1: -fock_op(nsoR, [(2 * j, 0)])}, 1, dN=-1)
            Yc = Ys[j]
            C = np.zeros_like(H)
            for kk, (ia, ib) in enumerate(basis):  # ket
                Na, tS = mL[ia][0], mL[ia][1]
                for ja in np.flatnonzero(Xc[:, ia]):
                    tSp = mL[ja][1]
                    for jb in np.flatnonzero(Yc[:, ib]):
                        k = index.get((int(ja), int(jb)))
                        if k is None:
                            continue
                        if (tSp, tS) not in F:
                            F[(tSp, tS)] = singlet_product_factor(tSp, tS, 1)
                        C[k, kk] += (-1) ** Na * F[(tSp, tS)] * Xc[ja, ia] * Yc[jb, ib]
            H += t * (-sqrt(2.0)) * (C + C.T)
    return H, basis
