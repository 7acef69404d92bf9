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

Tests check these against orthogonality sums, closed forms, brute-force
diagonalisation of S^2 and the matrix elements of the plain Fock-space
operators (``tests/test_oracle_su2.py``).
"""
from fractions import Fraction
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
