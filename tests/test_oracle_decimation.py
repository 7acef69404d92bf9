"""Pins of the oracle's decimation (Diag_D) on states with a known Schmidt
spectrum.

A two-site vector with k nonzero elements, no two of which share a row of
the cut (left enlarged block state (a, s1, i)) or a column ((s2, b, j)), is
already in Schmidt form: its reduced density matrix on either side is
diagonal with the squared elements as eigenvalues.  Choosing those squares
p_1..p_k fixes, by the definitions of Sec. II.B, everything decimation
reports:

* truncation error = the discarded weight, sum of the k - D smallest p;
* von Neumann entropy S_vN = -sum p ln p (natural logarithm);
* half-Renyi entropy S_1/2 = 2 ln sum sqrt(p);
* for D <= k, the D kept states lie in the sectors of the D largest p;
* tie flag when p_D and p_(D+1) coincide.

The entropies and the truncation error are properties of the normalised
state, so a scaled vector must give the same values.  A log2-for-ln slip,
an unnormalised density matrix, a dropped square root or a wrong discarded
set each fails one of these tests.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import dmrg
from oracle import integrals as I


def _problem(spinful):
    if spinful:
        T, W = I.hubbard_momentum(3, 2, 1.0, 4.0)
        ch = dmrg.Chain(T, W, 6, True, (2, 2))
        D0, l = 6, 2
    else:
        T, W = I.spinless_real_space(3, 3, 1.0, 1.0)
        ch = dmrg.Chain(T, W, 9, False, (4, 0))
        D0, l = 8, 3
    bonds = si.bond_profile(ch.n, spinful, ch.target, D0)
    mps = dmrg.MPS(ch, bonds, si.random_mps(bonds, spinful, 3, l))
    return mps, l


def _schmidt_state(mps, l, p, seed):
    """Two-site vector whose Schmidt coefficients across the cut are sqrt(p):
    len(p) elements with pairwise distinct rows (a, s1, i) and columns
    (s2, b, j), random signs.  Returns the vector and the sector (quantum
    numbers of the left enlarged block) of each placed element."""
    layout, dim = dmrg.psi_layout(mps, l)
    ch = mps.chain
    rng = np.random.default_rng(seed)
    cells = []
    for (a, s1, s2, b, off, ma, mb) in layout:
        for i in range(ma):
            for j in range(mb):
                cells.append((off + i * mb + j, (a, s1, i), (s2, b, j),
                              dmrg.add(mps.bonds[l][a][0], ch.q(s1))))
    order = rng.permutation(len(cells))
    x = np.zeros(dim)
    used_r, used_c, sect = set(), set(), []
    it = iter(order)
    for pv in p:
        for c in it:
            pos, r, col, Q = cells[c]
            if r in used_r or col in used_c:
                continue
            used_r.add(r)
            used_c.add(col)
            x[pos] = np.sqrt(pv) * rng.choice([-1.0, 1.0])
            sect.append(Q)
            break
        else:
            raise AssertionError('not enough independent rows and columns for the spectrum')
    return x, sect


def _entropies(p):
    p = np.asarray(p, dtype=np.float64)
    p = p / p.sum()
    return float(-(p * np.log(p)).sum()), float(2.0 * np.log(np.sqrt(p).sum()))


@pytest.mark.parametrize('spinful', [False, True])
@pytest.mark.parametrize('direction', [+1, -1])
def test_product_state_has_no_entanglement(spinful, direction):
    mps, l = _problem(spinful)
    x, sect = _schmidt_state(mps, l, [1.0], 11)
    # D = 1 keeps the one state, in its own sector
    nb, t, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, 1, direction)
    assert trunc == 0.0
    assert abs(svn) < 1e-15 and abs(shalf) < 1e-15
    assert nb == [(sect[0], 1)]
    assert not tie
    # a larger D still keeps exactly D states (zero weights included) and
    # reports the same entropies
    nb, t, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, 4, direction)
    assert trunc == 0.0 and abs(svn) < 1e-15 and abs(shalf) < 1e-15
    assert sum(m for _, m in nb) == 4


@pytest.mark.parametrize('spinful', [False, True])
@pytest.mark.parametrize('direction', [+1, -1])
def test_known_spectrum_gives_entropies_and_discarded_weight(spinful, direction):
    mps, l = _problem(spinful)
    w = np.array([0.30, 0.20, 0.15, 0.12, 0.09, 0.07, 0.04, 0.02, 0.01])
    x, sect = _schmidt_state(mps, l, w, 21)
    svn_ref, shalf_ref = _entropies(w)
    for D in (len(w), 5, 3, 1):
        nb, t, trunc, svn, shalf, tie = dmrg.decimate(mps, l, x, D, direction)
        # entropies are those of the full spectrum, whatever D keeps
        assert abs(svn - svn_ref) <= 1e-13 * svn_ref
        assert abs(shalf - shalf_ref) <= 1e-13 * shalf_ref
        # the D largest weights are kept, the rest is the truncation error
        assert abs(trunc - w[D:].sum()) <= 1e-14
        assert sum(m for _, m in nb) == D
        # the kept states lie in the sectors of the D largest weights
        # (labelled by the quantum numbers of sites [0, l+1) either way)
        kept = {}
        for Q in sect[:D]:
            kept[Q] = kept.get(Q, 0) + 1
        assert dict(nb) == kept
        assert not tie


@pytest.mark.parametrize('direction', [+1, -1])
def test_scaled_state_reports_normalised_quantities(direction):
    mps, l = _problem(False)
    w = np.array([0.5, 0.25, 0.125, 0.0625, 0.0625])
    x, _ = _schmidt_state(mps, l, w, 31)
    ref = dmrg.decimate(mps, l, x, 3, direction)
    for c in (3.0, 0.01):
        got = dmrg.decimate(mps, l, c * x, 3, direction)
        assert abs(got[2] - ref[2]) <= 1e-14
        assert abs(got[3] - ref[3]) <= 1e-13 * ref[3]
        assert abs(got[4] - ref[4]) <= 1e-13 * ref[4]
        assert abs(ref[2] - 0.125) <= 1e-14
        # the new site tensor is an isometry whatever the scale
        for key, blk in got[1].items():
            assert np.allclose(np.abs(blk), np.abs(ref[1][key]), atol=1e-12)


@pytest.mark.parametrize('direction', [+1, -1])
def test_tied_spectrum_raises_the_tie_flag(direction):
    mps, l = _problem(True)
    w = np.array([0.4, 0.2, 0.2, 0.1, 0.1])
    x, _ = _schmidt_state(mps, l, w, 41)
    # D = 2 cuts between the two equal weights 0.2: tie
    assert dmrg.decimate(mps, l, x, 2, direction)[5]
    # D = 3 cuts between 0.2 and 0.1: no tie
    assert not dmrg.decimate(mps, l, x, 3, direction)[5]
    # D = 4 cuts between the two 0.1 weights: tie
    assert dmrg.decimate(mps, l, x, 4, direction)[5]
