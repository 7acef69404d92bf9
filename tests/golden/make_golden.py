"""Writes tests/golden/ed_energies.json using only the CPU oracle.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seeded_inputs as si  # noqa: E402
from oracle import dmrg, ed  # noqa: E402
from oracle import integrals as I  # noqa: E402


def main():
    out = {}
    T, W = I.spinless_real_space(4, 4, 1.0, 1.0)
    out['spinless_4x4_t1_V1_N8'] = float(ed.ground_energy(T, W, 8)[0])
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    out['hubbard_3x3_t1_U4_4up4dn'] = float(ed.ground_energy(T, W, 8, True, 4)[0])
    T, W = I.spinless_real_space(4, 5, 1.0, 1.0)
    out['spinless_4x5_t1_V1_N10'] = float(ed.ground_energy(T, W, 10)[0])
    # truncated two-site DMRG of the oracle: 4x4 spinless V=1, D=64, 6 sweeps
    # (initial MPS: bond_profile(D=16), random_mps seed 1; start vectors seed 3)
    T, W = I.spinless_real_space(4, 4, 1.0, 1.0)
    ch = dmrg.Chain(T, W, 16, False, (8, 0))
    bonds = si.bond_profile(16, False, (8, 0), 16)
    mps = dmrg.MPS(ch, bonds, si.random_mps(bonds, False, 1, 0))
    out['spinless_4x4_t1_V1_N8_dmrg_D64_6sweeps'] = float(dmrg.sweep_energy(ch, mps, [64], 6)[-1])
    with open(os.path.join(HERE, 'ed_energies.json'), 'w') as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write('\n')
    print(out)


if __name__ == '__main__':
    main()
