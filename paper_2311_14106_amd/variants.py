"""Per-variant timing of the H_eff product at one bond.

Builds the environment of one bond of a benchmark workload (the recorded
sector profile scaled to D, seeded random isometries; as ``bench.py``), then
runs the product of the effective Hamiltonian with a fixed vector in each
requested precision form with each requested tile variant of the grouped
kernel forced (MDMRG_OPT_GEMM_VARIANT), and prints the GEMM milliseconds per
product from the library's HIP events.  All variants give the same bits,
which is checked against the autotuned product.

    python -m paper_2311_14106_amd.variants --workload hubbard6x6 --D 2048 --bond 17

Used for the tuning record of the kernel and, under rocprofv3 counter
collection, for per-variant counter summaries.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PREC = {'fp64': 0, 'fp32': 1, 'bf16x3': 2, 'bf16x6': 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--workload', choices=('hubbard6x6', 'spinless8x8'), default='hubbard6x6')
    ap.add_argument('--D', type=int, default=2048)
    ap.add_argument('--bond', type=int, default=None, help='default: the middle bond')
    ap.add_argument('--reps', type=int, default=4)
    ap.add_argument('--variants', default='-1,0,1,2,3', help='-1: autotuned')
    ap.add_argument('--precs', default='fp64,fp32,bf16x3')
    ap.add_argument('--lib', default=None, help='path of another build of libmdmrg.so (default: the in-tree one)')
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch

    import seeded_inputs as si
    from paper_2311_14106_amd import mdmrg
    ctx = mdmrg.Context(0, path=a.lib)
    if a.workload == 'hubbard6x6':
        n, spin, target = 36, True, (18, 18)
        T, V = mdmrg.build_lattice(mdmrg.HUBBARD, mdmrg.MOMENTUM, 6, 6, 1.0, 4.0)
        prof = 'sector_profile_hubbard6x6_D128.json'
    else:
        n, spin, target = 64, False, (32, 0)
        T, V = mdmrg.build_lattice(mdmrg.SPINLESS, mdmrg.MOMENTUM, 8, 8, 1.0, 2.0)
        T, V = mdmrg.rotate_modes(si.shell_rotation(np.diag(T), 0), T, V, False)
        prof = 'sector_profile_spinless8x8_D64.json'
    ctx.set_hamiltonian(n, spin, T, V, target)
    with open(os.path.join(HERE, 'data', prof)) as f:
        small = [[(tuple(q), m) for q, m in b] for b in json.load(f)['bonds']]
    bonds = si.scale_profile(small, n, spin, target, a.D)
    l = n // 2 - 1 if a.bond is None else a.bond
    ctx.set_option(mdmrg.OPT_KEEP_ENVS, 3)
    ctx.set_mps(*si.flatten_mps(bonds, si.random_mps(bonds, spin, 1, l), spin))
    t0 = time.time()
    ctx.prepare_bond(l)
    torch.cuda.synchronize()
    _, ne = ctx.psi_layout()
    flop = ctx.heff_cost()['flop']
    print(f'{a.workload} D={a.D} bond {l}: environment {time.time() - t0:.1f} s, |psi| {ne}, '
          f'{flop / 1e12:.3f} TFLOP per product', flush=True)
    x = torch.from_numpy(si.random_vector(ne, 3)).to('cuda:0')
    y = torch.empty_like(x)
    for pname in a.precs.split(','):
        prec = PREC[pname]
        ref = None
        for v in [int(s) for s in a.variants.split(',')]:
            ctx.set_option(mdmrg.OPT_GEMM_VARIANT, v)
            for _ in range(5 if v < 0 else 1):  # autotuning trials / warm-up
                ctx.heff_apply(x, y, prec=prec)
            torch.cuda.synchronize()
            s0 = ctx.stats()
            for _ in range(a.reps):
                ctx.heff_apply(x, y, prec=prec)
            torch.cuda.synchronize()
            s1 = ctx.stats()
            key = 'heff_kernel_ms' if prec == 0 else 'split_gemm_ms'
            ms = (s1[key] - s0[key]) / a.reps
            yc = y.cpu().numpy()
            if ref is None:
                ref = yc
            same = bool(np.array_equal(yc, ref))
            name = 'autotuned' if v < 0 else mdmrg.Context.KERNELS[v]
            print(f'{pname:7s} {name:12s} {ms:9.2f} ms per product  {flop / ms / 1e9:7.1f} TFLOP/s  '
                  f'same bits {same}', flush=True)
            assert same, 'tile variants must give the same bits'
    ctx.set_option(mdmrg.OPT_GEMM_VARIANT, -1)
    ctx.close()


if __name__ == '__main__':
    main()
