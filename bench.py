"""Benchmark: H_eff psi TFLOP/s and Davidson s/step on one MI355X.

Workload (default): Hubbard model on a 6x6 torus, t=1, U=4, 18 up + 18 down
electrons, momentum basis, U(1)xU(1), bond dimension D=1024, FP64 plain form.
A step is one pass of the hot path at one bond: Davidson diagonalisation of
H_eff (every product on the GPU), density-matrix decimation, renormalisation
of the grown block (with the operator tables of the next bond) and the start
vector for the next bond.  Steps walk to the right across the chain centre.

Synthetic environment: a short real two-site run at low bond dimension gives
the sector-dimension profile of every bond; it is scaled to D and filled with
seeded random isometries (seed 1); the operators of both blocks are then
renormalised on the GPU.  Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported:
this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 MFMA
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(mdmrg, ctx, args):
    import seeded_inputs as si
    Lx = Ly = 6
    n = Lx * Ly
    target = (18, 18)
    T, V = mdmrg.build_lattice(mdmrg.HUBBARD, mdmrg.MOMENTUM, Lx, Ly, 1.0, 4.0)
    ctx.set_hamiltonian(n, True, T, V, target)
    # profile from a short real run at low D
    b0 = si.bond_profile(n, True, target, 16)
    ctx.set_mps(*si.flatten_mps(b0, si.random_mps(b0, True, 1, 0), True))
    t0 = time.time()
    ctx.sweep(1, [args.profile_D], 1e-6)
    small = [ctx.get_bond(i) for i in range(n + 1)]
    log(f'[bench] profile run D={args.profile_D}: {time.time() - t0:.1f}s')
    bonds = si.scale_profile(small, n, True, target, args.D)
    return n, target, bonds


def cpu_baseline(mdmrg, budget_s):
    """Oracle H_eff psi on a bounded sample of the same model family
    (3x3 Hubbard, momentum basis, D=64, centre bond), timed on host cores."""
    import torch

    import seeded_inputs as si
    from oracle import dmrg
    from oracle import integrals as I
    n, spin, target, l = 9, True, (4, 4), 3
    T, W = I.hubbard_momentum(3, 3, 1.0, 4.0)
    bonds = si.bond_profile(n, spin, target, 64)
    tens = si.random_mps(bonds, spin, 5, l)
    prob = dmrg.TwoSiteProblem(dmrg.MPS(dmrg.Chain(T, W, n, spin, target), bonds, tens), l)
    ctx = mdmrg.Context(0)
    ctx.set_hamiltonian(n, spin, T, W, target)
    ctx.set_mps(*si.flatten_mps(bonds, tens, spin))
    ctx.prepare_bond(l)
    flop = ctx.heff_cost()['flop']
    x = si.random_vector(prob.dim, 1)
    t0 = time.time()
    reps = 0
    while time.time() - t0 < budget_s:
        prob.matvec(x)
        reps += 1
    dt = (time.time() - t0) / reps
    ctx.close()
    del torch
    cores = len(os.sched_getaffinity(0))
    return {'value': flop / dt / 1e12, 'unit': 'TFLOP/s', 'cores': cores, 'kind': 'oracle',
            'sample': f'oracle H_eff psi (explicit Fock projection) on 3x3 Hubbard momentum basis, D=64, '
                      f'bond 3 (dim {prob.dim}), {reps} products in {reps * dt:.1f}s; FLOP = the GPU task-list '
                      f'count of the same product ({flop:.3e}); OMP threads '
                      f'{os.environ.get("OMP_NUM_THREADS", "default")}'}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--D', type=int, default=1024)
    ap.add_argument('--profile-D', type=int, default=128)
    ap.add_argument('--tol', type=float, default=1e-7)
    ap.add_argument('--cpu-budget', type=float, default=15.0)
    ap.add_argument('--no-cpu', action='store_true')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py: --gpus {args.gpus} is not supported; this build runs on exactly one GPU '
              f'(run with --gpus 1)', file=sys.stderr)
        sys.exit(2)

    import torch

    import seeded_inputs as si
    from paper_2311_14106_amd import mdmrg
    assert torch.cuda.is_available(), 'bench.py needs a GPU'

    ctx = mdmrg.Context(0)
    n, target, bonds = make_workload(mdmrg, ctx, args)
    l0 = n // 2 - 1 - args.warmup - args.steps // 2
    t0 = time.time()
    ctx.set_mps(*si.flatten_mps(bonds, si.random_mps(bonds, True, 1, l0), True))
    ctx.prepare_bond(l0)
    log(f'[bench] environment at bond {l0} built in {time.time() - t0:.1f}s')
    _, ne = ctx.psi_layout()
    x = torch.from_numpy(si.random_vector(ne, 3)).to('cuda:0')

    def step(x):
        e, r, nmv, conv = ctx.davidson(x, tol=args.tol, max_iter=400)
        ctx.decimate(x, args.D, +1)
        ctx.renormalize(+1)
        _, ne2 = ctx.psi_layout()
        x2 = torch.empty(ne2, dtype=torch.float64, device='cuda:0')
        ctx.stvec(x, x2)
        return x2, e, r, nmv

    for w in range(args.warmup):
        x, e, r, nmv = step(x)
        log(f'[bench] warmup step {w}: E={e:.10f} |r|={r:.1e} matvecs={nmv}')
    torch.cuda.synchronize()
    s0 = ctx.stats()
    costs = []
    t0 = time.time()
    energies = []
    for k in range(args.steps):
        costs.append(ctx.heff_cost())
        x, e, r, nmv = step(x)
        energies.append(e)
        log(f'[bench] step {k}: E={e:.10f} |r|={r:.1e} matvecs={nmv}')
    torch.cuda.synchronize()
    wall = time.time() - t0
    s1 = ctx.stats()
    d = {k: s1[k] - s0[k] for k in s1}
    heff_flop = d['heff_flop']
    gemm_ms = d['heff_gemm_ms'] + d['heff_p1_ms']
    gemm_flop = d['heff_gemm_flop'] + d['heff_p1_flop']
    launches = max(1.0, d['heff_gemm_launches'] + d['heff_p1_launches'])
    # algorithmic bytes of the timed products (per-bond cost x products)
    nmv_total = d['n_matvec']
    bytes_per_mv = float(np.mean([c['bytes'] for c in costs]))
    flop_per_mv = float(np.mean([c['flop'] for c in costs]))
    intensity = flop_per_mv / max(bytes_per_mv, 1.0)
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    achieved_tf = gemm_flop / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    if intensity >= ridge:
        roof = {'bound': 'mfma', 'achieved': achieved_tf, 'peak': PEAK_FP64_TFLOPS, 'unit': 'TFLOP/s',
                'frac': achieved_tf / PEAK_FP64_TFLOPS, 'traffic': None}
    else:
        gbs = bytes_per_mv * nmv_total / (gemm_ms * 1e-3) / 1e9 if gemm_ms > 0 else 0.0
        roof = {'bound': 'hbm', 'achieved': gbs, 'peak': PEAK_HBM_GBS, 'unit': 'GB/s',
                'frac': gbs / PEAK_HBM_GBS, 'traffic': None}
    roof.update({'kernel': 'k_gemm_f64 (H_eff psi grouped sector GEMM)',
                 'launches': int(launches), 'avg_launch_ms': gemm_ms / launches,
                 'flop_per_launch': gemm_flop / launches, 'intensity_flop_per_byte': intensity,
                 'kernel_tflops': achieved_tf,
                 'phase1_ms': d['heff_p1_ms'], 'phase2_ms': d['heff_gemm_ms'],
                 'phase1_tflops': d['heff_p1_flop'] / max(d['heff_p1_ms'], 1e-9) / 1e9,
                 'phase2_tflops': d['heff_gemm_flop'] / max(d['heff_gemm_ms'], 1e-9) / 1e9})
    out = {
        'metric': 'H_eff·ψ TFLOP/s and Davidson s/step, FP64 vs split-precision at fixed ΔE',
        'value': heff_flop / wall / 1e12,
        'unit': 'TFLOP/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': wall / args.steps * 1e3,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64',
        'data': 'synthetic',
        'config': {'workload': f'Hubbard 6x6 torus t=1 U=4 momentum basis, 18up+18dn, U(1)xU(1), '
                               f'D={args.D}, two-site DMRG steps from bond {l0 + args.warmup}',
                   'D': args.D, 'n_sites': n, 'precision_form': 'plain FP64',
                   'davidson_tol': args.tol},
        'davidson_s_per_step': d['diag_h_s'] / args.steps,
        'matvecs_per_step': nmv_total / args.steps,
        'heff_flop_per_matvec': flop_per_mv,
        'step_breakdown_s': {k: d[k] / args.steps for k in
                             ('diag_h_s', 'ren_s', 'tables_s', 'diag_d_s', 'stvec_s')},
        'energies': energies,
        'roofline': roof,
    }
    if not args.no_cpu:
        out['cpu_baseline'] = cpu_baseline(mdmrg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
