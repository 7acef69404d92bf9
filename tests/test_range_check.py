"""The library's host planner on the range-checking device layer
(libmdmrg_check.so: device.hip replaced by csrc/device_check.cpp, no GPU, no
arithmetic).  Every device access of the full-size workloads -- each grouped
GEMM operand and output block, split-K partials, diagonal tasks, gathers,
vector operations and copies -- is checked against the live allocations,
and the allocated bytes are tracked:

* one DMRG step of the 6x6 Hubbard model (momentum basis) at D=1024 and of
  the rotated 8x8 spinless model at D=2048 stays inside its allocations in
  every precision form;
* the 8x8 rotated spinless model at D=4096 (the largest workload: one step at
  the middle bond, right blocks built first, renormalisation combinations in
  bounded batches, keep-envs 3) peaks below 265 GB of device memory, so it
  fits the 288 GB of one MI355X;
* a buffer shorter than the layout (a mistake planted on the CPU) is caught;
* a renormalisation that runs out of device memory leaves no current bond
  (products refused with ESTATE) and the context recovers.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import seeded_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHK = os.path.join(ROOT, 'paper_2311_14106_amd', 'libmdmrg_check.so')


@pytest.fixture(scope='module')
def chk():
    from paper_2311_14106_amd import build, mdmrg
    if not os.path.exists(CHK):
        build.build_check()
    L = mdmrg.load(CHK)
    for f in ('mdmrg_check_live_bytes', 'mdmrg_check_peak_bytes', 'mdmrg_check_launches'):
        getattr(L, f).restype = ctypes.c_int64
    L.mdmrg_check_alloc.restype = ctypes.c_void_p
    L.mdmrg_check_alloc.argtypes = [ctypes.c_int64]
    return mdmrg, L


def _context(mdmrg, L, workload, D, keep):
    ctx = mdmrg.Context(0, path=CHK)
    if workload == 'hubbard6x6':
        n, spin, target = 36, True, (18, 18)
        T, V = mdmrg.build_lattice(mdmrg.HUBBARD, mdmrg.MOMENTUM, 6, 6, 1.0, 4.0, L=L)
        prof = 'sector_profile_hubbard6x6_D128.json'
    else:
        n, spin, target = 64, False, (32, 0)
        T, V = mdmrg.build_lattice(mdmrg.SPINLESS, mdmrg.MOMENTUM, 8, 8, 1.0, 2.0, L=L)
        T, V = mdmrg.rotate_modes(si.shell_rotation(np.diag(T), 0), T, V, False, L=L)
        prof = 'sector_profile_spinless8x8_D64.json'
    ctx.set_hamiltonian(n, spin, T, V, target)
    with open(os.path.join(ROOT, 'paper_2311_14106_amd', 'data', prof)) as f:
        small = [[(tuple(q), m) for q, m in b] for b in json.load(f)['bonds']]
    bonds = si.scale_profile(small, n, spin, target, D)
    d = 4 if spin else 2
    n_sect = np.array([len(b) for b in bonds], dtype=np.int32)
    sect_qn = np.array([q for b in bonds for (Q, m) in b for q in Q], dtype=np.int32)
    sect_dim = np.array([m for b in bonds for (Q, m) in b], dtype=np.int32)
    tot = 0
    for i in range(n):
        for (Ql, ml) in bonds[i]:
            for s in range(d):
                q = si.local_qn(s, spin)
                for (Qr, mr) in bonds[i + 1]:
                    if (Ql[0] + q[0], Ql[1] + q[1]) == Qr:
                        tot += ml * mr
    data = np.empty(tot)  # never read: the checking layer copies nothing
    ctx.set_option(mdmrg.OPT_KEEP_ENVS, keep)
    i32 = ctypes.POINTER(ctypes.c_int32)
    st = ctx.lib.mdmrg_set_mps(ctx.h, n_sect.ctypes.data_as(i32), sect_qn.ctypes.data_as(i32),
                               sect_dim.ctypes.data_as(i32), data.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               tot)
    assert st == 0, ctx.lib.mdmrg_last_error(ctx.h)
    return ctx, n


def _step(mdmrg, L, ctx, l, D, precs):
    """prepare, products in each precision form, Davidson, decimation,
    renormalisation in each form (on fresh bonds) and the start vector."""
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = L.mdmrg_check_alloc(8 * ne)
    y = L.mdmrg_check_alloc(8 * ne)
    for prec in precs:
        assert ctx.lib.mdmrg_heff_apply(ctx.h, prec, ctypes.c_void_p(x), ctypes.c_void_p(y)) == 0, \
            ctx.lib.mdmrg_last_error(ctx.h)
    assert ctx.lib.mdmrg_heff_diag(ctx.h, ctypes.c_void_p(y)) == 0
    e, r, nm = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    st = ctx.lib.mdmrg_davidson(ctx.h, ctypes.c_void_p(x), ctypes.c_double(1e-7), 3, 24, ctypes.byref(e),
                                ctypes.byref(r), ctypes.byref(nm))
    assert st in (0, mdmrg.ENOCONV), ctx.lib.mdmrg_last_error(ctx.h)
    assert ctx.lib.mdmrg_decimate(ctx.h, ctypes.c_void_p(x), D, 1, None, None, None) == 0
    assert ctx.lib.mdmrg_renormalize(ctx.h, 1, precs[-1]) == 0, ctx.lib.mdmrg_last_error(ctx.h)
    _, ne2 = ctx.psi_layout()
    x2 = L.mdmrg_check_alloc(8 * ne2)
    assert ctx.lib.mdmrg_stvec(ctx.h, ctypes.c_void_p(x), ctypes.c_void_p(x2)) == 0, ctx.lib.mdmrg_last_error(ctx.h)
    return ne


@pytest.mark.parametrize('workload,D,l,keep', [('hubbard6x6', 1024, 16, 2), ('spinless8x8', 2048, 30, 0)])
def test_full_size_step_stays_in_bounds(chk, workload, D, l, keep):
    mdmrg, L = chk
    ctx, n = _context(mdmrg, L, workload, D, keep)
    n0 = L.mdmrg_check_launches()
    for prec in (mdmrg.FP64, mdmrg.FP32, mdmrg.BF16X3, mdmrg.BF16X6):
        _step(mdmrg, L, ctx, l, D, [mdmrg.FP64, prec])
        l += 1
    assert L.mdmrg_check_launches() - n0 > 100
    ctx.close()


def test_largest_workload_fits_one_gpu(chk):
    """8x8 rotated spinless, D=4096, middle bond, keep-envs 3 (one step to
    the right): environment build, products in all forms, one step."""
    mdmrg, L = chk
    ctx, n = _context(mdmrg, L, 'spinless8x8', 4096, 3)
    ne = _step(mdmrg, L, ctx, n // 2 - 1, 4096, [mdmrg.FP64, mdmrg.FP32, mdmrg.BF16X3, mdmrg.BF16X6, mdmrg.FP64])
    peak = L.mdmrg_check_peak_bytes()
    print(f'|psi| {ne}, peak device memory {peak / 1e9:.1f} GB')
    assert ne > 10_000_000
    assert peak < 265e9
    ctx.close()


def test_short_buffer_is_caught(chk):
    mdmrg, L = chk
    ctx, n = _context(mdmrg, L, 'hubbard6x6', 256, 1)
    ctx.prepare_bond(n // 2 - 1)
    _, ne = ctx.psi_layout()
    x = L.mdmrg_check_alloc(8 * ne)
    y = L.mdmrg_check_alloc(8 * ne - 8)  # one element short
    st = ctx.lib.mdmrg_heff_apply(ctx.h, mdmrg.FP64, ctypes.c_void_p(x), ctypes.c_void_p(y))
    assert st == mdmrg.EDEVICE
    assert 'range check' in ctx.lib.mdmrg_last_error(ctx.h).decode()
    ctx.close()


def test_failed_renormalisation_leaves_no_current_bond(chk):
    """A renormalisation that runs out of device memory (budget set just
    above what the context holds) reports ENOMEM; products are then refused
    with ESTATE instead of running on the released plans, and the context
    recovers with prepare_bond once memory is available."""
    mdmrg, L = chk
    ctx, n = _context(mdmrg, L, 'hubbard6x6', 256, 0)
    l = n // 2 - 1
    ctx.prepare_bond(l)
    _, ne = ctx.psi_layout()
    x = L.mdmrg_check_alloc(8 * ne)
    y = L.mdmrg_check_alloc(8 * ne)
    assert ctx.lib.mdmrg_decimate(ctx.h, ctypes.c_void_p(x), 256, 1, None, None, None) == 0
    ctx.set_option(mdmrg.OPT_MEMORY_BUDGET, L.mdmrg_check_live_bytes() + 4096)
    st = ctx.lib.mdmrg_renormalize(ctx.h, 1, mdmrg.FP64)
    assert st == mdmrg.ENOMEM, ctx.lib.mdmrg_last_error(ctx.h)
    assert ctx.lib.mdmrg_heff_apply(ctx.h, mdmrg.FP64, ctypes.c_void_p(x), ctypes.c_void_p(y)) == mdmrg.ESTATE
    ctx.set_option(mdmrg.OPT_MEMORY_BUDGET, 0)
    ctx.prepare_bond(l)
    _, ne2 = ctx.psi_layout()
    assert ne2 == ne
    assert ctx.lib.mdmrg_heff_apply(ctx.h, mdmrg.FP64, ctypes.c_void_p(x), ctypes.c_void_p(y)) == 0
    ctx.close()
