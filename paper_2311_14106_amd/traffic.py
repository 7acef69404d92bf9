"""HBM traffic of the dominant grouped-GEMM kernel from rocprofv3 counters.

Three commands, run under ``rocprofv3 --pmc FETCH_SIZE`` and then, in a
separate run, ``--pmc WRITE_SIZE`` (one counter pass per run):

* ``python3 -m paper_2311_14106_amd.traffic copy`` launches a plain
  elementwise copy of 1 GiB three times.  What the counters read for it,
  against the 1 GiB actually read and written, is the scale factor of each
  counter on this GPU.
* ``python3 -m paper_2311_14106_amd.traffic summarize CSV OUT [--windows
  JSON]`` reduces a counter_collection.csv to per-kernel sums and, for each
  entry {kernel: [LO, HI]} of JSON, to the sum over that kernel's dispatches
  LO..HI-1 in dispatch order (bench.py prints these windows for its timed
  steps, one per kernel name).
* ``python3 -m paper_2311_14106_amd.traffic record ...`` combines the four
  summaries into the text record that bench.py reads back: HBM bytes per
  launch of the kernel, tied to a digest of the kernel and planner sources so
  that a changed kernel reports no traffic until it is measured again.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ('paper_2311_14106_amd/csrc/device.hip', 'paper_2311_14106_amd/csrc/engine.cpp')
COPY_BYTES = 1 << 30


def sources_digest(root=ROOT):
    h = hashlib.sha256()
    for p in SOURCES:
        with open(os.path.join(root, p), 'rb') as f:
            h.update(f.read())
    return h.hexdigest()


def copy_kernel():
    import torch
    n = COPY_BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device='cuda')
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)   # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    print(f'copy: 3 launches of {COPY_BYTES} B read + {COPY_BYTES} B written', flush=True)


def summarize(path, windows=None):
    per = collections.defaultdict(lambda: [set(), 0.0])
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r['Dispatch_Id']), r['Kernel_Name'], r['Counter_Name'], float(r['Counter_Value'])))
    rows.sort()
    for d, k, c, v in rows:
        e = per[(k, c)]
        e[0].add(d)
        e[1] += v
    res = {'file': os.path.basename(path),
           'kernels': sorted(({'kernel': k[:120], 'counter': c, 'dispatches': len(ds), 'sum_kib': s}
                              for (k, c), (ds, s) in per.items()), key=lambda x: -x['sum_kib'])[:12]}
    if windows:
        res['windows'] = {}
        tot_n, tot_s = 0, 0.0
        for name, (lo, hi) in windows.items():
            # kernel names print as 'void mdmrg::<name>(...)'
            pat = re.compile(r'mdmrg::' + re.escape(name) + r'\(')
            disp = collections.OrderedDict()
            for d, k, c, v in rows:
                if pat.search(k):
                    disp[d] = disp.get(d, 0.0) + v
            sel = list(disp)[lo:hi]
            s = sum(disp[i] for i in sel)
            res['windows'][name] = {'window': [lo, hi], 'dispatches': len(sel), 'sum_kib': s,
                                    'kernel_dispatches': len(disp)}
            tot_n += len(sel)
            tot_s += s
        res['window_dispatches'] = tot_n
        res['window_sum_kib'] = tot_s
    return res


def record(args):
    def load(p):
        with open(p) as f:
            return json.load(f)
    fc, wc = load(args.fetch_copy), load(args.write_copy)
    fb, wb = load(args.fetch_bench), load(args.write_bench)

    def copy_kib(s):   # the elementwise copy kernel: largest counter sum over 3 dispatches
        top = max((k for k in s['kernels'] if 'elementwise' in k['kernel'] and 'Fill' not in k['kernel']),
                  key=lambda k: k['sum_kib'])
        return top['sum_kib'] / top['dispatches']
    f_scale = COPY_BYTES / (copy_kib(fc) * 1024.0)
    w_scale = COPY_BYTES / (copy_kib(wc) * 1024.0)
    n = fb['window_dispatches']
    assert n == wb['window_dispatches'] and n > 0
    fetch = fb['window_sum_kib'] * 1024.0 * f_scale / n
    write = wb['window_sum_kib'] * 1024.0 * w_scale / n
    rec = {'kernel_key': args.kernel_key, 'kernel': args.kernel_name, 'D': args.D,
           'sources_sha256': sources_digest(), 'window_dispatches': n,
           'fetch_scale': f_scale, 'write_scale': w_scale,
           'fetch_bytes_per_launch': fetch, 'write_bytes_per_launch': write,
           'hbm_bytes_per_launch': fetch + write}
    with open(args.out, 'w') as f:
        f.write(args.header.replace('\\n', '\n') + '\n\n' if args.header else '')
        f.write(json.dumps(rec, indent=1) + '\n')
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest='cmd', required=True)
    sub.add_parser('copy')
    s = sub.add_parser('summarize')
    s.add_argument('csv')
    s.add_argument('out')
    s.add_argument('--windows', type=json.loads, default=None)
    r = sub.add_parser('record')
    for a in ('fetch_copy', 'write_copy', 'fetch_bench', 'write_bench', 'out'):
        r.add_argument('--' + a.replace('_', '-'), dest=a, required=True)
    r.add_argument('--kernel-key', default='k_gemm<double> family')
    r.add_argument('--kernel-name',
                   default='k_gemm<double>, k_gemm_w16<double>, k_gemm_w4<double>, k_gemm_t128<double>')
    r.add_argument('--D', type=int, default=1024)
    r.add_argument('--header', default='')
    a = ap.parse_args()
    if a.cmd == 'copy':
        copy_kernel()
    elif a.cmd == 'summarize':
        res = summarize(a.csv, a.windows)
        with open(a.out, 'w') as f:
            json.dump(res, f, indent=1)
        print(json.dumps({k: v for k, v in res.items() if k != 'kernels'}))
    else:
        record(a)


if __name__ == '__main__':
    sys.exit(main())
