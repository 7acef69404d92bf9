"""Host logic of the measurement tools (no GPU): the counter summary and
traffic record of paper_2311_14106_amd.traffic on a synthetic
counter_collection.csv, and bench.py's refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csv(path, rows):
    with open(path, 'w', newline='') as f:
        w = csv.writer(f)
        w.writerow(['Dispatch_Id', 'Kernel_Name', 'Counter_Name', 'Counter_Value'])
        w.writerows(rows)


def test_traffic_summary_and_record(tmp_path):
    from paper_2311_14106_amd import traffic
    copy = 'void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<double>>(int)'
    # the copy kernel reads 1 GiB per launch, the counter reports half of it
    _csv(tmp_path / 'cf.csv', [(i, copy, 'FETCH_SIZE', 524288.0) for i in (1, 2, 3)])
    _csv(tmp_path / 'cw.csv', [(i, copy, 'WRITE_SIZE', 1048576.0) for i in (1, 2, 3)])
    names = ['void mdmrg::k_gemm<double>(a)', 'void mdmrg::k_gemm_w4<double>(a)', 'void mdmrg::k_gemm<float>(a)']
    rows_f = [(i, names[i % 3], 'FETCH_SIZE', 10.0 * i) for i in range(1, 31)]
    rows_w = [(i, names[i % 3], 'WRITE_SIZE', 1.0 * i) for i in range(1, 31)]
    _csv(tmp_path / 'bf.csv', rows_f)
    _csv(tmp_path / 'bw.csv', rows_w)
    windows = {'k_gemm<double>': [2, 5], 'k_gemm_w4<double>': [0, 2]}
    sf = traffic.summarize(str(tmp_path / 'bf.csv'), windows)
    # k_gemm<double> dispatches are i = 3, 6, ..., 30; window 2..4 -> 9, 12, 15
    assert sf['windows']['k_gemm<double>']['dispatches'] == 3
    assert sf['windows']['k_gemm<double>']['sum_kib'] == 10.0 * (9 + 12 + 15)
    # the FP32 kernel never matches the FP64 names
    assert sf['windows']['k_gemm_w4<double>']['sum_kib'] == 10.0 * (1 + 4)
    assert sf['window_dispatches'] == 5
    sw = traffic.summarize(str(tmp_path / 'bw.csv'), windows)
    for name, s in (('fc', traffic.summarize(str(tmp_path / 'cf.csv'))),
                    ('wc', traffic.summarize(str(tmp_path / 'cw.csv'))), ('fb', sf), ('wb', sw)):
        with open(tmp_path / f'{name}.json', 'w') as f:
            json.dump(s, f)
    out = tmp_path / 'rec.txt'
    r = subprocess.run([sys.executable, '-m', 'paper_2311_14106_amd.traffic', 'record',
                        '--fetch-copy', str(tmp_path / 'fc.json'), '--write-copy', str(tmp_path / 'wc.json'),
                        '--fetch-bench', str(tmp_path / 'fb.json'), '--write-bench', str(tmp_path / 'wb.json'),
                        '--out', str(out), '--header', 'test record'], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    txt = open(out).read()
    rec = json.loads(txt[txt.index('{'):txt.rindex('}') + 1])
    assert abs(rec['fetch_scale'] - 2.0) < 1e-12 and abs(rec['write_scale'] - 1.0) < 1e-12
    fetch_kib = 10.0 * (9 + 12 + 15 + 1 + 4)
    write_kib = 1.0 * (9 + 12 + 15 + 1 + 4)
    assert abs(rec['hbm_bytes_per_launch'] - (2.0 * fetch_kib + write_kib) * 1024 / 5) < 1e-6
    assert rec['sources_sha256'] == traffic.sources_digest()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], capture_output=True, text=True)
    assert r.returncode == 2
    assert 'one GPU' in r.stderr
