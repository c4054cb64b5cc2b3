"""Host-side tools, no GPU: the choice-table lookup and the profile summaries."""
import json
import os

import numpy as np
import pytest

import bench
from paper_1609_06779_amd import tune


def _bucket_reference(batch):
    # nearest power of two 2^k (k <= 20) in linear distance, ties to the lower one
    best = 0
    for k in range(21):
        if abs(batch - 2 ** k) < abs(batch - 2 ** best):
            best = k
    return best


@pytest.mark.parametrize("batch", [1, 2, 3, 5, 6, 7, 11, 12, 13, 100, 383, 384, 385, 65535, 65536, 98303,
                                   98305, 1 << 20, (1 << 20) + 1, 10 ** 7])
def test_batch_bucket_is_the_nearest_power_of_two(batch):
    assert tune.batch_bucket(batch) == _bucket_reference(batch)


def test_best_algo_follows_the_table(tmp_path):
    entry = {"n": [8, 64], "batch": [1, 65536], "algo": [["jsiia", "abia"], ["cfa", "abia"]]}
    path = tmp_path / "table.json"
    path.write_text(json.dumps({"best": {"f64": entry}}))
    assert tune.best_algo("f64", 5, 1, path=str(path)) == "jsiia"       # n rounds up to 8
    assert tune.best_algo("f64", 9, 2, path=str(path)) == "cfa"         # n rounds up to 64
    assert tune.best_algo("f64", 64, 70000, path=str(path)) == "abia"
    assert tune.best_algo("f32", 64, 1, path=str(path)) == "abia"       # no table for this precision
    arr = tune.table_array(entry)
    assert arr.shape == (257, 21) and arr[200, 0] == 2                  # past the grid: the last row


def _write_csv(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            f.write(",".join(f'"{v}"' if isinstance(v, str) else str(v) for v in r) + "\n")


def test_trace_and_counter_summaries(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1609_06779_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_1609_06779_amd" / "csrc" / "k.hip").write_text("// kernel\n")
    tr = tmp_path / "trace"
    tr.mkdir()
    _write_csv(tr / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                             "MaxNs", "StdDev"],
               [["void fdk::k_cfa<double, 64>(int)", 4, 4e6, 1e6, 60.0, 9e5, 1.1e6, 1.0],
                ["__amd_rocclr_copyBuffer", 3, 3e5, 1e5, 5.0, 1e5, 1e5, 0.0]])
    log = tmp_path / "trace.log"
    log.write_text('[bench] x\n' + json.dumps({"per_algo": {"cfa": {"ms_per_launch": 1.01}}}) + "\n")
    out = bench.summarize_trace(str(tr), "w", ["cmd"], "summary", str(log))
    text = open(out).read()
    assert "`fdk::k_cfa<double, 64>` | 4 | 1000.0" in text and "1010.0" in text and "copyBuffer" not in text
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    for sub, counter, copy_val, k_val in (("f", "FETCH_SIZE", 131072.0, 1000.0), ("w", "WRITE_SIZE", 262144.0, 500.0)):
        d = tmp_path / sub
        d.mkdir()
        _write_csv(d / "run_counter_collection.csv", hdr,
                   [[1, "__amd_rocclr_copyBuffer", counter, 0.5],                   # a small copy of torch's
                    [2, "__amd_rocclr_copyBuffer", counter, copy_val],
                    [3, "__amd_rocclr_copyBuffer", counter, copy_val],
                    [4, "__amd_rocclr_copyBuffer", counter, copy_val],
                    [5, "void fdk::k_cfa<double, 64>(int)", counter, k_val]])
    out = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "w", ["a", "b"], "summary")
    data = json.loads(open(out).read().split("```json\n")[1].split("\n```")[0])
    assert data["fetch_scale"] == pytest.approx(2.0) and data["write_scale"] == pytest.approx(1.0)
    assert data["kernels"]["cfa"]["bytes_per_launch"] == pytest.approx((1000.0 * 2 + 500.0) * 1024)
    assert bench.measured_traffic("cfa", "w") == pytest.approx((1000.0 * 2 + 500.0) * 1024)
    (tmp_path / "paper_1609_06779_amd" / "csrc" / "k.hip").write_text("// changed\n")
    assert bench.measured_traffic("cfa", "w") is None              # stale once the kernels change


def test_flops_summary_scales_the_wave_counter_by_64_lanes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void fdk::k_cfa<double, 64>(int)"
    for sub, rows in (("p1", [[1, k, "SQ_INSTS_VALU_FLOPS_FP64", 5e8]]),
                      ("p2", [[1, k, "SQ_INSTS_MFMA", 0], [1, k, "SQ_INSTS_VALU", 4e8],
                              [1, k, "SQ_INSTS_VALU_FMA_F64", 2e8], [1, k, "SQ_INSTS_VALU_MUL_F64", 6e7],
                              [1, k, "SQ_INSTS_VALU_ADD_F64", 4e7]]),
                      ("p3", [[1, k, "SQ_INSTS_LDS", 2e7], [1, k, "SQ_LDS_BANK_CONFLICT", 0],
                              [1, k, "SQ_WAVES", 65536]])):
        d = tmp_path / sub
        d.mkdir()
        _write_csv(d / "run_counter_collection.csv", hdr, rows)
    log = tmp_path / "bench.log"
    log.write_text(json.dumps({"per_algo": {"cfa": {"ms_per_launch": 1.0}}}) + "\n")
    out = bench.summarize_flops(str(tmp_path / "p1"), str(tmp_path / "p2"), "w", ["c"], "s", str(log), 64, 65536,
                                "f64", str(tmp_path / "p3"))
    row = next(ln for ln in open(out) if ln.startswith("| cfa | `"))
    cells = [c.strip() for c in row.split("|")[1:-1]]
    assert float(cells[2]) == pytest.approx(5e8 * 64 / 1e9)              # executed GFLOP per launch
    assert float(cells[5]) == pytest.approx(5e8 * 64 / 1e-3 / 1e12, rel=1e-3)   # TFLOP/s at 1 ms
    assert cells[7] == "0" and float(cells[8]) == pytest.approx(3e8 / 4e8)   # no MFMA; FP64 share
    lds = next(ln for ln in open(out) if ln.startswith("| cfa | 65536"))
    assert "| 305 |" in lds                                               # 2e7 / 65536 LDS instructions


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
