"""Autotuner for the forward-dynamics launch choices.

Times every algorithm on uniform batches over a grid of chain lengths and
batch sizes (HIP events on the launch stream, inputs resident in HBM) and
writes a JSON table: for each (precision, chain length, batch size) the
fastest algorithm. ``fd_forward(..., algo=AUTO)`` follows the table once it is
loaded with ``load_table`` (the binding calls it on first use when the cache
file exists). The same sweep reproduces the paper's two experiments: the time
of one call against the number of links and against the number of robots
(Sec. V).

    python -m paper_1609_06779_amd.tune --out paper_1609_06779_amd/tuning_gfx950.json
    python -m paper_1609_06779_amd.tune --experiments --dtypes f64 --out experiments.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning_gfx950.json")
ALGOS = ("abia", "jsiia", "cfa", "abia_scan")
CODES = {"abia": 0, "jsiia": 1, "cfa": 2, "abia_scan": 4, "cfa_proj": 5}   # fd_algo_t
NAMES = {v: k for k, v in CODES.items()}
N_GRID = (4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256)
BATCH_GRID = (1, 16, 256, 4096, 65536)


def time_forward(model, tq, tqd, ttau, batch, algo, reps=20, warmup=3):
    """Mean milliseconds of one fd_forward launch over ``reps`` back-to-back launches."""
    import torch

    out = torch.empty_like(tq)
    ws = model.workspace(batch, algo)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        model.forward(tq, tqd, ttau, batch=batch, algo=algo, out=out, workspace=ws, stream=stream)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        model.forward(tq, tqd, ttau, batch=batch, algo=algo, out=out, workspace=ws, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def sweep(ns=N_GRID, batches=BATCH_GRID, algos=ALGOS, dtype="f64", max_links_total=1 << 23, log=None):
    """Rows of {n, batch, algo, dtype, ms, solves_per_s} for every grid point that fits."""
    import torch

    from . import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rows = []
    for n in ns:
        bmax = max(b for b in batches if b * n <= max_links_total)
        lengths = synth.uniform_lengths(bmax, n)
        rb = synth.make_robots(lengths, cfg=2)
        q, qd, tau = synth.make_state(lengths, cfg=2)
        if dtype == "f32":
            rb = rb.astype_rounded(np.float32)
        model = fd.Model(rb, dtype, device=dev)
        tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
        for batch in batches:
            if batch > bmax:
                continue
            for algo in algos:
                if n > model.max_links(algo):
                    continue
                ms = time_forward(model, tq[: batch * n], tqd[: batch * n], ttau[: batch * n], batch, algo,
                                  reps=50 if batch <= 256 else 10)
                row = {"n": n, "batch": batch, "algo": algo, "dtype": dtype, "ms": ms,
                       "solves_per_s": batch / (ms * 1e-3)}
                rows.append(row)
                if log:
                    print(json.dumps(row), file=log, flush=True)
        model.close()
        del model, tq, tqd, ttau
        torch.cuda.empty_cache()
    return rows


def best_table(rows):
    """{dtype: {"n": [...], "batch": [...], "algo": [[...]]}}: fastest algorithm per grid point."""
    out = {}
    for dtype in sorted({r["dtype"] for r in rows}):
        sub = [r for r in rows if r["dtype"] == dtype]
        ns = sorted({r["n"] for r in sub})
        bs = sorted({r["batch"] for r in sub})
        grid = []
        for n in ns:
            line = []
            for b in bs:
                cand = [r for r in sub if r["n"] == n and r["batch"] == b]
                line.append(min(cand, key=lambda r: r["ms"])["algo"] if cand else None)
            grid.append(line)
        out[dtype] = {"n": ns, "batch": bs, "algo": grid}
    return out


def table_array(entry):
    """Dense [257][21] int8 array: best algorithm for chain length n and batch 2^k
    (nearest measured grid point, lengths rounded up, batches in log scale)."""
    ns = entry["n"]
    bs = entry["batch"]
    codes = {**CODES, None: 0}
    arr = np.zeros((257, 21), dtype=np.int8)
    for n in range(1, 257):
        i = next((k for k, v in enumerate(ns) if v >= n), len(ns) - 1)
        for k in range(21):
            b = 2 ** k
            j = int(np.argmin([abs(math.log2(x) - math.log2(b)) for x in bs]))
            arr[n, k] = codes[entry["algo"][i][j]]
    return arr


_TABLES = {}


def best_algo(dtype: str, n: int, batch: int, path=DEFAULT_TABLE) -> str:
    """The algorithm the tuned table picks for ``batch`` chains of ``n`` links (the
    library's AUTO rule on the same table); "abia" when there is no table."""
    key = (path, dtype)
    if key not in _TABLES:
        entry = json.load(open(path)).get("best", {}).get(dtype) if os.path.exists(path) else None
        _TABLES[key] = None if entry is None else table_array(entry)
    arr = _TABLES[key]
    if arr is None:
        return "abia"
    return NAMES[int(arr[min(256, max(1, n)), batch_bucket(batch)])]


def batch_bucket(batch: int) -> int:
    """Column of the choice table for a batch: the nearest power of two 2^k, k <= 20
    (the same rule as the library's AUTO lookup)."""
    k = 0
    while k < 20 and (1 << (k + 1)) <= batch:
        k += 1
    if k < 20 and batch - (1 << k) > (1 << (k + 1)) - batch:
        k += 1
    return k


def ragged_grid(dtype: str, path=DEFAULT_TABLE) -> int:
    """Persistent grid size for ragged batches chosen by ``tune_ragged`` (0 = resident capacity)."""
    if not os.path.exists(path):
        return 0
    return int(json.load(open(path)).get("ragged_grid", {}).get(dtype, 0))


def tune_ragged(dtype: str = "f64", batch: int = 100000, lo: int = 4, hi: int = 256, reps: int = 5, log=None):
    """Time the persistent launch over grid sizes (multiples of the CU count) on a
    ragged batch like the ragged workload and return {grid: ms}."""
    import torch

    from . import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    lengths = synth.ragged_lengths(batch, lo, hi, cfg=3)
    rb = synth.make_robots(lengths, cfg=3)
    q, qd, tau = synth.make_state(lengths, cfg=3)
    model = fd.Model(rb, dtype, device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
    toff = torch.from_numpy(rb.offsets).to(dev)
    out = torch.empty_like(tq)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = {}
    for per_cu in (1, 2, 3, 4, 6, 8, 12, 16):
        grid = cus * per_cu
        ws = model.persistent_workspace(batch, grid, offsets=toff)
        model.forward_persistent(tq, tqd, ttau, batch=batch, grid=grid, offsets=toff, out=out, workspace=ws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            model.forward_persistent(tq, tqd, ttau, batch=batch, grid=grid, offsets=toff, out=out, workspace=ws)
        b.record()
        torch.cuda.synchronize()
        res[grid] = a.elapsed_time(b) / reps
        if log:
            print(json.dumps({"ragged_grid": grid, "dtype": dtype, "ms": res[grid]}), file=log, flush=True)
    model.close()
    return res


EXP1_N = (2, 4, 8, 16, 32, 64, 96, 128, 160, 200, 256)
EXP2_N = (10, 200)
EXP2_GROUPS = (1, 10, 100, 1000, 10000, 100000)


def _time_calls(model, tq, tqd, ttau, n, batch, algo, calls):
    """(ms per call, ms on the device per call) of fd_forward over ``calls``
    back-to-back calls, each on its own slice of pre-drawn random inputs. The
    first is the paper's measure (launch overhead included: the binding and the
    launch); the second brackets each launch with its own pair of HIP events
    behind a spin kernel of about 0.2 ms, which keeps the GPU busy while the
    host issues the events and the call, so the pair times the kernel alone."""
    import torch

    out = torch.empty(batch * n, dtype=tq.dtype, device=tq.device)
    ws = model.workspace(batch, algo)
    stream = torch.cuda.current_stream()
    per = batch * n
    slices = max(1, tq.numel() // per)
    # the inputs of each call as views made before the timing (a view costs
    # microseconds of Python, which is the harness's work, not the call's)
    views = [(tq[o:o + per], tqd[o:o + per], ttau[o:o + per]) for o in range(0, slices * per, per)]

    def call(k):
        a, b, c = views[k % slices]
        model.forward(a, b, c, batch=batch, algo=algo, out=out, workspace=ws, stream=stream)

    for k in range(3):
        call(k)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for k in range(calls):
        call(k)
    b.record(stream)
    torch.cuda.synchronize()
    wall = a.elapsed_time(b) / calls
    reps = min(calls, 50)
    a.record(stream)
    torch.cuda._sleep(100000)
    b.record(stream)
    torch.cuda.synchronize()
    cycles = max(1000, int(100000 * 0.2 / max(a.elapsed_time(b), 1e-6)))   # about 0.2 ms of spinning
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for k in range(reps):
        torch.cuda._sleep(cycles)
        ev[k][0].record(stream)
        call(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    return wall, float(np.median([x.elapsed_time(y) for x, y in ev]))


def experiments(dtype="f64", calls=1000, log=None):
    """The paper's two experiments (Sec. V) on this GPU: the time of one call for one
    robot against its number of links, and the time of one call over a group of
    independent robots of 10 and of 200 links against the group size. Each robot
    has its own random parameters; each call gets its own random joint inputs."""
    import torch

    from . import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rows = []

    def run(n, batch, exp, reps):
        lengths = synth.uniform_lengths(batch, n)
        rb = synth.make_robots(lengths, cfg=6)
        slices = max(1, min(reps, (1 << 22) // (batch * n)))      # distinct inputs, at most 4M entries
        q, qd, tau = synth.make_state(synth.uniform_lengths(batch * slices, n), cfg=6)
        model = fd.Model(rb, dtype, device=dev)
        tq, tqd, ttau = (torch.from_numpy(x).to(dev, tdt) for x in (q, qd, tau))
        for algo in ALGOS:
            row = {"exp": exp, "n": n, "groups": batch, "algo": algo, "dtype": dtype}
            if n > model.max_links(algo):
                row["ms"] = row["device_ms"] = None                 # longer than this algorithm's kernels take
            else:
                row["ms"], row["device_ms"] = _time_calls(model, tq, tqd, ttau, n, batch, algo, reps)
            rows.append(row)
            if log:
                print(json.dumps(row), file=log, flush=True)
        model.close()

    for n in EXP1_N:
        run(n, 1, 1, calls)
    for n in EXP2_N:
        for g in EXP2_GROUPS:
            run(n, g, 2, calls if g * n <= 100000 else max(10, calls * 100000 // (g * n)))
    return rows


def load_table(path=DEFAULT_TABLE):
    """Hand the tuned table to the library (per precision). Returns False if there is none."""
    if not os.path.exists(path):
        return False
    import ctypes

    from . import _lib

    data = json.load(open(path))
    lib = _lib.load()
    for dtype, entry in data.get("best", {}).items():
        arr = np.ascontiguousarray(table_array(entry))
        _lib.check(lib.fd_set_auto_table(_lib.DTYPES[dtype], arr.ctypes.data_as(ctypes.c_void_p)),
                   "fd_set_auto_table")
    for dtype, grid in data.get("ragged_grid", {}).items():
        _lib.check(lib.fd_set_persistent_grid(_lib.DTYPES[dtype], int(grid)), "fd_set_persistent_grid")
    return True


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--dtypes", default="f64,f32")
    ap.add_argument("--ns", default=",".join(map(str, N_GRID)))
    ap.add_argument("--batches", default=",".join(map(str, BATCH_GRID)))
    ap.add_argument("--ragged-only", action="store_true", help="keep the existing sweep, redo the ragged grid")
    ap.add_argument("--experiments", action="store_true",
                    help="run the paper's two experiment shapes instead and write them to --out")
    args = ap.parse_args()
    import torch

    if args.experiments:
        rows = []
        for dtype in args.dtypes.split(","):
            rows += experiments(dtype, log=sys.stderr)
        with open(args.out, "w") as f:
            json.dump({"arch": torch.cuda.get_device_properties(0).gcnArchName, "rows": rows}, f, indent=1)
        return

    if args.ragged_only and os.path.exists(args.out):
        data = json.load(open(args.out))
    else:
        rows = []
        for dtype in args.dtypes.split(","):
            rows += sweep(tuple(int(x) for x in args.ns.split(",")), tuple(int(x) for x in args.batches.split(",")),
                          dtype=dtype, log=sys.stderr)
        data = {"arch": torch.cuda.get_device_properties(0).gcnArchName, "rows": rows, "best": best_table(rows)}
    data["ragged_timings"] = {}
    data["ragged_grid"] = {}
    for dtype in args.dtypes.split(","):
        res = tune_ragged(dtype, log=sys.stderr)
        data["ragged_timings"][dtype] = {str(k): v for k, v in res.items()}
        data["ragged_grid"][dtype] = int(min(res, key=res.get))
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(data["best"]))


if __name__ == "__main__":
    main()
