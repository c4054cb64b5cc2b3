"""Throughput benchmark: batched forward dynamics on one MI355X.

One step = one pass of the whole hot path over one batch: qdd for every chain
by ABIA, JSIIA and CFA (three launches of the library's fused kernels on the
same stream). Inputs are generated once and stay resident in HBM; the timed
region holds only the library calls.

Prints one JSON line: throughput (solves per second over the three
algorithms), per-algorithm rates, the roofline of the dominant kernel (FP64
vector-ALU bound: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6
TFLOP/s) and the CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FD solves/sec at n=64 links, batch 64k (FP64); p99 latency at fixed load"
PEAK_FLOPS = {"f64": 78.6e12, "f32": 157.3e12}


def fma_per_solve(algo: str, n: int) -> float:
    """Multiply-adds one solve needs in the formulation the kernels implement
    (canonical joint frames, S = e3; scans counted at their serial work, the
    odd-even elimination at its n log n work; transcendental calls excluded)."""
    rnea = 162.0 * n                                    # poses, velocity/acceleration/force sweeps
    if algo == "abia":
        return rnea + 360.0 * n + 30.0 * n              # articulated inertias + p sweep, a/qdd sweep
    if algo == "jsiia":
        return rnea + 94.0 * n + 3.0 * n * n + n ** 3 / 6.0 + n * n   # composite inertia, M, Cholesky, solves
    if algo == "cfa":
        levels = int(math.ceil(math.log2(n))) if n > 1 else 0
        oee = 0.0
        for j in range(1, levels + 1):
            s = 2 ** (j - 1)
            oee += 20.0 * n + 575.0 * max(0, n - s)     # factor own D; E- and K-part of rows with neighbours
        return rnea + 480.0 * n + oee + 45.0 * n + 18.0 * n   # Phi/A/B assembly, OEE, final solve, CalcAcc
    raise ValueError(algo)


def cpu_baseline(rb, q, qd, tau, chains: int):
    import oracle
    from paper_1609_06779_amd import synth

    sub = rb.take(np.arange(chains))
    n = int(rb.n_links[0])
    idx = slice(0, chains * n)
    oracle.fd(sub.take(np.arange(min(64, chains))), q[: 64 * n], qd[: 64 * n], tau[: 64 * n])   # warm
    t0 = time.perf_counter()
    oracle.fd(sub, q[idx], qd[idx], tau[idx], threads=0)
    dt = time.perf_counter() - t0
    return {"value": chains / dt, "unit": "solves/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"first {chains} chains of the same workload (n={n}, FP64), plain CRBA + RNEA + "
                      f"Cholesky, all host threads, {dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--algos", default="abia,jsiia,cfa")
    ap.add_argument("--cpu-chains", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); chains are independent, so a "
              "multi-GPU run would shard the batch with no exchange. Nothing was run.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1609_06779_amd import fd, synth

    algos = [a for a in args.algos.split(",") if a]
    dev = torch.device("cuda:0")
    lengths = synth.uniform_lengths(args.batch, args.n)
    rb = synth.make_robots(lengths, cfg=2)
    q, qd, tau = synth.make_state(lengths, cfg=2)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    if args.dtype == "f32":
        rb = rb.astype_rounded(np.float32)
    print(f"[bench] workload uniform-n{args.n}-b{args.batch} {args.dtype}, algos {algos}", file=sys.stderr, flush=True)
    model = fd.Model(rb, args.dtype, device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
    outs = {a: torch.empty_like(tq) for a in algos}
    wss = {a: model.workspace(args.batch, a) for a in algos}
    stream = torch.cuda.current_stream()

    def step(events=None):
        for a in algos:
            if events is not None:
                events[a][0].record(stream)
            model.forward(tq, tqd, ttau, batch=args.batch, algo=a, out=outs[a], workspace=wss[a], stream=stream)
            if events is not None:
                events[a][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    ev = [{a: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for a in algos}
          for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(ev[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (host wall {wall:.3f} s)", file=sys.stderr,
          flush=True)
    per_algo = {}
    for a in algos:
        ms = float(np.mean([e[a][0].elapsed_time(e[a][1]) for e in ev]))
        fl = 2.0 * fma_per_solve(a, args.n) * args.batch
        per_algo[a] = {"ms_per_launch": ms, "solves_per_s": args.batch / (ms * 1e-3),
                       "tflops": fl / (ms * 1e-3) / 1e12}
    for a in algos:
        assert torch.isfinite(outs[a]).all().item(), f"{a} produced non-finite qdd"
    dominant = max(algos, key=lambda a: per_algo[a]["ms_per_launch"])
    ms_dom = per_algo[dominant]["ms_per_launch"]
    achieved = 2.0 * fma_per_solve(dominant, args.n) * args.batch / (ms_dom * 1e-3) / 1e12
    peak = PEAK_FLOPS[args.dtype] / 1e12
    result = {
        "metric": METRIC,
        "value": len(algos) * args.batch / (ms_step * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"uniform-n{args.n}-b{args.batch}", "batch": args.batch, "n_links": args.n,
                   "algos": algos, "solves_per_step": len(algos) * args.batch},
        "per_algo": per_algo,
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None},
    }
    if not args.no_cpu and args.dtype == "f64":
        result["cpu_baseline"] = cpu_baseline(rb, q, qd, tau, min(args.cpu_chains, args.batch))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
