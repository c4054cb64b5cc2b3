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


def serving_leg(dtype: str, requests: int = 3000):
    """Continuous batching over 32 resident robots (n ~ U{7..200}), requests of
    1..4096 chains (log-uniform), Poisson arrivals at 50% and 80% of the
    measured saturation rate; latency is arrival to result in host memory."""
    import torch

    from paper_1609_06779_amd import fd, serve, synth

    dev = torch.device("cuda:0")
    lengths = synth.ragged_lengths(32, 7, 200, cfg=4)
    model = fd.Model(synth.make_robots(lengths, cfg=4), dtype, device=dev)
    ex = serve.GpuExecutor(model, lengths, algo="abia", streams=4)
    budget = 8 << 30

    def run(qps, count, seed):
        reqs = serve.make_requests(lengths, count, qps, seed=seed, dtype=dtype, shared=True)
        sched = serve.Scheduler(ex, budget, max_inflight=8, idle=serve.spin_idle)
        torch.cuda.synchronize()
        return sched.run(reqs), reqs

    run(float("inf"), 64, 1)                     # warm up allocator and kernels
    sat, reqs = run(float("inf"), requests // 2, 2)
    mean_chains = float(np.mean([r.chains for r in reqs]))
    out = {"robots": 32, "n_links": "U{7..200}", "chains_per_request": "log-uniform 1..4096",
           "budget_bytes": budget, "streams": 4, "saturation_solves_per_s": sat.solves_per_s,
           "saturation_launches": sat.launches}
    for load in (0.5, 0.8):
        qps = load * sat.solves_per_s / mean_chains
        st, _ = run(qps, requests, 3 + int(load * 10))
        out[f"load_{int(load * 100)}pct"] = {"qps": qps, "p50_ms": st.p50 * 1e3, "p99_ms": st.p99 * 1e3,
                                             "solves_per_s": st.solves_per_s, "launches": st.launches,
                                             "max_inflight": st.max_inflight}
    model.close()
    return out


def ragged_leg(dtype: str, batch: int = 100000, lo: int = 4, hi: int = 256, reps: int = 5):
    """100000 chains with n ~ U{4..256}, each its own robot: one persistent launch
    (grid from the autotuner's table) against a plain ragged launch and against
    one launch per distinct length."""
    import torch

    from paper_1609_06779_amd import fd, synth, tune

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    lengths = synth.ragged_lengths(batch, lo, hi, cfg=3)
    rb = synth.make_robots(lengths, cfg=3)
    q, qd, tau = synth.make_state(lengths, cfg=3)
    off = rb.offsets
    model = fd.Model(rb, dtype, device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
    toff = torch.from_numpy(off).to(dev)
    out = torch.empty_like(tq)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    grid = tune.ragged_grid(dtype)
    pws = model.persistent_workspace(batch, grid, offsets=toff)
    ms_pers = timed(lambda: model.forward_persistent(tq, tqd, ttau, batch=batch, grid=grid, offsets=toff, out=out,
                                                     workspace=pws, stream=stream))
    aws = model.workspace(batch, "abia", offsets=toff)
    ms_plain = timed(lambda: model.forward(tq, tqd, ttau, batch=batch, algo="abia", offsets=toff, out=out,
                                           workspace=aws, stream=stream))
    groups = []
    for n in np.unique(lengths):
        ids = np.nonzero(lengths == n)[0].astype(np.int32)
        groups.append((len(ids), torch.from_numpy(ids).to(dev), torch.from_numpy(off[ids]).to(dev),
                       model.workspace(len(ids), "abia", robot_id=torch.from_numpy(ids).to(dev))))

    def per_length():
        for cnt, rid, goff, ws in groups:
            model.forward(tq, tqd, ttau, batch=cnt, algo="abia", robot_id=rid, offsets=goff, out=out, workspace=ws,
                          stream=stream)

    ms_split = timed(per_length)
    model.close()
    return {"workload": f"ragged-b{batch}-n{lo}..{hi}", "links": int(lengths.sum()), "grid": grid,
            "persistent_ms": ms_pers, "persistent_solves_per_s": batch / (ms_pers * 1e-3),
            "plain_ragged_ms": ms_plain, "per_length_launches": len(groups), "per_length_ms": ms_split}


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
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
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
    if not args.no_ragged:
        print("[bench] ragged leg", file=sys.stderr, flush=True)
        result["ragged"] = ragged_leg(args.dtype)
    if not args.no_serve:
        print("[bench] serving leg", file=sys.stderr, flush=True)
        result["serving"] = serving_leg(args.dtype)
        l80 = result["serving"]["load_80pct"]
        result["p99_latency_ms_at_80pct_load"] = l80["p99_ms"]
    if not args.no_cpu and args.dtype == "f64":
        result["cpu_baseline"] = cpu_baseline(rb, q, qd, tau, min(args.cpu_chains, args.batch))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
