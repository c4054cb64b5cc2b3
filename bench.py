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
import collections
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
    if algo in ("abia", "abia_scan"):                  # the scan form does the same method's work
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


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_06779_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, if the
    kernel sources are unchanged since it was taken (else None)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    import re

    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    data = json.loads(m.group(1))
    if data.get("source_hash") != kernel_source_hash():
        return None
    k = data.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


KERNEL_PATTERNS = (("abia", r"k_abia<"), ("jsiia", r"k_jsiia"), ("cfa", r"k_cfa<"),
                   ("abia_persistent", r"k_abia_persistent<"), ("abia_scan", r"k_abia_scan<"))
COPY_CALIB_BYTES = 256 << 20


def summarize_pmc(fetch_dir: str, write_dir: str, workload: str, commands, summary_cmd: str) -> str:
    """Write profiles/<workload>_hbm_traffic.md from two rocprofv3 --pmc runs of
    ``bench.py --copy-calib`` (one with FETCH_SIZE, one with WRITE_SIZE). Each
    kernel's counters are scaled by what the same counter reads for the device
    copy of known size in the same run."""
    import collections
    import csv
    import glob
    import re

    def load(d, counter):
        vals = collections.defaultdict(list)
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return vals

    def pick(vals, pat):
        for k, v in vals.items():
            if re.search(pat, k):
                return sum(v) / len(v), len(v), k
        return None

    def calib(vals):
        # the calibration copies are the largest copy dispatches of the run (torch
        # issues small copies of its own)
        v = [x for k, xs in vals.items() if "copyBuffer" in k for x in xs]
        if not v:
            return None
        top = sorted(v)[-3:]
        return sum(top) / len(top), len(top), "copyBuffer"

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    cf, cw = calib(fe), calib(wr)
    if cf is None or cw is None:
        raise SystemExit("no copy kernel in the counter runs (run bench.py with --copy-calib)")
    ffac, wfac = COPY_CALIB_BYTES / 1024 / cf[0], COPY_CALIB_BYTES / 1024 / cw[0]
    out = {"source_hash": kernel_source_hash(), "copy_bytes": COPY_CALIB_BYTES, "copy_fetch_kib": cf[0],
           "copy_write_kib": cw[0], "fetch_scale": ffac, "write_scale": wfac, "kernels": {}}
    for algo, pat in KERNEL_PATTERNS:
        f, w = pick(fe, pat), pick(wr, pat)
        if f and w:
            out["kernels"][algo] = {"kernel": f[2].split("(")[0].replace("void ", ""), "dispatches": f[1],
                                    "fetch_kib": f[0],
                                    "write_kib": w[0], "bytes_per_launch": (f[0] * ffac + w[0] * wfac) * 1024}
    mib = COPY_CALIB_BYTES >> 20
    lines = [f"# HBM traffic per launch: {workload}", "",
             "Two counter passes (one counter each) of the same program, then this summary:", "", "```",
             *commands, summary_cmd, "```",
             "", f"Calibration: a {mib} MiB device copy (`__amd_rocclr_copyBuffer`) in the same run reads "
             f"FETCH_SIZE {cf[0]:.0f} KiB and WRITE_SIZE {cw[0]:.0f} KiB for {COPY_CALIB_BYTES >> 10} KiB moved "
             f"each way; kernel counters are scaled by {ffac:.3f} (fetch) and {wfac:.3f} (write).", "",
             "| algorithm | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes / launch |",
             "|---|---|---|---|---|---|"]
    for a, k in out["kernels"].items():
        lines.append(f"| {a} | `{k['kernel']}` | {k['dispatches']} | {k['fetch_kib']:.0f} | {k['write_kib']:.0f} "
                     f"| {k['bytes_per_launch']:.3e} |")
    lines += ["", "Machine-readable (bench.py reads `bytes_per_launch` while `source_hash` matches the kernel "
              "sources):", "", "```json", json.dumps(out, indent=1), "```"]
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def summarize_flops(p1_dir: str, p2_dir: str, workload: str, commands, summary_cmd: str, bench_log: str,
                    n: int, batch: int, dtype: str, p3_dir=None) -> str:
    """Write profiles/<workload>_valu_flops.md from two rocprofv3 --pmc passes:
    SQ_INSTS_VALU_FLOPS_FP64 (FP32: _FP32; flops per wave instruction: 2 per FMA,
    1 per add or multiply), then SQ_INSTS_MFMA, SQ_INSTS_VALU and the FMA / MUL /
    ADD counts of that precision. Executed flops per launch = the flops counter x
    64 lanes (masked lanes included); the time per launch is bench.py's HIP-event
    average from `bench_log` (an unprofiled or trace-only run of the same step).
    An optional third pass (SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT, SQ_WAVES) adds the
    LDS instructions per wave and the bank-conflict cycles per LDS instruction."""
    import csv
    import glob
    import re

    def load(d):
        vals = collections.defaultdict(lambda: collections.defaultdict(list))
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return vals

    c1, c2 = load(p1_dir), load(p2_dir)
    c3 = load(p3_dir) if p3_dir else {}
    events = {}
    for line in open(bench_log):
        if line.startswith("{"):
            events = {a: v["ms_per_launch"] for a, v in json.loads(line).get("per_algo", {}).items()}
    peak = PEAK_FLOPS[dtype] / 1e12
    P = "FP64" if dtype == "f64" else "FP32"
    sfx = "F64" if dtype == "f64" else "F32"
    lds_rows = []
    lines = [f"# {P} VALU work per launch: {workload}", "", "Commands:", "", "```", *commands, summary_cmd, "```", "",
             f"Executed flops = `SQ_INSTS_VALU_FLOPS_{P}` x 64 lanes (it counts 2 per FMA and 1 per add or "
             "multiply, per wave instruction, so masked lanes are included). The algorithmic count is "
             "bench.py's `fma_per_solve` x 2 x batch. Times: the HIP-event average per launch of the "
             "bench log named above (a bench.py run of the same workload, unprofiled or under the kernel "
             "trace only).", "",
             "| algorithm | kernel | executed GFLOP / launch | algorithmic GFLOP / launch | ms / launch | "
             f"executed TFLOP/s | frac of peak | MFMA instructions | {P} share of VALU instructions |",
             "|---|---|---|---|---|---|---|---|---|"]
    for algo, pat in KERNEL_PATTERNS:
        k1 = next((k for k in c1 if re.search(pat, k)), None)
        k2 = next((k for k in c2 if re.search(pat, k)), None)
        if not k1 or not k2 or algo not in events:
            continue
        mean = lambda d, c: sum(d[c]) / len(d[c])
        ex = mean(c1[k1], f"SQ_INSTS_VALU_FLOPS_{P}") * 64
        alg = 2.0 * fma_per_solve(algo, n) * batch
        ms = events[algo]
        f64 = sum(mean(c2[k2], c) for c in (f"SQ_INSTS_VALU_FMA_{sfx}", f"SQ_INSTS_VALU_MUL_{sfx}",
                                             f"SQ_INSTS_VALU_ADD_{sfx}"))
        rate = ex / (ms * 1e-3) / 1e12
        lines.append(f"| {algo} | `{k1.split('(')[0].replace('void ', '')}` | {ex / 1e9:.2f} | {alg / 1e9:.2f} | "
                     f"{ms:.3f} | {rate:.1f} | {rate / peak:.2f} | {mean(c2[k2], 'SQ_INSTS_MFMA'):.0f} | "
                     f"{f64 / mean(c2[k2], 'SQ_INSTS_VALU'):.2f} |")
        k3 = next((k for k in c3 if re.search(pat, k)), None)
        if k3:
            waves = mean(c3[k3], "SQ_WAVES")
            lds = mean(c3[k3], "SQ_INSTS_LDS")
            lds_rows.append(f"| {algo} | {waves:.0f} | {lds / waves:.0f} | {mean(c2[k2], 'SQ_INSTS_VALU') / waves:.0f} | "
                            f"{mean(c3[k3], 'SQ_LDS_BANK_CONFLICT') / max(lds, 1.0):.2f} |")
    if lds_rows:
        lines += ["", "LDS use (third pass; counters per launch, divided by the waves of the launch):", "",
                  "| algorithm | waves | LDS instructions / wave | VALU instructions / wave | "
                  "bank-conflict cycles / LDS instruction |", "|---|---|---|---|---|", *lds_rows]
    path = os.path.join(ROOT, "profiles", f"{workload}_valu_flops.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def summarize_trace(trace_dir: str, workload: str, commands, summary_cmd: str, bench_log=None) -> str:
    """Write profiles/<workload>_kernel_trace.md from a rocprofv3 --kernel-trace --stats run;
    with ``bench_log`` (the profiled bench.py's output) its own HIP-event averages go beside."""
    import csv
    import glob
    import re

    events = {}
    if bench_log:
        for line in open(bench_log):
            if line.startswith("{"):
                rec = json.loads(line)
                events = {a: v["ms_per_launch"] * 1e3 for a, v in rec.get("per_algo", {}).items()}
                trees = rec.get("trees", {})
                if not events and len(trees) == 1:      # a run of one tree workload alone
                    events = {a: v["ms_per_launch"] * 1e3 for a, v in next(iter(trees.values())).items()
                              if isinstance(v, dict)}

    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {trace_dir}")
    rows = list(csv.DictReader(open(files[0])))
    lines = [f"# Kernel trace: {workload}", "", "Commands:", "", "```", *commands, summary_cmd, "```", "",
             "`--stats` summary of the library's kernels (times in microseconds). The last column is "
             "bench.py's own HIP-event average per launch in the same profiled run (back-to-back "
             "launches; the trace times each dispatch on its own):", "",
             "| kernel | calls | average | min | max | share of GPU time | bench.py events |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("void ", "")
        if "fdk::" not in name:
            continue
        algo = next((a for a, pat in KERNEL_PATTERNS if re.search(pat, name)), None)
        ev = f"{events[algo]:.1f}" if algo in events else "-"
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} "
                     f"| {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% | {ev} |")
    path = os.path.join(ROOT, "profiles", f"{workload}_kernel_trace.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def cpu_baseline(rb, q, qd, tau, chains: int, min_s: float = 10.0, max_s: float = 30.0):
    import oracle
    from paper_1609_06779_amd import synth

    sub = rb.take(np.arange(chains))
    n = int(rb.n_links[0])
    idx = slice(0, chains * n)
    oracle.fd(sub.take(np.arange(min(64, chains))), q[: 64 * n], qd[: 64 * n], tau[: 64 * n])   # warm
    # whole passes over the sample until at least min_s seconds of CPU work (at most max_s)
    passes, t0 = 0, time.perf_counter()
    while True:
        oracle.fd(sub, q[idx], qd[idx], tau[idx], threads=0)
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or dt * (passes + 1) / passes > max_s:
            break
    cores = oracle.max_threads()
    one = min(chains, 4096)                     # one host thread, a smaller slice of the same chains
    sl = slice(0, one * n)
    t1 = time.perf_counter()
    oracle.fd(sub.take(np.arange(one)), q[sl], qd[sl], tau[sl], threads=1)
    dt1 = time.perf_counter() - t1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": passes * chains / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu": model, "host_cpus": os.cpu_count(), "single_thread_value": one / dt1,
            "sample": f"{passes} passes over the first {chains} chains of the same workload (n={n}, FP64), "
                      f"plain CRBA + RNEA + Cholesky, all host threads, {dt:.1f} s wall; single thread: "
                      f"the first {one} chains, {dt1:.1f} s"}


ACCURACY_TARGET = {"f64": 1e-10, "f32": 1e-4}
ACCURACY_CAP = {"f64": 1e-9, "f32": 1e-3}


def cpu_baseline_accuracy(ns=(16, 32, 64, 128), batch: int = 65536, sample: int = 8192, eta_sample: int = 512):
    """Part of the CPU-baseline leg: the oracle's reference q-ddot (evaluated in
    long double, so that its own rounding is not counted) on a sample of
    each uniform 65536-chain workload (n = 16..128; the first `sample` chains),
    FP64 and FP32 (robots and states rounded to FP32 first, the oracle in FP64 on
    the rounded values), against the library's q-ddot for the whole batch.
    Per (dtype, n, algorithm): max, p99 and median per-chain relative error
    ||qdd - qdd_ref|| / ||qdd_ref||, the fraction of chains within the target
    (1e-10 FP64, 1e-4 FP32) and within the parity tests' cap (10x the target),
    and the largest normwise backward error ||M qdd - tau_delta|| /
    (||M|| ||qdd|| + ||tau|| + ||tau_bias||) over the first `eta_sample` chains,
    in units of the precision's unit roundoff."""
    import torch

    import oracle
    from paper_1609_06779_amd import fd, synth

    dev = torch.device("cuda:0")
    u = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}
    out = {"chains_checked": sample, "batch": batch, "target": ACCURACY_TARGET, "cap": ACCURACY_CAP}
    for dtype in ("f64", "f32"):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        out[dtype] = {}
        for n in ns:
            lengths = synth.uniform_lengths(batch, n)
            rb = synth.make_robots(lengths, cfg=2)
            q, qd, tau = synth.make_state(lengths, cfg=2)
            if dtype == "f32":
                rb = rb.astype_rounded(np.float32)
                q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in (q, qd, tau))
            sub = rb.take(np.arange(sample))
            sl = slice(0, sample * n)
            ref = oracle.fd_exact(sub, q[sl], qd[sl], tau[sl], threads=0)   # the oracle in long double
            es = slice(0, eta_sample * n)
            esub = rb.take(np.arange(eta_sample))
            ms = oracle.crba(esub, q[es], threads=0)
            bias = oracle.rnea(esub, q[es], qd[es], threads=0)
            mnorm = np.array([np.linalg.norm(m, 2) for m in ms])
            model = fd.Model(rb, dtype, device=dev)
            tq, tqd, tt = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
            cell = {}
            for algo in ("abia", "jsiia", "cfa", "abia_scan"):
                if n > model.max_links(algo):
                    continue
                got = model.forward(tq, tqd, tt, batch=batch, algo=algo)[: sample * n].cpu().numpy().astype(np.float64)
                err = oracle.relative_error(got, ref, sub.offsets)
                eta = [np.linalg.norm(ms[b] @ got[b * n:(b + 1) * n] - (tau[b * n:(b + 1) * n] - bias[b * n:(b + 1) * n]))
                       / (mnorm[b] * np.linalg.norm(got[b * n:(b + 1) * n]) + np.linalg.norm(tau[b * n:(b + 1) * n])
                          + np.linalg.norm(bias[b * n:(b + 1) * n])) for b in range(eta_sample)]
                cell[algo] = {"max": float(err.max()), "p99": float(np.quantile(err, 0.99)),
                              "median": float(np.median(err)),
                              "within_target": float(np.mean(err <= ACCURACY_TARGET[dtype])),
                              "within_cap": float(np.mean(err <= ACCURACY_CAP[dtype])),
                              "backward_error_max_u": float(np.max(eta) / u[dtype])}
            out[dtype][str(n)] = cell
            model.close()
            del tq, tqd, tt
            torch.cuda.empty_cache()
    return out


def serving_leg(dtype: str, requests: int = 30000):
    """Continuous batching over 32 resident robots (n ~ U{7..200}), requests of
    1..4096 chains (log-uniform), Poisson arrivals at 50%, 70% and 80% of the
    saturation rate (all requests present at once) and at the fixed rates of
    5000 and 10000 requests/s; latency is arrival to
    result in host memory. Each round's batch takes the library's AUTO choice.
    Saturation reports where the time goes (copies in, kernels, copies out:
    GPU time summed over launches, which overlap on the streams; and the host
    loop's own time) and, for reference, the plain per-batch launch on the same
    request mix: the same rounds of at most 65536 chains, state already in
    HBM, one AUTO launch each. 3e4 requests per point give about 300 samples
    past the 99th percentile."""
    import torch

    from paper_1609_06779_amd import fd, serve, synth

    dev = torch.device("cuda:0")
    lengths = synth.ragged_lengths(32, 7, 200, cfg=4)
    model = fd.Model(synth.make_robots(lengths, cfg=4), dtype, device=dev)
    budget = 8 << 30
    esz = 8 if dtype == "f64" else 4

    def run(qps, count, seed):
        ex = serve.GpuExecutor(model, lengths, algo="auto", streams=4, slots=8)
        reqs = serve.make_requests(lengths, count, qps, seed=seed, dtype=dtype, shared=True)
        sched = serve.Scheduler(ex, budget, max_inflight=8, idle=serve.spin_idle)
        torch.cuda.synchronize()
        return sched.run(reqs), reqs, ex

    run(float("inf"), 256, 1)                    # warm up allocator and kernels
    sat, reqs, ex = run(float("inf"), requests, 2)
    mean_chains = float(np.mean([r.chains for r in reqs]))
    algos = collections.Counter(r.algo for r in reqs)
    t = ex.timing
    moved = t["bytes_h2d"] + t["bytes_d2h"]
    out = {"robots": 32, "n_links": "U{7..200}", "chains_per_request": "log-uniform 1..4096",
           "algo": "AUTO per round (the whole round's batch)", "requests_per_load": requests,
           "budget_bytes": budget, "streams": 4, "slots": 8,
           "saturation_solves_per_s": sat.solves_per_s, "saturation_launches": sat.launches,
           "saturation_wall_s": sat.wall, "saturation_algo_mix": dict(algos),
           "breakdown": {"h2d_ms": t["h2d_ms"], "kernel_ms": t["kernel_ms"], "d2h_ms": t["d2h_ms"],
                         "host_launch_ms": t["host_launch_s"] * 1e3, "wall_ms": sat.wall * 1e3,
                         "bytes_over_pcie": moved, "pcie_gb_per_s": moved / sat.wall / 1e9,
                         "persistent_launches": t["persistent_launches"]}}
    # the plain per-batch launch on the same mix: the same packing, inputs resident in HBM
    rounds, cur = [], []
    for r in reqs:
        if cur and sum(x.chains for x in cur) + r.chains > 65536:
            rounds.append(cur)
            cur = []
        cur.append(r)
    if cur:
        rounds.append(cur)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    stream = torch.cuda.current_stream()
    ms_plain, chains_plain = 0.0, 0
    for grp in rounds:
        sizes = np.array([r.chains for r in grp])
        ns = np.array([r.n for r in grp])
        chains, links = int(sizes.sum()), int((sizes * ns).sum())
        rid = torch.from_numpy(np.repeat([r.robot for r in grp], sizes).astype(np.int32)).to(dev)
        first_chain = np.repeat(np.cumsum(sizes) - sizes, sizes)
        first_link = np.repeat(np.cumsum(sizes * ns) - sizes * ns, sizes)
        off_np = np.append(first_link + (np.arange(chains) - first_chain) * np.repeat(ns, sizes), links)
        off = torch.from_numpy(off_np.astype(np.int64)).to(dev)
        gen = torch.Generator(device=dev).manual_seed(len(grp))
        q = (torch.rand(links, generator=gen, device=dev, dtype=tdt) * 2 - 1) * math.pi
        qd = torch.rand(links, generator=gen, device=dev, dtype=tdt) * 2 - 1
        tau = torch.randn(links, generator=gen, device=dev, dtype=tdt)
        nmax = int(ns.max())
        ws = model.workspace(chains, "auto", robot_id=rid, offsets=off, max_links=nmax)
        o = torch.empty_like(q)
        call = lambda: model.forward(q, qd, tau, batch=chains, algo="auto", robot_id=rid, offsets=off, out=o,
                                     workspace=ws, stream=stream, max_links=nmax)
        call()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call()
        b.record(stream)
        torch.cuda.synchronize()
        ms_plain += a.elapsed_time(b)
        chains_plain += chains
        del q, qd, tau, o, ws, rid, off
    out["plain_per_batch"] = {"rounds": len(rounds), "kernel_ms": ms_plain,
                              "solves_per_s": chains_plain / (ms_plain * 1e-3)}
    for load in (0.5, 0.7, 0.8):
        qps = load * sat.solves_per_s / mean_chains
        st, _, _ = run(qps, requests, 3 + int(load * 10))
        out[f"load_{int(load * 100)}pct"] = {"qps": qps, "p50_ms": st.p50 * 1e3, "p99_ms": st.p99 * 1e3,
                                             "solves_per_s": st.solves_per_s, "launches": st.launches,
                                             "max_inflight": st.max_inflight}
    # fixed request rates, comparable from one build to the next whatever the saturation rate
    for qps in (5000.0, 10000.0):
        st, _, _ = run(qps, requests, 20 + int(qps // 1000))
        out[f"qps_{int(qps)}"] = {"qps": qps, "p50_ms": st.p50 * 1e3, "p99_ms": st.p99 * 1e3,
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
    autows = model.workspace(batch, "auto", offsets=toff)
    ms_auto = timed(lambda: model.forward(tq, tqd, ttau, batch=batch, algo="auto", offsets=toff, out=out,
                                          workspace=autows, stream=stream))
    groups = []
    for n in np.unique(lengths):
        ids = np.nonzero(lengths == n)[0].astype(np.int32)
        # chain starts of this length's chains, plus the end of the last one
        starts = np.append(off[ids], off[ids[-1]] + n).astype(np.int64)
        rid, goff = torch.from_numpy(ids).to(dev), torch.from_numpy(starts).to(dev)
        groups.append((len(ids), rid, goff, model.workspace(len(ids), "abia", robot_id=rid, offsets=goff)))

    def per_length():
        for cnt, rid, goff, ws in groups:
            model.forward(tq, tqd, ttau, batch=cnt, algo="abia", robot_id=rid, offsets=goff, out=out, workspace=ws,
                          stream=stream)

    ms_split = timed(per_length)
    model.close()
    return {"workload": f"ragged-b{batch}-n{lo}..{hi}", "links": int(lengths.sum()), "grid": grid,
            "persistent_ms": ms_pers, "persistent_solves_per_s": batch / (ms_pers * 1e-3),
            "plain_ragged_ms": ms_plain, "auto_ms": ms_auto, "auto_choice": tune.best_algo(dtype, int(lengths.max()), batch),
            "per_length_launches": len(groups), "per_length_ms": ms_split}


def copy_calibration(dev):
    """Device copies of COPY_CALIB_BYTES: the known-size reference for the HBM counters."""
    import torch

    src = torch.empty(COPY_CALIB_BYTES, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def transfer_leg(dtype: str, reps: int = 10):
    """The headline batch (65536 chains of 64 links) with its state handed over in
    pinned host memory: copy q, qd, tau in, one ABIA launch, copy qdd out, all on
    one stream. The library itself takes device buffers; this is the rate a
    caller holding host arrays sees."""
    import torch

    from paper_1609_06779_amd import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    batch, n = 65536, 64
    lengths = synth.uniform_lengths(batch, n)
    rb = synth.make_robots(lengths, cfg=2)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
    q, qd, tau = synth.make_state(lengths, cfg=2)
    model = fd.Model(rb, dtype, device=dev)
    host = [torch.from_numpy(a).to(tdt).pin_memory() for a in (q, qd, tau)]
    hout = torch.empty(len(q), dtype=tdt).pin_memory()
    dq, dqd, dtau = (torch.empty(len(q), dtype=tdt, device=dev) for _ in range(3))
    out = torch.empty_like(dq)
    ws = model.workspace(batch, "abia")
    stream = torch.cuda.current_stream()

    def step():
        for d, h in zip((dq, dqd, dtau), host):
            d.copy_(h, non_blocking=True)
        model.forward(dq, dqd, dtau, batch=batch, algo="abia", out=out, workspace=ws, stream=stream)
        hout.copy_(out, non_blocking=True)

    step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    model.close()
    return {"workload": f"uniform-n{n}-b{batch}", "algo": "abia", "ms_per_batch": ms,
            "solves_per_s": batch / (ms * 1e-3), "bytes_over_pcie": 4 * len(q) * (8 if dtype == "f64" else 4)}


def nsweep_leg(dtypes=("f64", "f32"), ns=(16, 32, 64, 128), batch: int = 65536, reps: int = 10):
    """The three algorithms at `batch` chains of n links for each n, in FP64 and
    FP32 (the headline workload's generator; FP32 robots rounded to FP32): ms per
    launch and solves/s. JSIIA stops at its largest lane grid (128 links)."""
    import torch

    from paper_1609_06779_amd import fd, synth, tune

    dev = torch.device("cuda:0")
    out = {}
    for dtype in dtypes:
        tdt = torch.float64 if dtype == "f64" else torch.float32
        out[dtype] = {}
        for n in ns:
            lengths = synth.uniform_lengths(batch, n)
            rb = synth.make_robots(lengths, cfg=2)
            if dtype == "f32":
                rb = rb.astype_rounded(np.float32)
            q, qd, tau = synth.make_state(lengths, cfg=2)
            model = fd.Model(rb, dtype, device=dev)
            tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
            row = {}
            for algo in ("abia", "jsiia", "cfa"):
                if n > model.max_links(algo):
                    continue
                ms = tune.time_forward(model, tq, tqd, ttau, batch, algo, reps=reps)
                row[algo] = {"ms_per_launch": ms, "solves_per_s": batch / (ms * 1e-3)}
            out[dtype][str(n)] = row
            model.close()
            del tq, tqd, ttau
            torch.cuda.empty_cache()
    return out


def levels_leg(dtype: str, ns=(16, 32, 64, 128), batch: int = 65536, reps: int = 20):
    """The two building blocks on their own at `batch` systems of n blocks each:
    the segmented scan of block bi-diagonal 6x6 systems (fd_scan6) and the
    odd-even elimination solve of SPD block tri-diagonal 6x6 systems
    (fd_btd_solve6), both with ceil(log2 n) levels. Reports the launch time,
    the time per level (launch time / levels, loads and stores included) and
    the algorithmic HBM rate. Inputs: 1024 seeded systems tiled to the batch."""
    import torch

    from paper_1609_06779_amd import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    w = 8 if dtype == "f64" else 4
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {}
    rep = batch // 1024
    for n in ns:
        lengths = np.full(1024, n, np.int64)
        off = torch.from_numpy(synth.offsets_of(np.full(batch, n, np.int64))).to(dev)
        levels = max(1, math.ceil(math.log2(n)))
        sb, sc = synth.make_scan_elements(lengths)
        sb, sc = (torch.from_numpy(x).to(dev, tdt).repeat(rep, *([1] * (x.ndim - 1))) for x in (sb, sc))
        sx = torch.empty_like(sc)
        ms_scan = timed(lambda: fd.scan6(sb, sc, off, n, out=sx, stream=stream))
        d, u, r = synth.make_btd(lengths)
        d, u, r = (torch.from_numpy(x).to(dev, tdt).repeat(rep, *([1] * (x.ndim - 1))) for x in (d, u, r))
        x = torch.empty_like(r)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        ms_oee = timed(lambda: fd.btd_solve6(d, u, r, off, n, out=x, status=st, stream=stream))
        status = int(st.item())
        # FP64 must factor every system; in FP32 the generator's worst systems
        # (cond_2 up to ~1e7 at 128 blocks) can lose a pivot, which the status reports
        if status != 0 and dtype == "f64":
            raise RuntimeError(f"btd_solve6 status {status} at n={n}")
        rows = batch * n
        out[str(n)] = {
            "levels": levels,
            "scan_ms": ms_scan, "scan_us_per_level": 1e3 * ms_scan / levels,
            "scan_gb_s": rows * (36 + 12) * w / (ms_scan * 1e-3) / 1e9,
            "oee_ms": ms_oee, "oee_us_per_level": 1e3 * ms_oee / levels, "oee_status": status,
            "oee_gb_s": rows * (72 + 12) * w / (ms_oee * 1e-3) / 1e9,
        }
        del sb, sc, sx, d, u, r, x
        torch.cuda.empty_cache()
    return out


def adjoint_leg(dtype: str, reps: int = 10):
    """Reverse mode. (1) At 65536 chains of 64 links: the vector-Jacobian product
    (fd_backward) per launch, with lambda = M^-1 g by each algorithm, beside that
    algorithm's plain forward launch. (2) The differentiation workload: 16384
    chains of 32 links, a 100-step semi-implicit Euler rollout (dt = 1e-3,
    tau ~ N(0, 1) per step), loss = sum of squared final q and qd, gradient with
    respect to q_0, qd_0 and every tau_t with checkpoints every 10 steps:
    forward and backward beside 100 plain forward + Euler steps."""
    import torch

    from paper_1609_06779_amd import fd, synth, tune

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    stream = torch.cuda.current_stream()

    def timed(fn, count):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(count):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / count

    batch, n = 65536, 64
    lengths = synth.uniform_lengths(batch, n)
    rb = synth.make_robots(lengths, cfg=2)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
    q, qd, tau = synth.make_state(lengths, cfg=2)
    model = fd.Model(rb, dtype, device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
    g = torch.from_numpy(np.random.default_rng(5).standard_normal(len(q))).to(dev, tdt)
    gq, gqd, gt = (torch.empty_like(tq) for _ in range(3))
    qdd = torch.empty_like(tq)
    out = {"workload": f"uniform-n{n}-b{batch}", "per_algo": {}}
    for algo in ("abia", "jsiia", "cfa"):
        ws = model.workspace(batch, algo)
        ms_fwd = timed(lambda: model.forward(tq, tqd, ttau, batch=batch, algo=algo, out=qdd, workspace=ws,
                                             stream=stream), reps)
        bws = model.backward_workspace(batch, algo)
        ms_vjp = timed(lambda: model.backward(tq, tqd, qdd, g, batch=batch, algo=algo, grad_q=gq, grad_qd=gqd,
                                              grad_tau=gt, workspace=bws, stream=stream), reps)
        out["per_algo"][algo] = {"forward_ms": ms_fwd, "vjp_ms": ms_vjp, "vjp_over_forward": ms_vjp / ms_fwd}
        del ws, bws
    out["abia_forward_ms"] = out["per_algo"]["abia"]["forward_ms"]
    out["vjp_ms"] = out["per_algo"]["abia"]["vjp_ms"]
    out["vjp_over_forward"] = out["per_algo"]["abia"]["vjp_over_forward"]
    model.close()
    del tq, tqd, ttau, qdd, g, gq, gqd, gt
    torch.cuda.empty_cache()

    # the differentiation workload, exactly
    batch, n, steps, dt, every = 16384, 32, 100, 1e-3, 10
    lengths = synth.uniform_lengths(batch, n)
    rb = synth.make_robots(lengths, cfg=5)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
    q0n, qd0n, _ = synth.make_state(lengths, cfg=5)
    model = fd.Model(rb, dtype, device=dev)
    tq, tqd = (torch.from_numpy(a).to(dev, tdt) for a in (q0n, qd0n))
    taus = torch.from_numpy(np.random.default_rng(5).standard_normal((steps, len(q0n)))).to(dev, tdt)
    algo = tune.best_algo(dtype, n, batch)
    ws = model.workspace(batch, algo)
    qdd = torch.empty_like(tq)
    qs, qds = tq.clone(), tqd.clone()

    def plain_steps():
        qs.copy_(tq)
        qds.copy_(tqd)
        for t in range(steps):
            model.forward(qs, qds, taus[t], batch=batch, algo=algo, out=qdd, workspace=ws, stream=stream)
            model.euler_step(qs, qds, qdd, dt, q_next=qs, qd_next=qds, stream=stream)

    ms_plain = timed(plain_steps, 2)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for rep in range(2):                           # the second pass is timed (allocator warm)
        q0, qd0 = tq.clone().requires_grad_(True), tqd.clone().requires_grad_(True)
        tt = taus.clone().requires_grad_(True)
        torch.cuda.synchronize()
        ev[0].record(stream)
        qT, qdT = fd.rollout(model, q0, qd0, tt, batch=batch, dt=dt, every=every, algo=algo)
        ev[1].record(stream)
        ((qT ** 2).sum() + (qdT ** 2).sum()).backward()
        ev[2].record(stream)
        torch.cuda.synchronize()
        assert torch.isfinite(tt.grad).all().item() and torch.isfinite(q0.grad).all().item()
    fwd_ms, bwd_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    out["rollout"] = {"workload": f"rollout-n{n}-b{batch}-T{steps}", "steps": steps, "dt": dt,
                      "checkpoint_every": every, "algo": algo, "forward_ms": fwd_ms, "backward_ms": bwd_ms,
                      "plain_forward_steps_ms": ms_plain, "forward_over_plain": fwd_ms / ms_plain,
                      "backward_over_plain": bwd_ms / ms_plain,
                      "gradient_solves_per_s": batch * steps / ((fwd_ms + bwd_ms) * 1e-3)}
    del qs, qds, q0, qd0, tt, qT, qdT
    model.close()
    del tq, tqd, taus, qdd, ws
    torch.cuda.empty_cache()
    # launch-bound sizes: a 100-step rollout (no gradient) of 64 chains of 16 links
    # (JSIIA, the fastest there), launched step by step against the same steps
    # recorded in one HIP graph
    sb, sn, ssteps = 64, 16, 100
    sl = synth.uniform_lengths(sb, sn)
    srb = synth.make_robots(sl, cfg=2)
    if dtype == "f32":
        srb = srb.astype_rounded(np.float32)
    smodel = fd.Model(srb, dtype, device=dev)
    sq0, sqd0, _ = (torch.from_numpy(a).to(dev, tdt) for a in synth.make_state(sl, cfg=2))
    staus = torch.from_numpy(np.random.default_rng(9).standard_normal((ssteps, sb * sn))).to(dev, tdt)
    sws = smodel.workspace(sb, "jsiia")
    sq, sqd, sqdd = sq0.clone(), sqd0.clone(), torch.empty_like(sq0)

    def eager_rollout():
        sq.copy_(sq0)
        sqd.copy_(sqd0)
        for t in range(ssteps):
            smodel.forward(sq, sqd, staus[t], batch=sb, algo="jsiia", out=sqdd, workspace=sws, stream=stream)
            smodel.euler_step(sq, sqd, sqdd, dt, q_next=sq, qd_next=sqd, stream=stream)

    rg = fd.RolloutGraph(smodel, sb, ssteps, dt, algo="jsiia")
    ms_eager = timed(eager_rollout, 5)
    ms_graph = timed(lambda: rg.run(sq0, sqd0, staus), 5)
    assert torch.equal(rg.q, sq) and torch.equal(rg.qd, sqd)
    out["small_batch_rollout"] = {"chains": sb, "n_links": sn, "steps": ssteps, "algo": "jsiia", "eager_ms": ms_eager,
                                  "graph_ms": ms_graph, "speedup": ms_eager / ms_graph}
    del rg
    smodel.close()
    # the same VJP on branched robots of the same size (tree workloads of the tree leg)
    out["trees"] = {}
    for key in TREE_WORKLOADS:
        w = synth.WORKLOADS[key]
        tl = synth.uniform_lengths(w["batch"], w["n"])
        rb = synth.make_tree_robots(tl, p_extend=w["p_extend"], cfg=w["cfg"],
                                    shared_topology=w.get("shared_topology", False))
        if dtype == "f32":
            rb = rb.astype_rounded(np.float32)
        q, qd, tau = synth.make_state(tl, cfg=w["cfg"])
        model = fd.Model(rb, dtype, device=dev)
        tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
        ws = model.workspace(w["batch"], "abia")
        qdd = torch.empty_like(tq)
        ms_fwd = timed(lambda: model.forward(tq, tqd, ttau, batch=w["batch"], algo="abia", out=qdd, workspace=ws,
                                             stream=stream), reps)
        g = torch.from_numpy(np.random.default_rng(5).standard_normal(len(q))).to(dev, tdt)
        bws = model.backward_workspace(w["batch"], "abia")
        gq, gqd, gt = (torch.empty_like(tq) for _ in range(3))
        ms_vjp = timed(lambda: model.backward(tq, tqd, qdd, g, batch=w["batch"], grad_q=gq, grad_qd=gqd,
                                              grad_tau=gt, workspace=bws, stream=stream), reps)
        assert torch.isfinite(gq).all().item() and torch.isfinite(gt).all().item()
        out["trees"][key] = {"abia_forward_ms": ms_fwd, "vjp_ms": ms_vjp, "vjp_over_forward": ms_vjp / ms_fwd}
        model.close()
        del tq, tqd, ttau, qdd, g, gq, gqd, gt, ws, bws
        torch.cuda.empty_cache()
    return out


def experiments_leg(dtype: str, calls: int = 200):
    """The paper's two experiment shapes (Sec. V) on this GPU, FP64: Exp. 1, the
    time of one call for one robot against its number of links; Exp. 2, the time
    of one call over a group of independent robots of 10 and of 200 links
    against the group size. Mean over back-to-back calls with fresh random
    inputs each (launch overhead included), as the paper times them."""
    from paper_1609_06779_amd import tune

    rows = tune.experiments(dtype, calls=calls)
    exp1, exp1d, exp2, exp2d = {}, {}, {}, {}
    for r in rows:
        if r["exp"] == 1:
            exp1.setdefault(r["algo"], {})[str(r["n"])] = None if r["ms"] is None else r["ms"] * 1e3
            exp1d.setdefault(r["algo"], {})[str(r["n"])] = None if r["device_ms"] is None else r["device_ms"] * 1e3
        else:
            exp2.setdefault(f"n{r['n']}", {}).setdefault(r["algo"], {})[str(r["groups"])] = r["ms"]
            exp2d.setdefault(f"n{r['n']}", {}).setdefault(r["algo"], {})[str(r["groups"])] = r["device_ms"]
    return {"calls": calls, "exp1_us_per_call": exp1, "exp1_device_us": exp1d, "exp2_ms_per_call": exp2,
            "exp2_device_ms": exp2d}


TREE_WORKLOADS = ("tree-shared-n64-b65536", "tree-n64-b65536")


def tree_leg(dtype: str, reps: int = 10, keys=TREE_WORKLOADS):
    """Branched robots, one launch (ABIA, then JSIIA) over 65536 trees of 64 links
    (depth-first numbered; each link extends the previous one with probability
    0.85, else hangs from a random link of the current path). Two topology
    mixes: one topology shared by every robot (each with its own parameters),
    and a random topology per robot (lanes of a wavefront branch at different
    links, the worst case for divergence)."""
    import torch

    from paper_1609_06779_amd import fd, synth

    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    esz = 8 if dtype == "f64" else 4
    out = {}
    for key in keys:
        w = synth.WORKLOADS[key]
        batch, n = w["batch"], w["n"]
        lengths = synth.uniform_lengths(batch, n)
        rb = synth.make_tree_robots(lengths, p_extend=w["p_extend"], cfg=w["cfg"],
                                    shared_topology=w.get("shared_topology", False))
        if dtype == "f32":
            rb = rb.astype_rounded(np.float32)
        q, qd, tau = synth.make_state(lengths, cfg=w["cfg"])
        model = fd.Model(rb, dtype, device=dev)
        tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
        res = torch.empty_like(tq)
        stream = torch.cuda.current_stream()
        par = rb.parents().reshape(batch, n)
        branch_points = float(np.mean([(np.bincount(p[p >= 0], minlength=n) > 1).sum() for p in par[:1024]]))
        algo_bytes = batch * n * ((4 + 17) * esz + 4)       # state, the model's 17 fields and one tree code
        entry = {"branch_points_per_tree": branch_points}
        for algo in ("abia", "jsiia"):
            ws = model.workspace(batch, algo)
            model.forward(tq, tqd, ttau, batch=batch, algo=algo, out=res, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                model.forward(tq, tqd, ttau, batch=batch, algo=algo, out=res, workspace=ws, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            assert torch.isfinite(res).all().item(), f"{key}: tree {algo} produced non-finite qdd"
            entry[algo] = {"ms_per_launch": ms, "solves_per_s": batch / (ms * 1e-3)}
            if algo == "abia":
                entry[algo].update({"algorithmic_bytes": algo_bytes,
                                    "algorithmic_gb_per_s": algo_bytes / (ms * 1e-3) / 1e9})
            del ws
        out[key] = entry
        model.close()
        del model, tq, tqd, ttau, res
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--algos", default="abia,jsiia,cfa")
    ap.add_argument("--cpu-chains", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the oracle's reference values for the per-(algorithm, n, dtype) error record")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-tree", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-transfer", action="store_true")
    ap.add_argument("--no-levels", action="store_true")
    ap.add_argument("--no-experiments", action="store_true")
    ap.add_argument("--no-nsweep", action="store_true")
    ap.add_argument("--only-step", action="store_true",
                    help="time the step alone: no legs and no CPU baseline (the profiled command)")
    ap.add_argument("--only-trees", action="store_true", help="run the branched-robot leg alone")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run the reverse-mode leg alone (VJPs and the differentiation workload)")
    ap.add_argument("--only-ragged", action="store_true",
                    help="run the ragged-batch leg alone (per_algo: the persistent launch's event time)")
    ap.add_argument("--tree-workloads", default=",".join(TREE_WORKLOADS))
    ap.add_argument("--workload", help="with --trace-summary or --pmc-summary: the workload name to file under")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device copy, the known-size reference for HBM counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into profiles/ and exit (no GPU use)")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="with --pmc-summary or --trace-summary: the profiler command lines to record")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run into profiles/ and exit (no GPU use)")
    ap.add_argument("--bench-log", help="with --trace-summary or --flops-summary: output of the profiled bench.py run")
    ap.add_argument("--lds-pass", metavar="P3_DIR", help="with --flops-summary: the LDS counter pass")
    ap.add_argument("--flops-summary", nargs=2, metavar=("P1_DIR", "P2_DIR"),
                    help="summarise the two FP64 VALU counter passes into profiles/ and exit (no GPU use)")
    args = ap.parse_args()
    if args.only_step:
        args.no_cpu = args.no_serve = args.no_ragged = args.no_tree = args.no_adjoint = args.no_transfer = True
        args.no_levels = args.no_nsweep = args.no_experiments = True
    wl = args.workload or f"fd_forward_n{args.n}_b{args.batch}_{args.dtype}"
    wl_flag = f" --workload {args.workload}" if args.workload else ""
    if args.trace_summary:
        print(summarize_trace(args.trace_summary, wl, args.pmc_command,
                              f"python bench.py --trace-summary {args.trace_summary} --n {args.n} "
                              f"--batch {args.batch} --dtype {args.dtype}{wl_flag} --bench-log {args.bench_log} "
                              f"--pmc-command ...", args.bench_log))
        return
    if args.flops_summary:
        print(summarize_flops(*args.flops_summary, wl, args.pmc_command,
                              f"python bench.py --flops-summary {' '.join(args.flops_summary)} --n {args.n} "
                              f"--batch {args.batch} --dtype {args.dtype}{wl_flag} --bench-log {args.bench_log} "
                              f"{' --lds-pass ' + args.lds_pass if args.lds_pass else ''} --pmc-command ...",
                              args.bench_log, args.n, args.batch, args.dtype, args.lds_pass))
        return
    if args.pmc_summary:
        print(summarize_pmc(*args.pmc_summary, wl, args.pmc_command,
                            f"python bench.py --pmc-summary {' '.join(args.pmc_summary)} --n {args.n} "
                            f"--batch {args.batch} --dtype {args.dtype}{wl_flag} --pmc-command ..."))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); chains are independent, so a "
              "multi-GPU run would shard the batch with no exchange. Nothing was run.", file=sys.stderr)
        sys.exit(2)

    tree_keys = [k for k in args.tree_workloads.split(",") if k]
    if args.only_ragged:
        print(f"[bench] ragged leg alone: {args.dtype}", file=sys.stderr, flush=True)
        if args.copy_calib:
            import torch
            copy_calibration(torch.device("cuda:0"))
        rg = ragged_leg(args.dtype)
        print(json.dumps({"ragged": rg, "dtype": args.dtype,
                          "per_algo": {"abia_persistent": {"ms_per_launch": rg["persistent_ms"]}}}), flush=True)
        return
    if args.only_adjoint:
        print(f"[bench] reverse-mode leg alone: {args.dtype}", file=sys.stderr, flush=True)
        print(json.dumps({"adjoint": adjoint_leg(args.dtype), "dtype": args.dtype}), flush=True)
        return
    if args.only_trees:
        print(f"[bench] tree leg alone: {tree_keys} {args.dtype}", file=sys.stderr, flush=True)
        if args.copy_calib:
            import torch
            copy_calibration(torch.device("cuda:0"))
        print(json.dumps({"trees": tree_leg(args.dtype, keys=tree_keys), "dtype": args.dtype}), flush=True)
        return

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

    if args.copy_calib:
        copy_calibration(dev)
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
        times = [e[a][0].elapsed_time(e[a][1]) for e in ev]
        ms = float(np.mean(times))
        fl = 2.0 * fma_per_solve(a, args.n) * args.batch
        per_algo[a] = {"ms_per_launch": ms, "median_ms": float(np.median(times)), "min_ms": float(np.min(times)),
                       "solves_per_s": args.batch / (ms * 1e-3), "tflops": fl / (ms * 1e-3) / 1e12}
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
                     "frac": achieved / peak,
                     "traffic": measured_traffic(dominant, f"fd_forward_n{args.n}_b{args.batch}_{args.dtype}")},
    }
    if not args.no_ragged:
        print("[bench] ragged leg", file=sys.stderr, flush=True)
        result["ragged"] = ragged_leg(args.dtype)
    if not args.no_transfer:
        print("[bench] transfer leg", file=sys.stderr, flush=True)
        result["host_transfer"] = transfer_leg(args.dtype)
    if not args.no_nsweep:
        print("[bench] n sweep leg", file=sys.stderr, flush=True)
        result["n_sweep"] = nsweep_leg()
    if not args.no_experiments:
        print("[bench] experiments leg", file=sys.stderr, flush=True)
        result["experiments"] = experiments_leg(args.dtype)
    if not args.no_levels:
        print("[bench] levels leg", file=sys.stderr, flush=True)
        result["levels"] = levels_leg(args.dtype)
    if not args.no_adjoint:
        print("[bench] adjoint leg", file=sys.stderr, flush=True)
        result["adjoint"] = adjoint_leg(args.dtype)
    if not args.no_tree:
        print("[bench] tree leg", file=sys.stderr, flush=True)
        result["trees"] = tree_leg(args.dtype, keys=tree_keys)
    if not args.no_serve:
        print("[bench] serving leg", file=sys.stderr, flush=True)
        result["serving"] = serving_leg(args.dtype)
        l80 = result["serving"]["load_80pct"]
        result["p99_latency_ms_at_80pct_load"] = l80["p99_ms"]
        result["p99_latency_ms_at_5000_qps"] = result["serving"]["qps_5000"]["p99_ms"]
    if not args.no_cpu and args.dtype == "f64":
        print("[bench] cpu baseline leg", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(rb, q, qd, tau, min(args.cpu_chains, args.batch))
        if not args.no_accuracy:
            result["cpu_baseline"]["accuracy"] = cpu_baseline_accuracy()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
