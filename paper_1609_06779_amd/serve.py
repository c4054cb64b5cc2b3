"""Continuous-batching server for forward-dynamics requests.

A request asks for qdd of ``chains`` chains of one resident robot. The server
keeps every robot of the model resident on the GPU and runs a host loop that,
at every turn,
  1. retires launches whose completion event has fired (their results are in
     host memory) and returns their device memory to the budget;
  2. admits arrived requests in arrival order, packing as many as fit the free
     HBM budget (state buffers and workspace) into one launch: a ragged batch
     of mixed robots (robot ids and chain offsets) for one ``fd_forward`` call;
  3. issues that launch on the next stream of a small pool, so the work of
     requests admitted at different times overlaps on the device.
Within a round, requests are grouped by algorithm (the tuned choice for
their robot length and chain count, by default), one launch per group. A
request larger than the whole budget is rejected. With the articulated-body
algorithm every chain stays on its own lane, so a chain's result does not
depend on what else shares its launch (the tests check it bit for bit).

The policy (``Scheduler``) is independent of the device: it drives an
``Executor`` (``GpuExecutor`` here, a simulated one in the tests) with a clock.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    robot: int
    chains: int
    n: int                       # links of the robot
    arrival: float               # seconds on the scheduler's clock
    q: object = None             # host tensors [chains * n] (pinned), filled by the caller
    qd: object = None
    tau: object = None
    out: object = None           # host tensor receiving qdd
    algo: str = ""               # algorithm that served it (set at launch)
    admitted: float = math.nan
    done: float = math.nan
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Executor:
    """What the scheduler needs from a device."""

    def bytes_needed(self, reqs: List[Request]) -> int:
        raise NotImplementedError

    def launch(self, reqs: List[Request]):
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def retire(self, handle) -> None:
        raise NotImplementedError


@dataclasses.dataclass
class Stats:
    completed: int
    rejected: int
    chains: int
    wall: float
    p50: float
    p99: float
    mean: float
    launches: int
    max_inflight: int

    @property
    def solves_per_s(self) -> float:
        return self.chains / self.wall if self.wall > 0 else 0.0


class Scheduler:
    def __init__(self, executor: Executor, budget_bytes: int, max_inflight: int = 4,
                 max_chains_per_launch: int = 65536, clock: Callable[[], float] = time.perf_counter,
                 idle: Optional[Callable[[float], None]] = None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.max_chains = int(max_chains_per_launch)
        self.clock = clock
        self.idle = idle

    def run(self, requests: List[Request]) -> Stats:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        inflight = []                    # (handle, reqs, bytes)
        used = 0
        launches = 0
        peak = 0
        t0 = self.clock()
        start = None
        while pending or queue or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for item in list(inflight):
                handle, reqs, nbytes = item
                if self.ex.poll(handle):
                    self.ex.retire(handle)
                    t = self.clock() - t0
                    for r in reqs:
                        r.done = t
                    used -= nbytes
                    inflight.remove(item)
                    progressed = True
            while queue and len(inflight) < self.max_inflight:
                group = []
                chains = 0
                while queue and chains + queue[0].chains <= self.max_chains:
                    cand = group + [queue[0]]
                    if used + self.ex.bytes_needed(cand) > self.budget:
                        break
                    group.append(queue.popleft())
                    chains += group[-1].chains
                if not group:
                    head = queue[0]
                    if self.ex.bytes_needed([head]) > self.budget or head.chains > self.max_chains:
                        head.rejected = True
                        queue.popleft()
                        progressed = True
                        continue
                    break                          # wait for memory to come back
                nbytes = self.ex.bytes_needed(group)
                t = self.clock() - t0
                for r in group:
                    r.admitted = t
                if start is None:
                    start = t
                inflight.append((self.ex.launch(group), group, nbytes))
                used += nbytes
                launches += 1
                peak = max(peak, len(inflight))
                progressed = True
            if not progressed and self.idle is not None:
                # seconds until the next arrival (None: nothing left to arrive)
                self.idle(pending[0].arrival - (self.clock() - t0) if pending else None)
        done = [r for r in requests if not r.rejected]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        end = max((r.done for r in done), default=0.0)
        first = min((r.arrival for r in done), default=0.0)
        return Stats(completed=len(done), rejected=sum(r.rejected for r in requests),
                     chains=sum(r.chains for r in done), wall=end - first,
                     p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                     mean=float(lat.mean()), launches=launches, max_inflight=peak)


class GpuExecutor(Executor):
    """Launches ``fd_forward`` over packed ragged batches on a pool of streams.

    Each launch round copies its requests' pinned host inputs into fresh device
    buffers and runs one forward-dynamics call per algorithm among its
    requests (robot ids and chain offsets), copies qdd back into the requests'
    pinned outputs and records one event. ``algo`` is an algorithm name,
    "auto" (the tuned table's choice for the request's robot length and chain
    count) or a function of the request.
    """

    def __init__(self, model, n_links: np.ndarray, algo="auto", streams: int = 4):
        import torch

        from . import tune

        self.torch = torch
        self.model = model
        self.n_links = np.asarray(n_links, dtype=np.int64)
        if algo == "auto":
            self.pick = lambda r: tune.best_algo(model.dtype, r.n, r.chains)
        elif callable(algo):
            self.pick = algo
        else:
            self.pick = lambda r, a=algo: a
        self.streams = [torch.cuda.Stream(device=model.device) for _ in range(streams)]   # default priority
        self.turn = 0
        self.esz = 8 if model.dtype == "f64" else 4
        # ABIA workspace values per link and lane: 7, plus a 33-value branch-point record on trees
        self.abia_fields = 40 if getattr(model, "branched", False) else 7

    def _groups(self, reqs):
        groups = collections.OrderedDict()
        for r in reqs:
            algo = self.pick(r)
            if r.n > self.model.max_links(algo):
                algo = "abia"
            groups.setdefault(algo, []).append(r)
        return groups

    def bytes_needed(self, reqs):
        total = 0
        for algo, grp in self._groups(reqs).items():
            chains = sum(r.chains for r in grp)
            links = sum(r.chains * r.n for r in grp)
            nmax = max(r.n for r in grp)
            ws = ((chains + 63) // 64) * nmax * self.abia_fields * 64 * self.esz if algo == "abia" else 0
            total += 4 * links * self.esz + 12 * chains + 8 + ws
        return total

    def launch(self, reqs):
        torch = self.torch
        stream = self.streams[self.turn % len(self.streams)]
        self.turn += 1
        keep = []
        with torch.cuda.stream(stream):
            for algo, grp in self._groups(reqs).items():
                keep.append(self._launch_group(algo, grp, stream))
            ev = torch.cuda.Event()
            ev.record(stream)
        # keep the device buffers and pinned staging alive until the event fires
        return (ev, keep)

    def _launch_group(self, algo, reqs, stream):
        torch = self.torch
        dev = self.model.device
        dt = self.model.torch_dtype
        chains = sum(r.chains for r in reqs)
        links = sum(r.chains * r.n for r in reqs)
        rid_h = torch.empty(chains, dtype=torch.int32, pin_memory=True)
        off_h = torch.empty(chains + 1, dtype=torch.int64, pin_memory=True)
        rid_np, off_np = rid_h.numpy(), off_h.numpy()
        pos, c = 0, 0
        for r in reqs:
            rid_np[c:c + r.chains] = r.robot
            off_np[c:c + r.chains] = pos + r.n * np.arange(r.chains)
            c += r.chains
            pos += r.chains * r.n
        off_np[chains] = pos
        q = torch.empty(links, dtype=dt, device=dev)
        qd = torch.empty_like(q)
        tau = torch.empty_like(q)
        out = torch.empty_like(q)
        rid = rid_h.to(dev, non_blocking=True)
        off = off_h.to(dev, non_blocking=True)
        pos = 0
        for r in reqs:
            k = r.chains * r.n
            q[pos:pos + k].copy_(r.q, non_blocking=True)
            qd[pos:pos + k].copy_(r.qd, non_blocking=True)
            tau[pos:pos + k].copy_(r.tau, non_blocking=True)
            pos += k
        nmax = max(r.n for r in reqs)                  # lane groups sized to this group's longest robot
        ws = self.model.workspace(chains, algo, robot_id=rid, offsets=off, max_links=nmax)
        self.model.forward(q, qd, tau, batch=chains, algo=algo, robot_id=rid, offsets=off, out=out,
                           workspace=ws, stream=stream, max_links=nmax)
        pos = 0
        for r in reqs:
            k = r.chains * r.n
            r.out.copy_(out[pos:pos + k], non_blocking=True)
            r.algo = algo
            pos += k
        return (q, qd, tau, out, rid, off, ws, rid_h, off_h)

    def poll(self, handle):
        return handle[0].query()

    def retire(self, handle):
        handle[0].synchronize()


def poisson_arrivals(count: int, qps: float, seed: int = 1609) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def request_sizes(count: int, lo: int = 1, hi: int = 4096, seed: int = 1609) -> np.ndarray:
    """Log-uniform integer chain counts in [lo, hi]."""
    rng = np.random.default_rng(seed + 1)
    return np.minimum(hi, np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=count)))).astype(np.int64)


def make_requests(robot_lengths, count: int, qps: float, seed: int = 1609, dtype: str = "f64",
                  max_chains: int = 4096, shared: bool = False):
    """Seeded request stream: robot uniform over the resident set, chains
    log-uniform in [1, max_chains], Poisson arrivals at ``qps`` (qps = inf: all
    at t = 0). Inputs are pinned host tensors drawn like the synthetic states;
    with ``shared`` every request views one pinned pool (inputs and outputs),
    which bounds host memory for long benchmark streams."""
    import torch

    from . import synth

    robot_lengths = np.asarray(robot_lengths, dtype=np.int64)
    rng = np.random.default_rng(seed + 2)
    robots = rng.integers(0, len(robot_lengths), size=count)
    sizes = request_sizes(count, 1, max_chains, seed=seed)
    arrivals = np.zeros(count) if math.isinf(qps) else poisson_arrivals(count, qps, seed=seed)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    pool = None
    if shared:
        k = int(max_chains * robot_lengths.max())
        q, qd, tau = synth.make_state([k], seed=seed, cfg=4)
        pool = [torch.from_numpy(a).to(tdt).pin_memory() for a in (q, qd, tau)]
        pool.append(torch.empty(k, dtype=tdt).pin_memory())
    reqs = []
    for i in range(count):
        n = int(robot_lengths[robots[i]])
        k = int(sizes[i]) * n
        r = Request(rid=i, robot=int(robots[i]), chains=int(sizes[i]), n=n, arrival=float(arrivals[i]))
        if pool is None:
            q, qd, tau = synth.make_state([k], seed=seed, cfg=4, rep=i)
            r.q = torch.from_numpy(q).to(tdt).pin_memory()
            r.qd = torch.from_numpy(qd).to(tdt).pin_memory()
            r.tau = torch.from_numpy(tau).to(tdt).pin_memory()
            r.out = torch.empty(k, dtype=tdt).pin_memory()
        else:
            r.q, r.qd, r.tau, r.out = (t[:k] for t in pool)
        reqs.append(r)
    return reqs


def spin_idle(seconds):
    """Idle hook for a real device: sleep only while waiting for a distant arrival."""
    if seconds is not None and seconds > 2e-4:
        time.sleep(min(seconds, 1e-3) - 1e-4)
