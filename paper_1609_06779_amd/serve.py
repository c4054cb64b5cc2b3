"""Continuous-batching server for forward-dynamics requests.

A request asks for qdd of ``chains`` chains of one resident robot. The server
keeps every robot of the model resident on the GPU and runs a host loop that,
at every turn,
  1. retires launches whose completion event has fired (their results are in
     host memory) and returns their device memory to the budget;
  2. admits arrived requests in arrival order, packing as many as fit the free
     HBM budget (state buffers and workspace) into one launch: a ragged batch
     of mixed robots (robot ids and chain offsets) for one ``fd_forward`` call;
  3. issues that launch on a free slot of a small pool of streams, so the work
     of requests admitted at different times overlaps on the device.
By default the library's AUTO rule picks the algorithm for each round's whole
batch; a fixed algorithm or a per-request choice groups the round by
algorithm instead, one launch per group. A request larger than the whole
budget is rejected. With the articulated-body
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
        # never more launches in flight than the executor has room for
        self.max_inflight = min(int(max_inflight), int(getattr(executor, "capacity", max_inflight)))
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

    ``algo="auto"`` (the default) runs one launch per round: the round's
    requests form one ragged batch (robot ids and chain offsets) and the
    library's AUTO rule picks the algorithm for that whole batch (its size and
    longest chain), so a round of many chains takes the length-sorted persistent
    launch and a round of a few chains a lane-per-link kernel. An algorithm name,
    or a function of the request, instead groups the round by algorithm, one
    launch per group.

    Each launch takes a free slot: a stream with its own pinned staging for the
    robot ids and offsets, reused launch after launch (a slot is only reused
    once its previous launch has retired). Inputs of requests whose pinned host
    buffers follow one another go over in one copy per array, and so do their
    outputs. Events around the copies in, the kernel and the copies out give
    the time breakdown in ``timing``.
    """

    def __init__(self, model, n_links, algo="auto", streams: int = 4, slots: int = 8, max_chains: int = 65536,
                 breakdown: bool = True):
        import torch

        self.torch = torch
        self.model = model
        self.n_links = np.asarray(n_links, dtype=np.int64)
        self.per_launch_auto = algo == "auto"
        if callable(algo):
            self.pick = algo
        else:
            self.pick = lambda r, a=algo: a
        self.max_chains = int(max_chains)
        self.breakdown = breakdown
        self.esz = 8 if model.dtype == "f64" else 4
        pool = [torch.cuda.Stream(device=model.device) for _ in range(streams)]   # default priority
        self.slots = []
        for k in range(max(slots, 1)):
            rid = torch.empty(self.max_chains, dtype=torch.int32, pin_memory=True)
            off = torch.empty(self.max_chains + 1, dtype=torch.int64, pin_memory=True)
            self.slots.append((pool[k % len(pool)], rid, off))
        self.free = list(range(len(self.slots)))[::-1]
        self.capacity = len(self.slots)       # launches in flight at most
        self.timing = collections.Counter()

    def _groups(self, reqs):
        if self.per_launch_auto:
            return {"auto": list(reqs)}
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
            ws = self.model.workspace_bytes(chains, algo, ragged=True, with_ids=True, max_links=nmax)
            total += 4 * links * self.esz + 12 * chains + 8 + ws
        return total

    def launch(self, reqs):
        torch = self.torch
        t0 = time.perf_counter()
        k = self.free.pop()
        stream = self.slots[k][0]
        keep = []
        ev = [torch.cuda.Event(enable_timing=self.breakdown) for _ in range(4)]
        with torch.cuda.stream(stream):
            groups = list(self._groups(reqs).items())
            ev[0].record(stream)
            staged = [self._stage_in(algo, grp, k, g) for g, (algo, grp) in enumerate(groups)]
            ev[1].record(stream)
            for (algo, grp), st in zip(groups, staged):
                keep.append(self._run(algo, grp, st, stream))
            ev[2].record(stream)
            for (algo, grp), st in zip(groups, staged):
                _copy_runs(grp, st[3], "out", to_host=True)
            ev[3].record(stream)
        self.timing["launches"] += 1
        self.timing["host_launch_s"] += time.perf_counter() - t0
        # keep the device buffers alive until the last event fires
        return (ev, keep, k)

    def _stage_in(self, algo, reqs, slot, group):
        torch = self.torch
        dev, dt = self.model.device, self.model.torch_dtype
        _, rid_h, off_h = self.slots[slot]
        sizes = np.fromiter((r.chains for r in reqs), np.int64, len(reqs))
        ns = np.fromiter((r.n for r in reqs), np.int64, len(reqs))
        chains, links = int(sizes.sum()), int((sizes * ns).sum())
        # the slot's staging holds the first group of a round; further groups
        # (rounds by algorithm) and oversized ones take fresh pinned memory
        if group == 0 and chains <= self.max_chains:
            rid_np, off_np = rid_h.numpy()[:chains], off_h.numpy()[:chains + 1]
        else:
            rid_h = torch.empty(chains, dtype=torch.int32, pin_memory=True)
            off_h = torch.empty(chains + 1, dtype=torch.int64, pin_memory=True)
            rid_np, off_np = rid_h.numpy(), off_h.numpy()
        rid_np[:] = np.repeat(np.fromiter((r.robot for r in reqs), np.int64, len(reqs)), sizes)
        first_chain = np.repeat(np.cumsum(sizes) - sizes, sizes)
        first_link = np.repeat(np.cumsum(sizes * ns) - sizes * ns, sizes)
        off_np[:chains] = first_link + (np.arange(chains) - first_chain) * np.repeat(ns, sizes)
        off_np[chains] = links
        q = torch.empty(links, dtype=dt, device=dev)
        qd, tau, out = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
        rid = torch.empty(chains, dtype=torch.int32, device=dev)
        off = torch.empty(chains + 1, dtype=torch.int64, device=dev)
        rid.copy_(rid_h[:chains], non_blocking=True)
        off.copy_(off_h[:chains + 1], non_blocking=True)
        for name, dst in (("q", q), ("qd", qd), ("tau", tau)):
            _copy_runs(reqs, dst, name, to_host=False)
        self.timing["bytes_h2d"] += 3 * links * self.esz + 12 * chains + 8
        self.timing["bytes_d2h"] += links * self.esz
        return (q, qd, tau, out, rid, off, chains, int(ns.max()), rid_h, off_h)

    def _run(self, algo, reqs, st, stream):
        q, qd, tau, out, rid, off, chains, nmax = st[:8]
        name = algo
        if algo == "auto":
            name, persistent = self.model.auto_algo(chains, ragged=True, with_ids=True, max_links=nmax)
            self.timing["persistent_launches"] += int(persistent)
        ws = self.model.workspace(chains, algo, robot_id=rid, offsets=off, max_links=nmax, stream=stream)
        self.model.forward(q, qd, tau, batch=chains, algo=algo, robot_id=rid, offsets=off, out=out,
                           workspace=ws, stream=stream, max_links=nmax)
        for r in reqs:
            r.algo = name
        self.timing[f"chains_{name}"] += chains
        return st + (ws,)

    def poll(self, handle):
        return handle[0][3].query()

    def retire(self, handle):
        ev, _, k = handle
        ev[3].synchronize()
        if self.breakdown:
            self.timing["h2d_ms"] += ev[0].elapsed_time(ev[1])
            self.timing["kernel_ms"] += ev[1].elapsed_time(ev[2])
            self.timing["d2h_ms"] += ev[2].elapsed_time(ev[3])
        self.free.append(k)


def _copy_runs(reqs, dev_buf, name, to_host):
    """Copy one per-request host array (q, qd, tau in; out back) between the
    requests' pinned buffers and a packed device buffer, merging requests whose
    host buffers are consecutive views of one storage into one copy."""
    pos = 0
    run_start, run_len, run_host = 0, 0, None
    for r in reqs:
        h = getattr(r, name)
        k = r.chains * r.n
        if (run_host is not None and h.untyped_storage().data_ptr() == run_host.untyped_storage().data_ptr()
                and h.data_ptr() == run_host.data_ptr() + run_len * run_host.element_size()):
            run_len += k
        else:
            if run_host is not None:
                _copy_one(run_host, run_len, dev_buf, run_start, to_host)
            run_start, run_len, run_host = pos, k, h
        pos += k
    if run_host is not None:
        _copy_one(run_host, run_len, dev_buf, run_start, to_host)


def _copy_one(first, length, dev_buf, start, to_host):
    """One copy of `length` entries of a host storage, from `first`'s first entry on."""
    if length == 0:
        return
    host = first.as_strided((length,), (1,), first.storage_offset())
    if to_host:
        host.copy_(dev_buf[start:start + length], non_blocking=True)
    else:
        dev_buf[start:start + length].copy_(host, non_blocking=True)


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
    at t = 0). Inputs are pinned host tensors drawn like the synthetic states.
    With ``shared``, requests view consecutive ranges of one pinned ring (inputs
    and outputs; a request that does not fit before the ring's end starts over
    at its beginning), which bounds host memory for long benchmark streams:
    like a receive ring, requests far apart in the stream share memory."""
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
        ring = int(8 * max_chains * robot_lengths.max())
        q, qd, tau = synth.make_state([ring], seed=seed, cfg=4)
        pool = [torch.from_numpy(a).to(tdt).pin_memory() for a in (q, qd, tau)]
        pool.append(torch.empty(ring, dtype=tdt).pin_memory())
    pos = 0
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
            if pos + k > len(pool[0]):
                pos = 0
            r.q, r.qd, r.tau, r.out = (t[pos:pos + k] for t in pool)
            pos += k
        reqs.append(r)
    return reqs


def spin_idle(seconds):
    """Idle hook for a real device: sleep only while waiting for a distant arrival."""
    if seconds is not None and seconds > 2e-4:
        time.sleep(min(seconds, 1e-3) - 1e-4)
