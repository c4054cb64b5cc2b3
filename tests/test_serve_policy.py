"""Serving policy on a simulated device (no GPU): admission by memory budget,
continuous batching, rejection of oversized requests, FIFO order and
deterministic latency accounting under a simulated clock."""
import numpy as np

from paper_1609_06779_amd.serve import Executor, Request, Scheduler, poisson_arrivals, request_sizes


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class SimDevice(Executor):
    """Each launch takes fixed + per_chain * chains seconds; it runs as soon as it is issued."""

    def __init__(self, clock, fixed=1e-4, per_chain=1e-6, bytes_per_chain=1000):
        self.clock = clock
        self.fixed = fixed
        self.per_chain = per_chain
        self.bpc = bytes_per_chain
        self.inflight = {}
        self.log = []
        self.used = 0
        self.peak_used = 0
        self.next_id = 0

    def bytes_needed(self, reqs):
        return self.bpc * sum(r.chains for r in reqs)

    def launch(self, reqs):
        h = self.next_id
        self.next_id += 1
        end = self.clock.t + self.fixed + self.per_chain * sum(r.chains for r in reqs)
        self.inflight[h] = (end, self.bytes_needed(reqs))
        self.used += self.bytes_needed(reqs)
        self.peak_used = max(self.peak_used, self.used)
        self.log.append((self.clock.t, [r.rid for r in reqs]))
        return h

    def poll(self, h):
        return self.clock.t >= self.inflight[h][0]

    def retire(self, h):
        self.used -= self.inflight.pop(h)[1]

    def next_completion(self):
        return min((e for e, _ in self.inflight.values()), default=None)


def _run(reqs, budget, max_inflight=4, max_chains=65536):
    clock = SimClock()
    dev = SimDevice(clock)

    def idle(until_arrival):
        cands = [clock.t + max(until_arrival, 0.0)] if until_arrival is not None else []
        nc = dev.next_completion()
        if nc is not None:
            cands.append(nc)
        clock.t = max(clock.t, min(cands)) if cands else clock.t + 1e-6

    sched = Scheduler(dev, budget, max_inflight=max_inflight, max_chains_per_launch=max_chains, clock=clock, idle=idle)
    stats = sched.run(reqs)
    return stats, dev


def _reqs(sizes, arrivals):
    return [Request(rid=i, robot=i % 3, chains=int(c), n=10, arrival=float(a)) for i, (c, a) in
            enumerate(zip(sizes, arrivals))]


def test_budget_bounds_memory_in_flight_and_fifo():
    reqs = _reqs([100] * 20, [0.0] * 20)
    stats, dev = _run(reqs, budget=100 * 1000 * 3, max_inflight=8)
    assert stats.completed == 20 and stats.rejected == 0
    assert dev.peak_used <= 300_000
    order = [rid for _, rids in dev.log for rid in rids]
    assert order == list(range(20))                       # admitted in arrival order
    # every launch packs as many queued requests as fit the free budget
    assert all(len(rids) <= 3 for _, rids in dev.log)


def test_oversized_request_rejected_others_served():
    reqs = _reqs([10, 5000, 10], [0.0, 0.0, 0.0])
    stats, _ = _run(reqs, budget=1_000_000)
    assert reqs[1].rejected and not reqs[0].rejected and not reqs[2].rejected
    assert stats.completed == 2 and stats.rejected == 1


def test_continuous_batching_admits_while_busy():
    # a long launch starts at t = 0; later arrivals are admitted before it ends
    reqs = _reqs([50000, 10, 10], [0.0, 0.001, 0.002])
    stats, dev = _run(reqs, budget=10**9, max_inflight=4)
    first_end = 1e-4 + 1e-6 * 50000
    starts = [t for t, _ in dev.log]
    assert len(dev.log) == 3 and starts[1] < first_end and starts[2] < first_end
    assert reqs[1].done < reqs[0].done                    # the short request overtakes
    assert stats.max_inflight >= 2


def test_latency_accounting_is_deterministic():
    arr = poisson_arrivals(200, qps=2000.0, seed=3)
    sizes = request_sizes(200, seed=3)
    a, _ = _run(_reqs(sizes, arr), budget=10**8)
    b, _ = _run(_reqs(sizes, arr), budget=10**8)
    assert a == b
    assert a.completed == 200 and a.p99 >= a.p50 > 0


def test_request_size_and_arrival_generators():
    s = request_sizes(10000, seed=1)
    assert s.min() >= 1 and s.max() <= 4096
    assert np.median(s) < 200 < s.mean() < 800           # log-uniform: heavy upper tail
    arr = poisson_arrivals(20000, qps=500.0, seed=1)
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 1 / 500.0) < 0.05 / 500.0 and np.all(gaps > 0)
