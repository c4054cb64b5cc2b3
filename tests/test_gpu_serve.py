"""Serving on the GPU: every request's result is the same alone and inside the
continuous-batching mix (bit for bit with one lane per chain), and matches
the oracle, also when the requests of one round use different algorithms."""
import numpy as np
import pytest

import oracle
from _errmodel import CAP
from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_served_results_equal_alone_and_oracle(dev):
    from paper_1609_06779_amd import fd, serve

    lengths = synth.ragged_lengths(32, 7, 200, cfg=4)
    robots = synth.make_robots(lengths, cfg=4)
    model = fd.Model(robots, "f64", device=dev)
    reqs = serve.make_requests(lengths, count=60, qps=20000.0, seed=7, max_chains=512)
    ex = serve.GpuExecutor(model, lengths, algo="abia", streams=4)
    sched = serve.Scheduler(ex, budget_bytes=64 << 20, max_inflight=4, idle=serve.spin_idle)
    stats = sched.run(reqs)
    assert stats.completed == 60 and stats.rejected == 0 and stats.launches >= 2
    for r in reqs[::7]:
        # the robots differ in length, so a batch names its chains' offsets
        offsets = torch.arange(0, (r.chains + 1) * r.n, r.n, dtype=torch.int64, device=dev)
        alone = model.forward(r.q.to(dev), r.qd.to(dev), r.tau.to(dev), batch=r.chains, algo="abia",
                              robot_id=torch.full((r.chains,), r.robot, dtype=torch.int32, device=dev),
                              offsets=offsets).cpu()
        assert torch.equal(alone, r.out), r.rid
        per_chain = robots.take(np.full(r.chains, r.robot))
        ref = oracle.fd_exact(per_chain, r.q.numpy(), r.qd.numpy(), r.tau.numpy())
        err = oracle.relative_error(r.out.numpy(), ref, per_chain.offsets)
        assert np.all(err <= CAP["f64"]), (r.rid, err.max())


def test_launches_overlap_and_results_do_not_depend_on_the_mix(dev):
    """A burst of requests (all present at once) with at most 512 chains per
    launch: the loop issues several launches before the first one retires, so
    requests are admitted while earlier ones are still on the device; every
    result equals the request served alone, bit for bit (ABIA)."""
    from paper_1609_06779_amd import fd, serve

    lengths = synth.ragged_lengths(32, 7, 200, cfg=4)
    robots = synth.make_robots(lengths, cfg=4)
    model = fd.Model(robots, "f64", device=dev)
    reqs = serve.make_requests(lengths, count=40, qps=float("inf"), seed=12, max_chains=256)
    ex = serve.GpuExecutor(model, lengths, algo="abia", streams=4, slots=4)
    stats = serve.Scheduler(ex, budget_bytes=256 << 20, max_inflight=4, max_chains_per_launch=512,
                            idle=serve.spin_idle).run(reqs)
    assert stats.completed == 40 and stats.launches >= 4
    assert stats.max_inflight >= 2, stats.max_inflight
    overlapped = [(a.rid, b.rid) for a in reqs for b in reqs if a.admitted < b.admitted < a.done]
    assert overlapped, "no request was admitted while an earlier launch was still running"
    assert ex.timing["launches"] == stats.launches and ex.timing["kernel_ms"] > 0
    for r in reqs[::5]:
        offsets = torch.arange(0, (r.chains + 1) * r.n, r.n, dtype=torch.int64, device=dev)
        alone = model.forward(r.q.to(dev), r.qd.to(dev), r.tau.to(dev), batch=r.chains, algo="abia",
                              robot_id=torch.full((r.chains,), r.robot, dtype=torch.int32, device=dev),
                              offsets=offsets).cpu()
        assert torch.equal(alone, r.out), r.rid


def test_budget_rejects_a_request_larger_than_the_device_budget(dev):
    from paper_1609_06779_amd import fd, serve

    lengths = np.array([50, 20], np.int32)
    model = fd.Model(synth.make_robots(lengths, cfg=4), "f64", device=dev)
    reqs = serve.make_requests(lengths, count=6, qps=float("inf"), seed=8, max_chains=2000)
    ex = serve.GpuExecutor(model, lengths)
    small = min(ex.bytes_needed([r]) for r in reqs)
    big = max(ex.bytes_needed([r]) for r in reqs)
    sched = serve.Scheduler(ex, budget_bytes=(small + big) // 2, max_inflight=2, idle=serve.spin_idle)
    stats = sched.run(reqs)
    assert stats.rejected >= 1 and stats.completed + stats.rejected == 6
    for r in reqs:
        if not r.rejected:
            assert torch.isfinite(r.out).all()


@pytest.mark.parametrize("mode", ["mixed", "auto"])
def test_rounds_with_several_algorithms_match_the_oracle(dev, mode):
    """Requests served by all three algorithms in the same rounds (cycled by request
    id), or by the AUTO choice for each round's whole batch, match the oracle on
    sampled chains."""
    from paper_1609_06779_amd import fd, serve

    lengths = synth.ragged_lengths(32, 7, 200, cfg=4)
    robots = synth.make_robots(lengths, cfg=4)
    model = fd.Model(robots, "f64", device=dev)
    reqs = serve.make_requests(lengths, count=48, qps=20000.0, seed=11, max_chains=256)
    algo = (lambda r: ("abia", "jsiia", "cfa")[r.rid % 3]) if mode == "mixed" else "auto"
    ex = serve.GpuExecutor(model, lengths, algo=algo, streams=4)
    stats = serve.Scheduler(ex, budget_bytes=64 << 20, max_inflight=4, idle=serve.spin_idle).run(reqs)
    assert stats.completed == 48 and stats.rejected == 0
    used = {r.algo for r in reqs}
    if mode == "mixed":
        assert used == {"abia", "jsiia", "cfa"} or used == {"abia", "cfa"}   # JSIIA gives way past 128 links
    for r in reqs:
        pick = np.unique(np.minimum([0, r.chains // 2, r.chains - 1], r.chains - 1))
        sub = robots.take(np.full(len(pick), r.robot))
        idx = np.concatenate([np.arange(r.n * b, r.n * b + r.n) for b in pick])
        q, qd, tau = (x.numpy()[idx] for x in (r.q, r.qd, r.tau))
        ref = oracle.fd_exact(sub, q, qd, tau)
        err = oracle.relative_error(r.out.numpy()[idx], ref, sub.offsets)
        assert np.all(err <= CAP["f64"]), (r.rid, r.algo, r.n, err.max())


def test_serving_branched_robots_runs_the_tree_kernels(dev):
    """A model of branched robots: requests the tuned table gives to the CFA
    (serial chains only) go to the articulated-body kernel instead; every
    request matches the oracle."""
    from paper_1609_06779_amd import fd, serve

    lengths = synth.ragged_lengths(16, 7, 120, seed=3, cfg=5)
    robots = synth.make_tree_robots(lengths, cfg=5, random_home=True)
    model = fd.Model(robots, "f64", device=dev)
    assert model.branched
    reqs = serve.make_requests(lengths, count=24, qps=20000.0, seed=5, max_chains=256)
    ex = serve.GpuExecutor(model, lengths, algo="auto", streams=2)
    stats = serve.Scheduler(ex, budget_bytes=64 << 20, max_inflight=2, idle=serve.spin_idle).run(reqs)
    assert stats.completed == 24 and stats.rejected == 0
    assert "abia" in {r.algo for r in reqs} and {r.algo for r in reqs} <= {"abia", "jsiia"}
    for r in reqs[::3]:
        pick = np.unique(np.minimum([0, r.chains // 2, r.chains - 1], r.chains - 1))
        sub = robots.take(np.full(len(pick), r.robot))
        idx = np.concatenate([np.arange(r.n * b, r.n * b + r.n) for b in pick])
        q, qd, tau = (x.numpy()[idx] for x in (r.q, r.qd, r.tau))
        err = oracle.relative_error(r.out.numpy()[idx], oracle.fd_exact(sub, q, qd, tau), sub.offsets)
        assert np.all(err <= CAP["f64"]), (r.rid, err.max())
