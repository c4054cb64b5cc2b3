"""A rollout recorded into a HIP graph (fd.RolloutGraph) against the same
rollout launched step by step: every replay, with eager work and
synchronisations between the replays, gives the eager result bit for bit
(the kernels are deterministic), and the eager result matches the oracle."""
import numpy as np
import pytest

import oracle
from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _eager(model, q, qd, taus, batch, dt, algo):
    q, qd = q.clone(), qd.clone()
    qdd = torch.empty_like(q)
    for t in range(taus.shape[0]):
        model.forward(q, qd, taus[t], batch=batch, algo=algo, out=qdd)
        model.euler_step(q, qd, qdd, dt, q_next=q, qd_next=qd)
    return q, qd


@pytest.mark.parametrize("algo", ["abia", "jsiia", "cfa"])
def test_recorded_rollout_replays_equal_the_eager_rollout(dev, algo):
    from paper_1609_06779_amd import fd

    batch, n, steps, dt = 48, 12, 25, 1e-3
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5, random_home=True)
    model = fd.Model(rb, "f64", device=dev)
    g = fd.RolloutGraph(model, batch, steps, dt, algo=algo)
    for rep in range(3):                                   # new inputs each replay
        q0, qd0, _ = synth.make_state(lengths, seed=100 + rep, cfg=5)
        taus = np.random.default_rng(rep).standard_normal((steps, len(q0)))
        tq0, tqd0, ttaus = (torch.from_numpy(a).to(dev) for a in (q0, qd0, taus))
        qe, qde = _eager(model, tq0, tqd0, ttaus, batch, dt, algo)
        torch.cuda.synchronize()
        qg, qdg = g.run(tq0, tqd0, ttaus)
        assert torch.equal(qg, qe) and torch.equal(qdg, qde), rep
        torch.cuda.synchronize()
        if rep == 0:                                       # the eager path against the oracle
            q, qd = q0.copy(), qd0.copy()
            for t in range(steps):
                qd = qd + dt * oracle.fd(rb, q, qd, taus[t])
                q = q + dt * qd
            np.testing.assert_allclose(qe.cpu().numpy(), q, rtol=0, atol=1e-10 * (1 + np.abs(q).max()))
            np.testing.assert_allclose(qde.cpu().numpy(), qd, rtol=0, atol=1e-10 * (1 + np.abs(qd).max()))


def test_recorded_rollout_rejects_auto_and_ragged_without_size(dev):
    from paper_1609_06779_amd import fd

    rb = synth.make_robots([5, 7], cfg=5)
    model = fd.Model(rb, "f64", device=dev)
    with pytest.raises(ValueError):
        fd.RolloutGraph(model, 2, 3, 1e-3, algo="auto")
    off = torch.from_numpy(rb.offsets).to(dev)
    with pytest.raises(ValueError):
        fd.RolloutGraph(model, 2, 3, 1e-3, algo="abia", offsets=off)
