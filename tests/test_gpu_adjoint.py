"""GPU parity of the reverse-mode derivative (fd_backward) and of the
checkpointed rollout gradient, against the oracle's complex-step JVPs
(exact to rounding) and central differences of the oracle.

The adjoint identity <VJP(g), v> = <g, JVP(v)> is checked per chain for
random cotangents g and directions v = (dq, dqd, dtau), and the gradients
entry by entry against the oracle's full Jacobian. Every bar is the cap of the
forward parity tests (1e-9 FP64, 1e-3 FP32), relative to the scale of the
compared quantity."""
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


@pytest.fixture(scope="module")
def fdm():
    from paper_1609_06779_amd import fd
    return fd


def _t(a, dev, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, dtype)


def _chain_sums(x, off):
    return np.add.reduceat(x, off[:-1])


@pytest.mark.parametrize("n", [1, 2, 5, 16, 32, 64, 100])
def test_vjp_adjoint_identity(fdm, dev, n):
    batch = 9
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5, random_home=True)
    q, qd, tau = synth.make_state(lengths, cfg=5)
    off = rb.offsets
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo="abia")
    rng = np.random.default_rng(n)
    ms = oracle.crba(rb, q)
    for _ in range(3):
        g = rng.standard_normal(len(q))
        gq, gqd, gtau = (x.cpu().numpy() for x in model.backward(tq, tqd, qdd, _t(g, dev), batch=batch))
        # tau_bar = M^-1 g
        for b in range(batch):
            sl = slice(off[b], off[b + 1])
            ref = np.linalg.solve(ms[b], g[sl])
            assert np.linalg.norm(gtau[sl] - ref) <= CAP["f64"] * np.linalg.norm(ref), (b, "tau_bar")
        dq, dqd, dtau = (rng.standard_normal(len(q)) for _ in range(3))
        _, dqdd = oracle.fd_jvp(rb, q, qd, tau, dq, dqd, dtau)
        lhs = _chain_sums(g * dqdd, off)
        rhs = _chain_sums(gq * dq + gqd * dqd + gtau * dtau, off)
        scale = _chain_sums(np.abs(g * dqdd), off) + _chain_sums(np.abs(gq * dq) + np.abs(gqd * dqd) +
                                                                 np.abs(gtau * dtau), off)
        assert np.all(np.abs(lhs - rhs) <= CAP["f64"] * scale), (np.abs(lhs - rhs) / scale).max()


def test_vjp_accumulates_and_matches_autograd_function(fdm, dev):
    lengths = np.full(6, 12, np.int32)
    rb = synth.make_robots(lengths, cfg=5)
    q, qd, tau = synth.make_state(lengths, cfg=5)
    model = fdm.Model(rb, "f64", device=dev)
    tq = _t(q, dev).requires_grad_(True)
    tqd = _t(qd, dev).requires_grad_(True)
    ttau = _t(tau, dev).requires_grad_(True)
    qdd = fdm.forward_dynamics(model, tq, tqd, ttau, batch=6, algo="cfa")
    g = torch.randn_like(qdd)
    (qdd * g).sum().backward()
    # the autograd function differentiates through the algorithm that gave qdd
    gq, gqd, gtau = model.backward(tq.detach(), tqd.detach(), qdd.detach(), g, batch=6, algo="cfa")
    assert torch.equal(tq.grad, gq) and torch.equal(tqd.grad, gqd) and torch.equal(ttau.grad, gtau)
    a, b_, c = (x.clone() for x in (gq, gqd, gtau))
    model.backward(tq.detach(), tqd.detach(), qdd.detach(), g, batch=6, algo="cfa", grad_q=a, grad_qd=b_,
                   grad_tau=c, accumulate=True)
    assert torch.allclose(a, 2 * gq, rtol=1e-15, atol=0) and torch.allclose(c, 2 * gtau, rtol=1e-15, atol=0)


def _oracle_rollout(rb, q, qd, taus, dt, dq=None, dqd=None, dtaus=None):
    """(q_T, qd_T) and, with directions, their derivatives (complex-step JVP each step)."""
    q, qd = q.copy(), qd.copy()
    tq = None if dq is None else dq.copy()
    tqd = None if dqd is None else dqd.copy()
    for t in range(taus.shape[0]):
        if tq is None:
            qdd = oracle.fd(rb, q, qd, taus[t])
        else:
            qdd, dqdd = oracle.fd_jvp(rb, q, qd, taus[t], tq, tqd, dtaus[t])
            tqd = tqd + dt * dqdd
            tq = tq + dt * tqd
        qd = qd + dt * qdd
        q = q + dt * qd
    return q, qd, tq, tqd


@pytest.mark.parametrize("algo", ["abia", "cfa"])
def test_rollout_gradient_matches_oracle(fdm, dev, algo):
    """100 semi-implicit Euler steps, dt = 1e-3, loss = sum(q_T^2 + qd_T^2), gradient
    with respect to q_0, qd_0 and every tau_t, checkpoints every 10 steps."""
    batch, n, steps, dt = 24, 32, 100, 1e-3
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5)
    q0, qd0, _ = synth.make_state(lengths, cfg=5)
    taus = np.random.default_rng(5).standard_normal((steps, len(q0)))
    off = rb.offsets
    model = fdm.Model(rb, "f64", device=dev)
    tq0 = _t(q0, dev).requires_grad_(True)
    tqd0 = _t(qd0, dev).requires_grad_(True)
    ttaus = _t(taus, dev).requires_grad_(True)
    qt, qdt = fdm.rollout(model, tq0, tqd0, ttaus, batch=batch, dt=dt, every=10, algo=algo)
    loss = (qt ** 2).sum() + (qdt ** 2).sum()
    loss.backward()
    g0, gd0, gt = tq0.grad.cpu().numpy(), tqd0.grad.cpu().numpy(), ttaus.grad.cpu().numpy()
    rq, rqd, _, _ = _oracle_rollout(rb, q0, qd0, taus, dt)
    np.testing.assert_allclose(qt.detach().cpu().numpy(), rq, rtol=0, atol=1e-10 * (1 + np.abs(rq).max()))
    bar = np.full(batch, CAP["f64"])
    rng = np.random.default_rng(55)
    h = 1e-6
    for _ in range(32):                            # random directions (dq_0, dqd_0, dtau_0..T-1)
        dq, dqd = rng.standard_normal(len(q0)), rng.standard_normal(len(q0))
        dtaus = rng.standard_normal(taus.shape)
        _, _, tq, tqd = _oracle_rollout(rb, q0, qd0, taus, dt, dq, dqd, dtaus)
        # per chain: dL = 2 q_T . dq_T + 2 qd_T . dqd_T (complex-step JVP of the oracle)
        exact = _chain_sums(2 * rq * tq + 2 * rqd * tqd, off)
        terms = g0 * dq + gd0 * dqd + (gt * dtaus).sum(axis=0)
        ours = _chain_sums(terms, off)
        # a sum of products with per-entry relative error e is off by at most
        # e * sum |products|, the scale the adjoint identity above uses too
        scale = _chain_sums(np.abs(g0 * dq) + np.abs(gd0 * dqd) + np.abs(gt * dtaus).sum(axis=0), off)
        ratio = np.abs(ours - exact) / (bar * (1 + np.maximum(np.abs(exact), scale)))
        assert np.all(ratio <= 1.0), (ratio.max(), int(ratio.argmax()))
        # central differences of the oracle's loss along the same direction, whole batch
        lp = sum(np.sum(x ** 2) for x in _oracle_rollout(rb, q0 + h * dq, qd0 + h * dqd, taus + h * dtaus, dt)[:2])
        lm = sum(np.sum(x ** 2) for x in _oracle_rollout(rb, q0 - h * dq, qd0 - h * dqd, taus - h * dtaus, dt)[:2])
        fd_dir = (lp - lm) / (2 * h)
        assert abs(ours.sum() - fd_dir) <= 1e-6 * max(1.0, abs(fd_dir)), (ours.sum(), fd_dir)


def test_rollout_full_size_sampled(fdm, dev):
    """16384 chains of 32 links, 100 steps: gradient of sampled chains against the oracle."""
    batch, n, steps, dt = 16384, 32, 100, 1e-3
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5)
    q0, qd0, _ = synth.make_state(lengths, cfg=5)
    taus = np.random.default_rng(6).standard_normal((steps, len(q0)))
    model = fdm.Model(rb, "f64", device=dev)
    tq0 = _t(q0, dev).requires_grad_(True)
    tqd0 = _t(qd0, dev).requires_grad_(True)
    ttaus = _t(taus, dev).requires_grad_(True)
    qt, qdt = fdm.rollout(model, tq0, tqd0, ttaus, batch=batch, dt=dt, every=10, algo="abia")
    ((qt ** 2).sum() + (qdt ** 2).sum()).backward()
    g0, gd0, gt = tq0.grad.cpu().numpy(), tqd0.grad.cpu().numpy(), ttaus.grad.cpu().numpy()
    assert np.all(np.isfinite(g0)) and np.all(np.isfinite(gt))
    pick = np.array([0, 777, 8191, 16383])
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(n * b, n * b + n) for b in pick])
    rng = np.random.default_rng(66)
    dq, dqd = rng.standard_normal(len(idx)), rng.standard_normal(len(idx))
    dtaus = rng.standard_normal((steps, len(idx)))
    rq, rqd, tq, tqd = _oracle_rollout(sub, q0[idx], qd0[idx], taus[:, idx], dt, dq, dqd, dtaus)
    off = sub.offsets
    exact = _chain_sums(2 * rq * tq + 2 * rqd * tqd, off)
    ours = _chain_sums(g0[idx] * dq + gd0[idx] * dqd + (gt[:, idx] * dtaus).sum(axis=0), off)
    scale = _chain_sums(np.abs(g0[idx] * dq) + np.abs(gd0[idx] * dqd) + np.abs(gt[:, idx] * dtaus).sum(axis=0), off)
    assert np.all(np.abs(ours - exact) <= 1e-10 * (1 + np.maximum(np.abs(exact), scale))), np.abs(ours - exact).max()


def test_vjp_full_size_streaming_sampled(fdm, dev):
    """65536 chains of 64 links: the launch outgrows the last-level cache, so the
    kernel streams its model and workspace. Sampled chains against the oracle
    through the adjoint identity, tau_bar against a dense solve, all finite."""
    batch, n = 65536, 64
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=2)
    q, qd, tau = synth.make_state(lengths, cfg=2)
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo="abia")
    g = np.random.default_rng(21).standard_normal(len(q))
    gq, gqd, gtau = (x.cpu().numpy() for x in model.backward(tq, tqd, qdd, _t(g, dev), batch=batch))
    assert np.all(np.isfinite(gq)) and np.all(np.isfinite(gqd)) and np.all(np.isfinite(gtau))
    pick = np.array([0, 1, 12345, 40000, 65535])
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(n * b, n * b + n) for b in pick])
    off = sub.offsets
    ms = oracle.crba(sub, q[idx])
    for k in range(len(pick)):
        sl = slice(off[k], off[k + 1])
        ref = np.linalg.solve(ms[k], g[idx][sl])
        assert np.linalg.norm(gtau[idx][sl] - ref) <= CAP["f64"] * np.linalg.norm(ref), (pick[k], "tau_bar")
    rng = np.random.default_rng(22)
    dq, dqd, dtau = (rng.standard_normal(len(idx)) for _ in range(3))
    _, dqdd = oracle.fd_jvp(sub, q[idx], qd[idx], tau[idx], dq, dqd, dtau)
    lhs = _chain_sums(g[idx] * dqdd, off)
    rhs = _chain_sums(gq[idx] * dq + gqd[idx] * dqd + gtau[idx] * dtau, off)
    scale = _chain_sums(np.abs(g[idx] * dqdd), off) + _chain_sums(
        np.abs(gq[idx] * dq) + np.abs(gqd[idx] * dqd) + np.abs(gtau[idx] * dtau), off)
    assert np.all(np.abs(lhs - rhs) <= CAP["f64"] * scale), (np.abs(lhs - rhs) / scale).max()


@pytest.mark.parametrize("algo", ["abia", "jsiia"])
def test_vjp_large_launch_matches_smaller_launches_every_chain(fdm, dev, algo):
    """A launch of 65536 chains of 64 links outgrows the last-level cache and moves
    the joint state and its adjoints through LDS tiles; launches of 16384 of the
    same chains (by robot id) do not. Every entry of both agrees, for the plain
    and the accumulating form, so no chain of a tile is misplaced. With JSIIA's
    lambda the reverse-mode kernel skips its own M^-1 sweep."""
    batch, n, part = 65536, 64, 16384
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=2)
    q, qd, tau = synth.make_state(lengths, cfg=2)
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo="abia")
    g = _t(np.random.default_rng(23).standard_normal(len(q)), dev)
    big = [x.cpu().numpy() for x in model.backward(tq, tqd, qdd, g, batch=batch, algo=algo)]
    base = [_t(np.random.default_rng(24 + k).standard_normal(len(q)), dev) for k in range(3)]
    acc = [x.clone() for x in base]
    model.backward(tq, tqd, qdd, g, batch=batch, algo=algo, grad_q=acc[0], grad_qd=acc[1], grad_tau=acc[2],
                   accumulate=True)
    small = [np.empty(len(q)) for _ in range(3)]
    small_acc = [x.clone() for x in base]
    for s0 in range(0, batch, part):
        sl = slice(s0 * n, (s0 + part) * n)
        rid = torch.arange(s0, s0 + part, dtype=torch.int32, device=dev)
        outs = model.backward(tq[sl], tqd[sl], qdd[sl], g[sl], batch=part, algo=algo, robot_id=rid)
        for k in range(3):
            small[k][sl] = outs[k].cpu().numpy()
        model.backward(tq[sl], tqd[sl], qdd[sl], g[sl], batch=part, algo=algo, robot_id=rid, grad_q=small_acc[0][sl],
                       grad_qd=small_acc[1][sl], grad_tau=small_acc[2][sl], accumulate=True)
    for k, name in enumerate(("q_bar", "qd_bar", "tau_bar")):
        a, b = big[k].reshape(batch, n), small[k].reshape(batch, n)
        scale = 1 + np.abs(b).max(axis=1, keepdims=True)
        assert np.all(np.abs(a - b) <= 1e-11 * scale), (name, np.abs(a - b).max())
        a, b = acc[k].cpu().numpy().reshape(batch, n), small_acc[k].cpu().numpy().reshape(batch, n)
        scale = 1 + np.abs(b).max(axis=1, keepdims=True)
        assert np.all(np.abs(a - b) <= 1e-11 * scale), (name, "accumulate", np.abs(a - b).max())


@pytest.mark.parametrize("tree", [False, True])
@pytest.mark.parametrize("n", [5, 16, 32])
def test_vjp_fp32(fdm, dev, n, tree):
    """fd_backward in FP32 (robots and states rounded to FP32 first, the oracle in
    FP64 on the rounded values): tau_bar against a dense solve and the adjoint
    identity, within the FP32 cap."""
    batch = 12
    lengths = np.full(batch, n, np.int32)
    if tree:
        rb = synth.make_tree_robots(lengths, seed=40 + n, cfg=5, random_home=True)
    else:
        rb = synth.make_robots(lengths, cfg=5, random_home=True)
    rb = rb.astype_rounded(np.float32)
    q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in synth.make_state(lengths, cfg=5))
    off = rb.offsets
    model = fdm.Model(rb, "f32", device=dev)
    f32 = torch.float32
    tq, tqd, ttau = _t(q, dev, f32), _t(qd, dev, f32), _t(tau, dev, f32)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo="abia")
    rng = np.random.default_rng(n)
    g = rng.standard_normal(len(q)).astype(np.float32).astype(np.float64)
    gq, gqd, gtau = (x.cpu().numpy().astype(np.float64) for x in model.backward(tq, tqd, qdd, _t(g, dev, f32),
                                                                                batch=batch))
    ms = oracle.crba(rb, q)
    for b in range(batch):
        sl = slice(off[b], off[b + 1])
        ref = np.linalg.solve(ms[b], g[sl])
        assert np.linalg.norm(gtau[sl] - ref) <= CAP["f32"] * np.linalg.norm(ref), (b, "tau_bar")
    dq, dqd, dtau = (rng.standard_normal(len(q)) for _ in range(3))
    _, dqdd = oracle.fd_jvp(rb, q, qd, tau, dq, dqd, dtau)
    lhs = _chain_sums(g * dqdd, off)
    rhs = _chain_sums(gq * dq + gqd * dqd + gtau * dtau, off)
    scale = _chain_sums(np.abs(g * dqdd), off) + _chain_sums(np.abs(gq * dq) + np.abs(gqd * dqd) +
                                                             np.abs(gtau * dtau), off)
    assert np.all(np.abs(lhs - rhs) <= CAP["f32"] * scale), (np.abs(lhs - rhs) / scale).max()


# ---------------- element-wise parity of the reverse mode ----------------

def _oracle_jacobian(rb, q, qd, tau, n):
    """d qdd / d(q, qd, tau) of every chain of a uniform batch of n-link chains,
    column by column from 3 n complex-step JVPs of the oracle along unit
    directions (exact to rounding): [batch, n, 3 n]."""
    batch = len(q) // n
    jac = np.empty((batch, n, 3 * n))
    zero = np.zeros(len(q))
    for blk in range(3):
        for k in range(n):
            e = np.zeros(len(q))
            e[k::n] = 1.0
            d = [zero, zero, zero]
            d[blk] = e
            _, dqdd = oracle.fd_jvp(rb, q, qd, tau, *d)
            jac[:, :, blk * n + k] = dqdd.reshape(batch, n)
    return jac


def _check_elementwise(got, ref, scale, dtype, what):
    """Each entry of each chain's gradient block within CAP times `scale`, the
    chain's largest gradient entry over (q_bar, qd_bar, tau_bar). A block can be
    zero in exact arithmetic (qd_bar of one link: no velocity product about a
    fixed axis), so entries are judged on the whole gradient's scale."""
    from _errmodel import CAP, TARGET
    err = np.abs(got - ref).max(axis=-1) / np.maximum(scale, np.finfo(float).tiny)
    worst = float(err.max())
    print(f"{what}: worst entry error {worst:.2e} of the block scale; "
          f"{int(np.sum(err <= TARGET[dtype]))} of {err.size} blocks within {TARGET[dtype]:g}", flush=True)
    assert worst <= CAP[dtype], f"{what}: {worst:.3e} above the cap {CAP[dtype]:g}"


def _elementwise_cases():
    for n in (1, 2, 7, 16, 33, 64):
        for algo in ("abia", "jsiia", "cfa", "abia_scan"):
            marks = ()
            if (n, algo) == (64, "cfa"):
                # measured 2.2e-8 on q_bar: the CFA's lambda = M^-1 g carries its
                # Schur-complement error (C - B^T A^-1 B, eq. (fijany-final)), and
                # q_bar = -(d ID / d q)^T lambda multiplies it by the gravity and
                # velocity terms of d ID / d q
                marks = pytest.mark.xfail(strict=True, reason="CFA reverse mode at n=64: q_bar over the 1e-9 cap")
            yield pytest.param(n, algo, marks=marks, id=f"{n}-{algo}")


@pytest.mark.parametrize("n,algo", list(_elementwise_cases()))
def test_vjp_elementwise_against_oracle_jacobian(fdm, dev, n, algo):
    """q_bar, qd_bar and tau_bar of fd_backward, entry by entry, against J^T g with
    J = d qdd / d(q, qd, tau) from the oracle (FP64), lambda = M^-1 g by `algo`."""
    batch = 8
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5, random_home=True)
    q, qd, tau = synth.make_state(lengths, cfg=5)
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo=algo)
    g = np.random.default_rng(100 + n).standard_normal(len(q))
    gq, gqd, gtau = (x.cpu().numpy().reshape(batch, n) for x in
                     model.backward(tq, tqd, qdd, _t(g, dev), batch=batch, algo=algo))
    jac = _oracle_jacobian(rb, q, qd, tau, n)
    ref = np.einsum("bij,bi->bj", jac, g.reshape(batch, n))
    scale = np.abs(ref).max(axis=-1)
    _check_elementwise(gq, ref[:, :n], scale, "f64", f"{algo} n={n} q_bar")
    _check_elementwise(gqd, ref[:, n:2 * n], scale, "f64", f"{algo} n={n} qd_bar")
    _check_elementwise(gtau, ref[:, 2 * n:], scale, "f64", f"{algo} n={n} tau_bar")


@pytest.mark.parametrize("algo", ["abia", "jsiia", "cfa", "abia_scan"])
def test_vjp_recomputes_qdd_from_tau(fdm, dev, algo):
    """fd_backward with qdd = NULL computes qdd from (q, qd, tau) by the same
    kernel first: the gradients equal those given that kernel's qdd, bit for bit;
    accumulate adds onto the given arrays."""
    batch, n = 70, 20                               # two 64-chain blocks, the second ragged
    lengths = np.full(batch, n, np.int32)
    rb = synth.make_robots(lengths, cfg=5)
    q, qd, tau = synth.make_state(lengths, cfg=5)
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    g = _t(np.random.default_rng(7).standard_normal(len(q)), dev)
    qdd = model.forward(tq, tqd, ttau, batch=batch, algo=algo)
    given = model.backward(tq, tqd, qdd, g, batch=batch, algo=algo)
    recomputed = model.backward(tq, tqd, None, g, batch=batch, algo=algo, tau=ttau)
    for a, b in zip(given, recomputed):
        assert torch.equal(a, b), algo
    acc = [x.clone() for x in given]
    model.backward(tq, tqd, None, g, batch=batch, algo=algo, tau=ttau, grad_q=acc[0], grad_qd=acc[1],
                   grad_tau=acc[2], accumulate=True)
    for a, b in zip(acc, given):
        assert torch.allclose(a, 2 * b, rtol=1e-15, atol=0), algo


def test_vjp_ragged_batch_with_every_algorithm(fdm, dev):
    """A ragged batch (offsets, robot ids) through every algorithm's lambda:
    tau_bar = M^-1 g against a dense solve of the oracle's M on every chain."""
    from _errmodel import CAP
    base_lengths = np.array([1, 5, 17, 40, 64], np.int32)
    base = synth.make_robots(base_lengths, cfg=4, random_home=True)
    rid = np.random.default_rng(8).integers(0, len(base_lengths), size=90).astype(np.int32)
    sub = base.take(rid)
    q, qd, tau = synth.make_state(sub.n_links, cfg=4)
    off = sub.offsets
    model = fdm.Model(base, "f64", device=dev)
    tq, tqd, ttau = _t(q, dev), _t(qd, dev), _t(tau, dev)
    toff, trid = torch.from_numpy(off).to(dev), torch.from_numpy(rid).to(dev)
    g = np.random.default_rng(9).standard_normal(len(q))
    ms = oracle.crba(sub, q, offsets=off)
    for algo in ("abia", "jsiia", "cfa", "abia_scan", "cfa_proj"):
        _, _, gtau = model.backward(tq, tqd, None, _t(g, dev), batch=len(rid), algo=algo, tau=ttau,
                                    offsets=toff, robot_id=trid)
        gtau = gtau.cpu().numpy()
        for b, m in enumerate(ms):
            sl = slice(off[b], off[b + 1])
            ref = np.linalg.solve(m, g[sl])
            assert np.linalg.norm(gtau[sl] - ref) <= CAP["f64"] * np.linalg.norm(ref), (algo, b)
