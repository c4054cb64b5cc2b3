"""GPU parity on branched robots (trees), through the C-ABI, against the oracle:
the articulated-body kernel's tree variant (any parent order), and the
lane-per-link kernels on trees numbered depth-first (JSIIA, inverse dynamics,
the joint-space inertia), whose scans run over root paths and subtrees.

A tree hangs link i from a parent p(i) < i (the paper treats serial chains).
The bars are those of the serial-chain parity tests: every tree's forward
error within the cap (1e-9 FP64, 1e-3 FP32: ten times the target) and a
normwise backward error of at most 64 u. FP32 runs round robots and states to
FP32 first.
"""
import numpy as np
import pytest

import oracle
from _errmodel import CAP, TARGET, U
from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BACKWARD_FACTOR = 64.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def fdm():
    from paper_1609_06779_amd import fd
    return fd


def _prep(lengths, dtype, cfg=5, seed=synth.ROOT_SEED, p_extend=0.85, random_home=True):
    rb = synth.make_tree_robots(lengths, p_extend=p_extend, seed=seed, cfg=cfg, random_home=random_home)
    q, qd, tau = synth.make_state(lengths, seed=seed, cfg=cfg)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
        q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in (q, qd, tau))
    return rb, q, qd, tau


def _t(a, dtype, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if dtype == "f64" else np.float32)).to(dev)


def _check(got, rb, q, qd, tau, off, dtype, what, backward=True):
    ref = oracle.fd_exact(rb, q, qd, tau, offsets=off)
    err = oracle.relative_error(got, ref, off)
    ms = oracle.crba(rb, q, offsets=off)
    if len(err):
        print(f"{what}: worst {err.max():.2e}, {int(np.sum(err <= TARGET[dtype]))} of {len(err)} trees within "
              f"{TARGET[dtype]:g}", flush=True)
    bad = np.nonzero(~(err <= CAP[dtype]))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} trees over the cap, worst {err.max():.3e} (tree {bad[:5]})"
    if not backward:
        return
    bias = oracle.rnea(rb, q, qd, offsets=off)
    for b, m in enumerate(ms):
        sl = slice(off[b], off[b + 1])
        eta = np.linalg.norm(m @ got[sl] - (tau[sl] - bias[sl])) / (
            np.linalg.norm(m, 2) * np.linalg.norm(got[sl]) + np.linalg.norm(tau[sl]) + np.linalg.norm(bias[sl]))
        assert eta <= BACKWARD_FACTOR * U[dtype], f"{what}: tree {b} backward error {eta:.3e}"


def _forward(m, rb, q, qd, tau, dtype, dev, algo="abia", offsets=None, robot_id=None):
    batch = len(rb.n_links) if robot_id is None else len(robot_id)
    toff = None if offsets is None else torch.from_numpy(np.asarray(offsets, np.int64)).to(dev)
    trid = None if robot_id is None else torch.from_numpy(np.asarray(robot_id, np.int32)).to(dev)
    out = m.forward(_t(q, dtype, dev), _t(qd, dtype, dev), _t(tau, dtype, dev), batch=batch, algo=algo,
                    offsets=toff, robot_id=trid)
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 7, 33, 64, 100, 256])
def test_tree_forward_uniform(fdm, dev, dtype, n):
    """96 trees of n links, each with its own topology (so lanes of one
    wavefront take different branch paths)."""
    lengths = [n] * 96
    rb, q, qd, tau = _prep(lengths, dtype, seed=100 + n)
    m = fdm.Model(rb, dtype, device=dev)
    assert m.branched or n <= 2
    got = _forward(m, rb, q, qd, tau, dtype, dev)
    _check(got, rb, q, qd, tau, rb.offsets, dtype, f"tree n={n} {dtype}")
    auto = _forward(m, rb, q, qd, tau, dtype, dev, algo="auto")   # never the CFA on a branched model
    _check(auto, rb, q, qd, tau, rb.offsets, dtype, f"tree n={n} {dtype} auto", backward=False)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_shared_topology(fdm, dev, dtype):
    """512 robots of one 64-link topology, each with its own parameters: the
    lanes of a wavefront branch at the same links."""
    lengths = [64] * 512
    rb = synth.make_tree_robots(lengths, seed=20, cfg=5, random_home=True, shared_topology=True)
    q, qd, tau = synth.make_state(lengths, seed=20, cfg=5)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
        q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in (q, qd, tau))
    m = fdm.Model(rb, dtype, device=dev)
    assert m.branched
    got = _forward(m, rb, q, qd, tau, dtype, dev)
    _check(got, rb, q, qd, tau, rb.offsets, dtype, f"shared topology {dtype}")


@pytest.mark.parametrize("p_extend", [0.0, 0.5, 0.97])
def test_tree_shapes_ragged_with_offsets(fdm, dev, p_extend):
    """Bushy (every link hangs from a random link of the current path) to
    nearly serial trees, lengths 1..200 with offsets."""
    lengths = synth.ragged_lengths(150, 1, 200, seed=7)
    rb, q, qd, tau = _prep(lengths, "f64", seed=8, p_extend=p_extend)
    m = fdm.Model(rb, "f64", device=dev)
    got = _forward(m, rb, q, qd, tau, "f64", dev, offsets=rb.offsets)
    _check(got, rb, q, qd, tau, rb.offsets, "f64", f"ragged trees p_extend={p_extend}")


def test_every_link_hung_from_the_base(fdm, dev):
    """A 'tree' of n single links on the base: each joint is a one-link robot."""
    lengths = [12] * 64
    rb, q, qd, tau = _prep(lengths, "f64", seed=9)
    rb.parent = np.full(len(rb.mass), -1, np.int32)
    m = fdm.Model(rb, "f64", device=dev)
    got = _forward(m, rb, q, qd, tau, "f64", dev)
    _check(got, rb, q, qd, tau, rb.offsets, "f64", "base-hung links")


def test_trees_and_chains_shared_by_robot_id(fdm, dev):
    """One model holding trees and serial chains; chains name robots by id."""
    lengths = np.array([40, 9, 64, 3, 25, 64, 1, 17], np.int32)
    rb = synth.make_tree_robots(lengths, seed=10, cfg=5, random_home=True)
    par = rb.parents().copy()
    off = rb.offsets
    for r in (1, 4, 6):                     # make three of them serial chains
        par[off[r]:off[r + 1]] = np.arange(lengths[r]) - 1
    rb.parent = par
    m = fdm.Model(rb, "f64", device=dev)
    rid = np.random.default_rng(11).integers(0, len(lengths), size=300).astype(np.int32)
    per = rb.take(rid)
    q, qd, tau = synth.make_state(per.n_links, seed=12, cfg=5)
    got = _forward(m, per, q, qd, tau, "f64", dev, offsets=per.offsets, robot_id=rid)
    _check(got, per, q, qd, tau, per.offsets, "f64", "trees and chains by id")


@pytest.mark.parametrize("with_ids", [False, True])
def test_persistent_equals_forward_bitwise_on_trees(fdm, dev, with_ids):
    lengths = synth.ragged_lengths(700, 1, 120, seed=13)
    rb, q, qd, tau = _prep(lengths, "f64", seed=14)
    m = fdm.Model(rb, "f64", device=dev)
    if with_ids:
        rid = np.random.default_rng(15).integers(0, len(lengths), size=900).astype(np.int32)
        per = rb.take(rid)
        q, qd, tau = synth.make_state(per.n_links, seed=16, cfg=5)
        trid = torch.from_numpy(rid).to(dev)
    else:
        per, trid = rb, None
    toff = torch.from_numpy(per.offsets).to(dev)
    args = (_t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev))
    a = m.forward(*args, batch=len(per.n_links), algo="abia", offsets=toff, robot_id=trid).cpu()
    b = m.forward_persistent(*args, batch=len(per.n_links), offsets=toff, robot_id=trid).cpu()
    assert torch.equal(a, b)
    sample = np.arange(0, len(per.n_links), 37)
    sub = per.take(sample)
    idx = np.concatenate([np.arange(per.offsets[k], per.offsets[k + 1]) for k in sample])
    _check(a.numpy()[idx], sub, q[idx], qd[idx], tau[idx], sub.offsets, "f64", "persistent trees")


def test_explicit_serial_parents_take_the_chain_kernel(fdm, dev):
    """parent = i - 1 everywhere is a serial model: the same bits as no parent array."""
    lengths = [30] * 64
    rb = synth.make_robots(lengths, seed=17, cfg=2, random_home=True)
    q, qd, tau = synth.make_state(lengths, seed=17, cfg=2)
    tree = rb.take(np.arange(64))
    tree.parent = rb.parents()
    m1 = fdm.Model(rb, "f64", device=dev)
    m2 = fdm.Model(tree, "f64", device=dev)
    assert not m2.branched
    np.testing.assert_array_equal(_forward(m1, rb, q, qd, tau, "f64", dev), _forward(m2, tree, q, qd, tau, "f64", dev))


def test_tree_model_rejects_the_chain_only_entry_points(fdm, dev):
    """The CFA is built for serial chains only."""
    from paper_1609_06779_amd import _lib

    lengths = [8] * 4
    rb, q, qd, tau = _prep(lengths, "f64", seed=18)
    m = fdm.Model(rb, "f64", device=dev)
    assert m.branched
    args = (_t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev))
    assert m.max_links("cfa") == 0
    with pytest.raises(_lib.FdError) as e:
        m.forward(*args, batch=4, algo="cfa")
    assert e.value.status == _lib.FD_ERR_UNSUPPORTED
    assert m.max_links("abia") == 256 and m.max_links("jsiia") == 256


def _not_depth_first(n, count):
    """Trees whose links are numbered parent-first but not depth-first: link i
    hangs from link i - 2 (two interleaved branches from the base)."""
    rb = synth.make_robots([n] * count, seed=21, cfg=5, random_home=True)
    rb.parent = np.tile(np.arange(n, dtype=np.int32) - 2, count)
    rb.parent[rb.parent < 0] = -1
    return rb


def test_parent_first_order_that_is_not_depth_first(fdm, dev):
    """ABIA takes any parent-first numbering; the lane-per-link kernels need
    depth-first numbering and say so."""
    from paper_1609_06779_amd import _lib

    n, count = 20, 64
    rb = _not_depth_first(n, count)
    q, qd, tau = synth.make_state([n] * count, seed=21, cfg=5)
    m = fdm.Model(rb, "f64", device=dev)
    got = _forward(m, rb, q, qd, tau, "f64", dev)
    _check(got, rb, q, qd, tau, rb.offsets, "f64", "interleaved branches")
    assert m.max_links("jsiia") == 0
    args = (_t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev))
    for call in (lambda: m.forward(*args, batch=count, algo="jsiia"),
                 lambda: m.inverse(args[0], args[1], None, batch=count),
                 lambda: m.joint_inertia(args[0], batch=count, n=n)):
        with pytest.raises(_lib.FdError) as e:
            call()
        assert e.value.status == _lib.FD_ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 5, 8, 17, 32, 33, 64, 100, 128, 129, 200, 256])
def test_jsiia_on_trees(fdm, dev, dtype, n):
    """JSIIA on trees: M from the subtree composite inertias, zero between
    branches, then the dense elimination; every lane-group width (8 .. 256)."""
    lengths = [n] * (40 if n <= 128 else 12)
    rb, q, qd, tau = _prep(lengths, dtype, seed=200 + n, p_extend=0.7)
    m = fdm.Model(rb, dtype, device=dev)
    got = _forward(m, rb, q, qd, tau, dtype, dev, algo="jsiia")
    _check(got, rb, q, qd, tau, rb.offsets, dtype, f"jsiia tree n={n} {dtype}", backward=False)


def test_jsiia_on_trees_ragged_and_shared(fdm, dev):
    lengths = synth.ragged_lengths(120, 1, 256, seed=22)
    rb, q, qd, tau = _prep(lengths, "f64", seed=23, p_extend=0.6)
    m = fdm.Model(rb, "f64", device=dev)
    got = _forward(m, rb, q, qd, tau, "f64", dev, algo="jsiia", offsets=rb.offsets)
    _check(got, rb, q, qd, tau, rb.offsets, "f64", "jsiia ragged trees", backward=False)
    lengths = [64] * 256
    rb = synth.make_tree_robots(lengths, seed=24, cfg=5, random_home=True, shared_topology=True)
    q, qd, tau = synth.make_state(lengths, seed=24, cfg=5)
    m = fdm.Model(rb, "f64", device=dev)
    got = _forward(m, rb, q, qd, tau, "f64", dev, algo="jsiia")
    _check(got, rb, q, qd, tau, rb.offsets, "f64", "jsiia shared topology", backward=False)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 7, 32, 64, 130, 256])
def test_inverse_dynamics_on_trees(fdm, dev, dtype, n):
    batch = 21
    lengths = [n] * batch
    rb, q, qd, _ = _prep(lengths, dtype, seed=300 + n, p_extend=0.7)
    qdd = np.random.default_rng(n).standard_normal(len(q))
    if dtype == "f32":
        qdd = qdd.astype(np.float32).astype(np.float64)
    m = fdm.Model(rb, dtype, device=dev)
    for gravity in (True, False):
        ref = oracle.rnea(rb, q, qd, qdd, gravity=gravity)
        got = m.inverse(_t(q, dtype, dev), _t(qd, dtype, dev), _t(qdd, dtype, dev), batch=batch,
                        gravity=gravity).cpu().numpy().astype(np.float64)
        err = oracle.relative_error(got, ref, rb.offsets)
        bar = 1e-12 if dtype == "f64" else 2e-5           # the serial-chain bar
        assert err.max() <= bar * max(1.0, n / 8), (gravity, err.max())


@pytest.mark.parametrize("n", [1, 5, 16, 64, 128, 256])
def test_joint_inertia_on_trees(fdm, dev, n):
    batch = 9
    lengths = [n] * batch
    rb, q, _, _ = _prep(lengths, "f64", seed=400 + n, p_extend=0.7)
    m = fdm.Model(rb, "f64", device=dev)
    got = m.joint_inertia(_t(q, "f64", dev), batch=batch, n=n).cpu().numpy()
    ref = oracle.crba(rb, q)
    for b in range(batch):
        scale = np.abs(ref[b]).max()
        assert np.abs(got[b] - ref[b]).max() <= 1e-13 * scale * max(1, n / 8), b
        np.testing.assert_array_equal(got[b][ref[b] == 0], 0.0)    # no coupling across branches


def test_round_trip_on_trees(fdm, dev):
    """inverse(q, qd, FD(q, qd, tau)) returns tau (ABIA and JSIIA)."""
    lengths = [48] * 64
    rb, q, qd, tau = _prep(lengths, "f64", seed=25)
    m = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev)
    for algo in ("abia", "jsiia"):
        qdd = m.forward(tq, tqd, ttau, batch=64, algo=algo)
        back = m.inverse(tq, tqd, qdd, batch=64).cpu().numpy()
        ms = oracle.crba(rb, q)
        bias = oracle.rnea(rb, q, qd)
        qn = qdd.cpu().numpy()
        for b, mm in enumerate(ms):                # the normwise backward error of the solve
            sl = slice(rb.offsets[b], rb.offsets[b + 1])
            eta = np.linalg.norm(back[sl] - tau[sl]) / (np.linalg.norm(mm, 2) * np.linalg.norm(qn[sl]) +
                                                       np.linalg.norm(tau[sl]) + np.linalg.norm(bias[sl]))
            assert eta <= BACKWARD_FACTOR * U["f64"], (algo, b, eta / U["f64"])


def test_full_size_tree_n64_b65536_sampled(fdm, dev):
    """The timed tree workload (65536 random trees of 64 links, FP64): every
    output finite, 256 sampled trees against the oracle, and the result
    independent of the launch (persistent equals the plain launch bit for bit)."""
    w = synth.WORKLOADS["tree-n64-b65536"]
    lengths = synth.uniform_lengths(w["batch"], w["n"])
    rb = synth.make_tree_robots(lengths, p_extend=w["p_extend"], cfg=w["cfg"])
    q, qd, tau = synth.make_state(lengths, cfg=w["cfg"])
    m = fdm.Model(rb, "f64", device=dev)
    args = (_t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev))
    got = m.forward(*args, batch=w["batch"], algo="abia")
    pers = m.forward_persistent(*args, batch=w["batch"])
    assert torch.equal(got, pers)
    got = got.cpu().numpy()
    assert np.isfinite(got).all()
    pick = np.random.default_rng(19).choice(w["batch"], 256, replace=False)
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(64 * k, 64 * k + 64) for k in pick])
    _check(got[idx], sub, q[idx], qd[idx], tau[idx], sub.offsets, "f64", "tree n64 b65536")


# ---------------- reverse mode on trees ----------------

def _chain_sums(x, off):
    return np.add.reduceat(x, off[:-1])


def _tree_set(kind, n, count, seed):
    if kind == "not_depth_first":
        rb = _not_depth_first(n, count)
        q, qd, tau = synth.make_state([n] * count, seed=seed, cfg=5)
        return rb, q, qd, tau
    if kind == "shared":
        rb = synth.make_tree_robots([n] * count, seed=seed, cfg=5, random_home=True, shared_topology=True)
        q, qd, tau = synth.make_state([n] * count, seed=seed, cfg=5)
        return rb, q, qd, tau
    return _prep([n] * count, "f64", seed=seed)


@pytest.mark.parametrize("kind", ["random", "shared", "not_depth_first"])
@pytest.mark.parametrize("n", [2, 5, 16, 64, 100])
def test_tree_vjp_adjoint_identity(fdm, dev, kind, n):
    """fd_backward on trees: tau_bar = M^-1 g against the oracle's M, and
    <VJP(g), v> = <g, JVP(v)> per tree against the oracle's complex-step JVP."""
    count = 9
    rb, q, qd, tau = _tree_set(kind, n, count, seed=300 + n)
    off = rb.offsets
    m = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = (_t(a, "f64", dev) for a in (q, qd, tau))
    qdd = m.forward(tq, tqd, ttau, batch=count, algo="abia")
    ms = oracle.crba(rb, q)
    rng = np.random.default_rng(n)
    for _ in range(3):
        g = rng.standard_normal(len(q))
        gq, gqd, gtau = (x.cpu().numpy() for x in m.backward(tq, tqd, qdd, _t(g, "f64", dev), batch=count))
        for b in range(count):
            sl = slice(off[b], off[b + 1])
            ref = np.linalg.solve(ms[b], g[sl])
            assert np.linalg.norm(gtau[sl] - ref) <= CAP["f64"] * np.linalg.norm(ref), (b, "tau_bar")
        dq, dqd, dtau = (rng.standard_normal(len(q)) for _ in range(3))
        _, dqdd = oracle.fd_jvp(rb, q, qd, tau, dq, dqd, dtau)
        lhs = _chain_sums(g * dqdd, off)
        rhs = _chain_sums(gq * dq + gqd * dqd + gtau * dtau, off)
        scale = _chain_sums(np.abs(g * dqdd), off) + _chain_sums(
            np.abs(gq * dq) + np.abs(gqd * dqd) + np.abs(gtau * dtau), off)
        assert np.all(np.abs(lhs - rhs) <= CAP["f64"] * scale), (np.abs(lhs - rhs) / scale).max()


def test_tree_vjp_of_two_chains_merged_at_the_base(fdm, dev):
    """Two chains merged into one tree from the base, their links interleaved,
    give the chains' own gradients (permuted)."""
    chains = synth.make_robots([3, 4], seed=5, cfg=5, random_home=True)
    q, qd, tau = synth.make_state([3, 4], seed=5, cfg=5)
    order = [(0, 0), (1, 0), (1, 1), (0, 1), (1, 2), (0, 2), (1, 3)]
    off = chains.offsets
    src = np.array([off[c] + i for c, i in order])
    pos = {ci: t for t, ci in enumerate(order)}
    parent = np.array([-1 if i == 0 else pos[(c, i - 1)] for c, i in order], np.int32)
    tree = synth.Robots(n_links=np.array([7], np.int32), axis=chains.axis[src], home_rot=chains.home_rot[src],
                        offset=chains.offset[src], mass=chains.mass[src], com=chains.com[src],
                        inertia=chains.inertia[src], gravity=chains.gravity, parent=parent)
    mc = fdm.Model(chains, "f64", device=dev)
    mt = fdm.Model(tree, "f64", device=dev)
    assert mt.branched
    g = np.random.default_rng(7).standard_normal(7)
    a = [_t(x, "f64", dev) for x in (q, qd, tau, g)]
    toff = torch.from_numpy(np.asarray(off, np.int64)).to(dev)
    qc = mc.forward(a[0], a[1], a[2], batch=2, algo="abia", offsets=toff)
    rc = [x.cpu().numpy() for x in mc.backward(a[0], a[1], qc, a[3], batch=2, offsets=toff)]
    b = [_t(x[src], "f64", dev) for x in (q, qd, tau, g)]
    qt = mt.forward(b[0], b[1], b[2], batch=1, algo="abia")
    rt = [x.cpu().numpy() for x in mt.backward(b[0], b[1], qt, b[3], batch=1)]
    for x, y in zip(rt, rc):
        np.testing.assert_allclose(x, y[src], rtol=1e-12, atol=1e-12)


def _oracle_rollout(rb, q, qd, taus, dt, dq, dqd, dtaus):
    """(q_T, qd_T) of semi-implicit Euler and their derivatives along a direction."""
    q, qd, tq, tqd = q.copy(), qd.copy(), dq.copy(), dqd.copy()
    for t in range(taus.shape[0]):
        qdd, dqdd = oracle.fd_jvp(rb, q, qd, taus[t], tq, tqd, dtaus[t])
        tqd = tqd + dt * dqdd
        tq = tq + dt * tqd
        qd = qd + dt * qdd
        q = q + dt * qd
    return q, qd, tq, tqd


def test_tree_rollout_gradient_matches_oracle(fdm, dev):
    """30 semi-implicit Euler steps on branched robots, dt = 1e-3, checkpoints every
    10 steps, loss = sum(q_T^2 + qd_T^2): the gradient with respect to q_0, qd_0 and
    every tau_t along random directions against the oracle's complex-step JVP."""
    batch, n, steps, dt = 12, 24, 30, 1e-3
    rb, q0, qd0, _ = _prep([n] * batch, "f64", seed=77)
    taus = np.random.default_rng(8).standard_normal((steps, len(q0)))
    off = rb.offsets
    m = fdm.Model(rb, "f64", device=dev)
    assert m.branched
    tq0 = _t(q0, "f64", dev).requires_grad_(True)
    tqd0 = _t(qd0, "f64", dev).requires_grad_(True)
    ttaus = _t(taus, "f64", dev).requires_grad_(True)
    qt, qdt = fdm.rollout(m, tq0, tqd0, ttaus, batch=batch, dt=dt, every=10, algo="abia")
    ((qt ** 2).sum() + (qdt ** 2).sum()).backward()
    g0, gd0, gt = tq0.grad.cpu().numpy(), tqd0.grad.cpu().numpy(), ttaus.grad.cpu().numpy()
    rng = np.random.default_rng(9)
    for _ in range(8):
        dq, dqd = rng.standard_normal(len(q0)), rng.standard_normal(len(q0))
        dtaus = rng.standard_normal(taus.shape)
        rq, rqd, tq, tqd = _oracle_rollout(rb, q0, qd0, taus, dt, dq, dqd, dtaus)
        exact = _chain_sums(2 * rq * tq + 2 * rqd * tqd, off)
        ours = _chain_sums(g0 * dq + gd0 * dqd + (gt * dtaus).sum(axis=0), off)
        scale = _chain_sums(np.abs(g0 * dq) + np.abs(gd0 * dqd) + np.abs(gt * dtaus).sum(axis=0), off)
        assert np.all(np.abs(ours - exact) <= 1e-10 * (1 + np.maximum(np.abs(exact), scale))), \
            np.abs(ours - exact).max()
    np.testing.assert_allclose(qt.detach().cpu().numpy(), rq, rtol=0, atol=1e-10 * (1 + np.abs(rq).max()))


def test_tree_vjp_full_size_sampled(fdm, dev):
    """65536 random trees of 64 links (the headline shape): sampled trees against
    the oracle through the adjoint identity, and every gradient finite."""
    batch, n = 65536, 64
    lengths = [n] * batch
    rb = synth.make_tree_robots(lengths, seed=11, cfg=2)
    q, qd, tau = synth.make_state(lengths, seed=11, cfg=2)
    m = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = (_t(a, "f64", dev) for a in (q, qd, tau))
    qdd = m.forward(tq, tqd, ttau, batch=batch, algo="abia")
    g = np.random.default_rng(12).standard_normal(len(q))
    gq, gqd, gtau = (x.cpu().numpy() for x in m.backward(tq, tqd, qdd, _t(g, "f64", dev), batch=batch))
    assert np.all(np.isfinite(gq)) and np.all(np.isfinite(gqd)) and np.all(np.isfinite(gtau))
    pick = np.array([0, 1, 4095, 33333, 65535])
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(n * b, n * b + n) for b in pick])
    off = sub.offsets
    rng = np.random.default_rng(13)
    dq, dqd, dtau = (rng.standard_normal(len(idx)) for _ in range(3))
    _, dqdd = oracle.fd_jvp(sub, q[idx], qd[idx], tau[idx], dq, dqd, dtau)
    lhs = _chain_sums(g[idx] * dqdd, off)
    rhs = _chain_sums(gq[idx] * dq + gqd[idx] * dqd + gtau[idx] * dtau, off)
    scale = _chain_sums(np.abs(g[idx] * dqdd), off) + _chain_sums(
        np.abs(gq[idx] * dq) + np.abs(gqd[idx] * dqd) + np.abs(gtau[idx] * dtau), off)
    assert np.all(np.abs(lhs - rhs) <= CAP["f64"] * scale), (np.abs(lhs - rhs) / scale).max()


def test_auto_takes_jsiia_for_trees_of_mixed_topologies(fdm, dev):
    """AUTO on branched robots: the tuned table's choice (the CFA mapped to ABIA)
    while every robot of a length shares one topology; JSIIA when topologies
    differ, where ABIA's lanes would diverge at every robot's branch points.
    Checked bit for bit against the explicit algorithm."""
    from paper_1609_06779_amd import tune

    n, count = 40, 300
    mixed = synth.make_tree_robots([n] * count, seed=31, cfg=5, random_home=True)
    shared = synth.make_tree_robots([n] * count, seed=31, cfg=5, random_home=True, shared_topology=True)
    q, qd, tau = synth.make_state([n] * count, seed=31, cfg=5)
    for rb, want in ((mixed, "jsiia"), (shared, None)):
        m = fdm.Model(rb, "f64", device=dev)
        assert m.branched
        if want is None:
            want = tune.best_algo("f64", n, count)
            want = "abia" if want == "cfa" else want
        auto = _forward(m, rb, q, qd, tau, "f64", dev, algo="auto")
        np.testing.assert_array_equal(auto, _forward(m, rb, q, qd, tau, "f64", dev, algo=want))
