"""GPU parity on branched robots (trees), through the C-ABI, against the oracle:
the articulated-body kernel's tree variant (any parent order), and the
lane-per-link kernels on trees numbered depth-first (JSIIA, inverse dynamics,
the joint-space inertia), whose scans run over root paths and subtrees.

A tree hangs link i from a parent p(i) < i (the paper treats serial chains).
The bars are those of the serial-chain parity tests: a forward error of 1e-10
(FP64) or 1e-4 (FP32) where conditioning allows, else 16 cond_2(M) u per chain;
for ABIA also a normwise backward error of at most 64 u. FP32 runs round robots
and states to FP32 first.
"""
import numpy as np
import pytest

import oracle
from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}
TOL = {"f64": 1e-10, "f32": 1e-4}
COND_FACTOR = 16.0
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
    ref = oracle.fd(rb, q, qd, tau, offsets=off)
    err = oracle.relative_error(got, ref, off)
    ms = oracle.crba(rb, q, offsets=off)
    bar = np.full(len(err), TOL[dtype])
    if len(err) and err.max() > TOL[dtype]:
        bar = np.maximum(bar, COND_FACTOR * np.array([np.linalg.cond(m) for m in ms]) * U[dtype])
    bad = np.nonzero(~(err <= bar))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} trees over the bar, worst {err.max():.3e} (tree {bad[:5]})"
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
    """The CFA and the reverse mode are built for serial chains only."""
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
    with pytest.raises(_lib.FdError) as e:
        m.backward(args[0], args[1], args[2], args[2], batch=4)
    assert e.value.status == _lib.FD_ERR_UNSUPPORTED
    assert m.max_links("abia") == 256 and m.max_links("jsiia") == 128


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
@pytest.mark.parametrize("n", [1, 5, 8, 17, 32, 33, 64, 100, 128])
def test_jsiia_on_trees(fdm, dev, dtype, n):
    """JSIIA on trees: M from the subtree composite inertias, zero between
    branches, then the dense elimination; every lane-group width (8 .. 128)."""
    lengths = [n] * 40
    rb, q, qd, tau = _prep(lengths, dtype, seed=200 + n, p_extend=0.7)
    m = fdm.Model(rb, dtype, device=dev)
    got = _forward(m, rb, q, qd, tau, dtype, dev, algo="jsiia")
    _check(got, rb, q, qd, tau, rb.offsets, dtype, f"jsiia tree n={n} {dtype}", backward=False)


def test_jsiia_on_trees_ragged_and_shared(fdm, dev):
    lengths = synth.ragged_lengths(120, 1, 128, seed=22)
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
        err = oracle.relative_error(back, tau, rb.offsets)
        kappa = np.array([np.linalg.cond(x) for x in oracle.crba(rb, q)])
        assert np.all(err <= np.maximum(1e-10, 64 * kappa * 2.0 ** -53)), (algo, err.max())


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
