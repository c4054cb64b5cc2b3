"""GPU parity on branched robots (trees): the articulated-body kernel's tree
variant, through the C-ABI, against the oracle.

A tree hangs link i from a parent p(i) < i (the paper treats serial chains).
The bar is the one of the serial-chain parity tests for ABIA: a forward error
of 1e-10 (FP64) or 1e-4 (FP32) where conditioning allows, else
16 cond_2(M) u per chain, and a normwise backward error of at most 64 u.
FP32 runs round robots and states to FP32 first.
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


def _check(got, rb, q, qd, tau, off, dtype, what):
    ref = oracle.fd(rb, q, qd, tau, offsets=off)
    err = oracle.relative_error(got, ref, off)
    ms = oracle.crba(rb, q, offsets=off)
    bar = np.full(len(err), TOL[dtype])
    if len(err) and err.max() > TOL[dtype]:
        bar = np.maximum(bar, COND_FACTOR * np.array([np.linalg.cond(m) for m in ms]) * U[dtype])
    bad = np.nonzero(~(err <= bar))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} trees over the bar, worst {err.max():.3e} (tree {bad[:5]})"
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
    if m.branched:                                       # AUTO takes ABIA on a branched model
        np.testing.assert_array_equal(_forward(m, rb, q, qd, tau, dtype, dev, algo="auto"), got)


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
    from paper_1609_06779_amd import _lib

    lengths = [8] * 4
    rb, q, qd, tau = _prep(lengths, "f64", seed=18)
    m = fdm.Model(rb, "f64", device=dev)
    assert m.branched
    args = (_t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev))
    for algo in ("jsiia", "cfa"):
        assert m.max_links(algo) == 0
        with pytest.raises(_lib.FdError) as e:
            m.forward(*args, batch=4, algo=algo)
        assert e.value.status == _lib.FD_ERR_UNSUPPORTED
    assert m.max_links("abia") == 256
    for call in (lambda: m.inverse(args[0], args[1], None, batch=4),
                 lambda: m.joint_inertia(args[0], batch=4, n=8),
                 lambda: m.backward(args[0], args[1], args[2], args[2], batch=4)):
        with pytest.raises(_lib.FdError) as e:
            call()
        assert e.value.status == _lib.FD_ERR_UNSUPPORTED


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
