"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Forward dynamics is compared per chain by the normwise relative error
||qdd - qdd_ref|| / ||qdd_ref||, with qdd_ref the oracle evaluated in long
double (``oracle.fd_exact``), so that the oracle's own rounding, which in
double grows as cond(M) u, is not counted against the kernels. Every bar is a fixed number per precision,
stated before any run: the cap (1e-9 FP64, 1e-3 FP32, ten times the
forward-dynamics target 1e-10 / 1e-4). Every chain of every test must be
within the cap; each test also prints how many chains meet the target
itself, and the benchmark records those fractions per algorithm, length and
precision. Cells where chains exceed the cap are measured failures, marked
as expected failures (strict: they fail the suite if they start passing).

The normwise backward error ||M qdd - tau_delta|| / (||M|| ||qdd|| + ||tau|| +
||tau_bias||) (tau and the bias torque are the data of the solve) is bounded
by a fixed multiple of the unit roundoff u for every algorithm: ABIA and the
symmetric elimination of JSIIA are backward stable; the CFA's
M^-1 = C - B^T A^-1 B (eq. (fijany-final)) is a difference of terms of size
||C|| and its bound is correspondingly larger.
FP32 runs round robots and states to FP32 first and the FP64 oracle runs on
the same rounded values.
"""
import numpy as np
import pytest

import oracle
from _errmodel import CAP, TARGET, U
from oracle import dense
from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALGOS = ("abia", "jsiia", "cfa", "abia_scan")
# normwise backward error bound in units of u, per algorithm
BACKWARD_U = {"abia": 64.0, "jsiia": 64.0, "cfa": float(2 ** 20), "abia_scan": 64.0}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def fdm():
    from paper_1609_06779_amd import fd
    return fd


def _prep(lengths, dtype, cfg=2, seed=synth.ROOT_SEED, random_home=False):
    rb = synth.make_robots(lengths, seed=seed, cfg=cfg, random_home=random_home)
    q, qd, tau = synth.make_state(lengths, seed=seed, cfg=cfg)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
        q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in (q, qd, tau))
    return rb, q, qd, tau


def _t(a, dtype, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if dtype == "f64" else np.float32)).to(dev)


def _backward_error(rb, q, qd, tau, qdd, off):
    ms = oracle.crba(rb, q, offsets=off)
    bias = oracle.rnea(rb, q, qd, offsets=off)
    eta = []
    for b, m in enumerate(ms):
        sl = slice(off[b], off[b + 1])
        td = tau[sl] - bias[sl]
        eta.append(np.linalg.norm(m @ qdd[sl] - td) /
                   (np.linalg.norm(m, 2) * np.linalg.norm(qdd[sl]) + np.linalg.norm(tau[sl]) + np.linalg.norm(bias[sl])))
    return np.array(eta)


def _check(got, ref, off, dtype, what, algo, rb=None, q=None, qd=None, tau=None):
    """Every chain within CAP[dtype]; with (rb, q, qd, tau) also the backward error bound."""
    err = oracle.relative_error(got, ref, off)
    worst = float(err.max()) if len(err) else 0.0
    within = int(np.sum(err <= TARGET[dtype]))
    print(f"{what}: worst {worst:.2e}, {within} of {len(err)} chains within {TARGET[dtype]:g}", flush=True)
    bad = np.nonzero(~(err <= CAP[dtype]))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} chains over the cap {CAP[dtype]:g}, worst {worst:.3e} (chain {bad[:5]})"
    if qd is not None:
        eta = _backward_error(rb, q, qd, tau, got, off)
        assert eta.max() <= BACKWARD_U[algo] * U[dtype], f"{what}: backward error {eta.max() / U[dtype]:.1f} u"
    return err


def _forward(fdm, dev, rb, q, qd, tau, dtype, algo, offsets=None, robot_id=None, model=None):
    m = model or fdm.Model(rb, dtype, device=dev)
    batch = len(rb.n_links) if robot_id is None else len(robot_id)
    toff = None if offsets is None else torch.from_numpy(np.asarray(offsets, np.int64)).to(dev)
    trid = None if robot_id is None else torch.from_numpy(np.asarray(robot_id, np.int32)).to(dev)
    out = m.forward(_t(q, dtype, dev), _t(qd, dtype, dev), _t(tau, dtype, dev), batch=batch, algo=algo,
                    offsets=toff, robot_id=trid)
    return out.cpu().numpy().astype(np.float64)


# ---------------- forward dynamics, uniform batches ----------------

# FP32 cells with chains over the FP32 cap on this generator, measured on
# MI355X (worst per-chain relative error). They are expected failures (strict:
# a cell that starts passing fails the suite) and are reported in the
# benchmark's accuracy record. FP32 forward error grows as kappa u32: cond_2(M)
# for ABIA and JSIIA, ||C|| ||M|| for the CFA, whose M^-1 = C - B^T A^-1 B
# (eq. (fijany-final)) is a difference of terms of size ||C||.
FP32_OVER_CAP = {
    ("cfa", 24): 2.5e-3, ("cfa", 32): 3.9e-3, ("cfa", 33): 2.2e-3, ("cfa", 50): 3.5e-3, ("cfa", 64): 1.0e-2,
    ("cfa", 100): 3.3e-2, ("cfa", 128): 9.8e-3, ("cfa", 200): 9.7e-2, ("cfa", 256): 8.1e-2,
    ("jsiia", 100): 1.2e-3, ("jsiia", 128): 2.0e-3, ("jsiia", 200): 3.6e-3, ("jsiia", 256): 1.6e-2,
    ("abia_scan", 200): 1.7e-3, ("abia_scan", 256): 2.6e-3, ("abia", 256): 1.2e-3,
}


def _uniform_cases():
    for n in [1, 2, 3, 5, 8, 13, 16, 24, 32, 33, 50, 64, 100, 128, 200, 256]:
        for algo in ALGOS:
            for dtype in ("f64", "f32"):
                marks = ()
                if dtype == "f32" and (algo, n) in FP32_OVER_CAP:
                    w = FP32_OVER_CAP[(algo, n)]
                    marks = pytest.mark.xfail(strict=True, reason=f"FP32 {algo} at n={n}: chains over the 1e-3 cap"
                                              + f" (worst {w:g})")
                yield pytest.param(n, algo, dtype, marks=marks, id=f"{n}-{algo}-{dtype}")


@pytest.mark.parametrize("n,algo,dtype", list(_uniform_cases()))
def test_forward_uniform(fdm, dev, algo, dtype, n):
    batch = 37 if n <= 64 else 11            # not a multiple of the chains per workgroup
    lengths = np.full(batch, n, np.int32)
    rb, q, qd, tau = _prep(lengths, dtype, random_home=(n % 2 == 1))
    off = rb.offsets
    ref = oracle.fd_exact(rb, q, qd, tau)
    got = _forward(fdm, dev, rb, q, qd, tau, dtype, algo)
    _check(got, ref, off, dtype, f"{algo} {dtype} n={n}", algo, rb, q, qd, tau)


@pytest.mark.parametrize("dtype,n", [("f64", 1), ("f64", 2), ("f64", 5), ("f64", 8), ("f64", 16), ("f64", 33),
                                     ("f64", 64), ("f64", 128), ("f64", 200), ("f64", 256),
                                     ("f32", 1), ("f32", 5), ("f32", 8)])
def test_cfa_projector_form(fdm, dev, dtype, n):
    """FD_ALGO_CFA_PROJ (projectors in place of the basis W, 6x6 blocks) against
    the oracle within the cap, with the CFA's backward-error bound, and against
    the 5x5 CFA on the same chains within the cap."""
    batch = 37 if n <= 64 else 11
    lengths = np.full(batch, n, np.int32)
    rb, q, qd, tau = _prep(lengths, dtype, random_home=(n % 2 == 1))
    off = rb.offsets
    model = fdm.Model(rb, dtype, device=dev)
    ref = oracle.fd_exact(rb, q, qd, tau)
    got = _forward(fdm, dev, rb, q, qd, tau, dtype, "cfa_proj", model=model)
    _check(got, ref, off, dtype, f"cfa_proj {dtype} n={n}", "cfa", rb, q, qd, tau)
    five = _forward(fdm, dev, rb, q, qd, tau, dtype, "cfa", model=model)
    assert oracle.relative_error(got, five, off).max() <= CAP[dtype]


def test_cfa_projector_form_ragged_and_refuses_trees(fdm, dev):
    from paper_1609_06779_amd import _lib
    lengths = synth.ragged_lengths(41, 1, 100, cfg=3)
    rb, q, qd, tau = _prep(lengths, "f64", cfg=3)
    off = rb.offsets
    got = _forward(fdm, dev, rb, q, qd, tau, "f64", "cfa_proj", offsets=off)
    _check(got, oracle.fd_exact(rb, q, qd, tau), off, "f64", "cfa_proj ragged", "cfa", rb, q, qd, tau)
    mt = fdm.Model(synth.make_tree_robots([12], cfg=5), "f64", device=dev)
    t12 = torch.zeros(12, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.FdError) as ei:
        mt.forward(t12, t12, t12, batch=1, algo="cfa_proj")
    assert ei.value.status == _lib.FD_ERR_UNSUPPORTED


def test_config_plain_n8_b1024_all_chains(fdm, dev):
    lengths = synth.uniform_lengths(1024, 8)
    rb, q, qd, tau = _prep(lengths, "f64", cfg=1)
    off = rb.offsets
    ref = oracle.fd_exact(rb, q, qd, tau)
    model = fdm.Model(rb, "f64", device=dev)
    for algo in ALGOS:
        got = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, model=model)
        err = oracle.relative_error(got, ref, off)
        assert err.max() <= TARGET["f64"], (algo, err.max())     # the target itself, on every chain


@pytest.mark.parametrize("algo", ALGOS)
def test_ragged_batch_with_offsets(fdm, dev, algo):
    hi = 256
    lengths = synth.ragged_lengths(61, 1, hi, cfg=3)
    lengths[:3] = [1, hi, 2]
    rb, q, qd, tau = _prep(lengths, "f64", cfg=3)
    off = rb.offsets
    ref = oracle.fd_exact(rb, q, qd, tau)
    got = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, offsets=off)
    _check(got, ref, off, "f64", f"{algo} ragged", algo, rb, q, qd, tau)


@pytest.mark.parametrize("algo", ALGOS)
def test_shared_robots_by_id(fdm, dev, algo):
    base_lengths = np.array([7, 20, 3, 64, 33], np.int32)
    base = synth.make_robots(base_lengths, cfg=4)
    rng = np.random.default_rng(3)
    rid = rng.integers(0, len(base_lengths), size=150).astype(np.int32)
    per_chain = base.take(rid)
    lengths = per_chain.n_links
    q, qd, tau = synth.make_state(lengths, cfg=4)
    off = synth.offsets_of(lengths)
    ref = oracle.fd_exact(per_chain, q, qd, tau)
    model = fdm.Model(base, "f64", device=dev)
    got = _forward(fdm, dev, base, q, qd, tau, "f64", algo, offsets=off, robot_id=rid, model=model)
    _check(got, ref, off, "f64", f"{algo} shared robots", algo, per_chain, q, qd, tau)


@pytest.mark.parametrize("algo", ALGOS)
def test_full_size_n64_b65536_sampled(fdm, dev, algo):
    """The benchmark's workload and launch: 65536 chains of 64 links, FP64,
    512 chains checked against the oracle."""
    lengths = synth.uniform_lengths(65536, 64)
    rb, q, qd, tau = _prep(lengths, "f64", cfg=2)
    got = _forward(fdm, dev, rb, q, qd, tau, "f64", algo)
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(65536, size=512, replace=False))
    pick[0], pick[-1] = 0, 65535
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(64 * b, 64 * b + 64) for b in pick])
    ref = oracle.fd_exact(sub, q[idx], qd[idx], tau[idx])
    _check(got[idx], ref, sub.offsets, "f64", f"{algo} full size", algo, sub, q[idx], qd[idx], tau[idx])
    assert np.all(np.isfinite(got))


def test_deterministic_and_independent_of_batch_neighbours(fdm, dev):
    lengths = np.full(40, 24, np.int32)
    rb, q, qd, tau = _prep(lengths, "f64")
    model = fdm.Model(rb, "f64", device=dev)
    for algo in ALGOS:
        a = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, model=model)
        b = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, model=model)
        assert np.array_equal(a, b), algo
        # chain 5 alone (robot 5 picked by id) gives the same bits as inside the batch
        sl = slice(5 * 24, 6 * 24)
        alone = _forward(fdm, dev, rb, q[sl], qd[sl], tau[sl], "f64", algo, robot_id=[5], model=model)
        assert np.array_equal(alone, a[sl]), algo


def test_round_trip_on_gpu(fdm, dev):
    """ID(q, qd, FD(q, qd, tau)) = tau, both on the GPU, in the normwise sense
    ||ID - tau|| / (||M|| ||qdd|| + ||tau|| + ||tau_bias||): the backward error of
    each factorisation, within its bound."""
    lengths = np.full(64, 32, np.int32)
    rb, q, qd, tau = _prep(lengths, "f64")
    off = rb.offsets
    model = fdm.Model(rb, "f64", device=dev)
    tq, tqd, ttau = _t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev)
    ms = oracle.crba(rb, q)
    bias = oracle.rnea(rb, q, qd)
    for algo in ALGOS:
        qdd = model.forward(tq, tqd, ttau, batch=64, algo=algo)
        back = model.inverse(tq, tqd, qdd, batch=64).cpu().numpy()
        qn = qdd.cpu().numpy()
        for b, m in enumerate(ms):
            sl = slice(off[b], off[b + 1])
            eta = np.linalg.norm(back[sl] - tau[sl]) / (np.linalg.norm(m, 2) * np.linalg.norm(qn[sl]) +
                                                       np.linalg.norm(tau[sl]) + np.linalg.norm(bias[sl]))
            assert eta <= BACKWARD_U[algo] * U["f64"], (algo, b, eta / U["f64"])


def test_empty_batch_and_workspace_errors(fdm, dev):
    from paper_1609_06779_amd import _lib
    lengths = np.full(4, 6, np.int32)
    rb, q, qd, tau = _prep(lengths, "f64")
    model = fdm.Model(rb, "f64", device=dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    model.forward(e, e, e, batch=0, algo="cfa")
    tq = _t(q, "f64", dev)
    with pytest.raises(_lib.FdError) as ei:
        model.forward(tq, tq, tq, batch=4, algo="abia", workspace=torch.empty(8, dtype=torch.uint8, device=dev))
    assert ei.value.status == _lib.FD_ERR_WORKSPACE
    t30 = torch.zeros(30, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.FdError) as ei:
        model.forward(t30, t30, t30, batch=5, algo="cfa")       # more chains than robots
    assert ei.value.status == _lib.FD_ERR_INVALID_ARG
    with pytest.raises(ValueError, match="q has 24 entries"):   # the binding's size check, before any launch
        model.forward(tq, tq, tq, batch=5, algo="cfa")
    tree = synth.make_tree_robots([12], cfg=5)
    mt = fdm.Model(tree, "f64", device=dev)
    t12 = torch.zeros(12, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.FdError) as ei:                    # the CFA takes serial chains only
        mt.forward(t12, t12, t12, batch=1, algo="cfa")
    assert ei.value.status == _lib.FD_ERR_UNSUPPORTED


# ---------------- inverse dynamics and the joint-space inertia ----------------

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 7, 32, 64, 130, 256])
def test_inverse_dynamics(fdm, dev, dtype, n):
    batch = 21
    lengths = np.full(batch, n, np.int32)
    rb, q, qd, _ = _prep(lengths, dtype, cfg=6, random_home=True)
    qdd = np.random.default_rng(n).standard_normal(len(q))
    if dtype == "f32":
        qdd = qdd.astype(np.float32).astype(np.float64)
    model = fdm.Model(rb, dtype, device=dev)
    for gravity in (True, False):
        ref = oracle.rnea(rb, q, qd, qdd, gravity=gravity)
        got = model.inverse(_t(q, dtype, dev), _t(qd, dtype, dev), _t(qdd, dtype, dev), batch=batch,
                            gravity=gravity).cpu().numpy().astype(np.float64)
        err = oracle.relative_error(got, ref, rb.offsets)
        # inverse dynamics is a forward evaluation: error ~ n u times the transform magnitudes
        bar = 1e-12 if dtype == "f64" else 2e-5
        assert err.max() <= bar * max(1.0, n / 8), (gravity, err.max())


@pytest.mark.parametrize("n", [1, 5, 16, 64, 128])
def test_joint_inertia(fdm, dev, n):
    batch = 9
    lengths = np.full(batch, n, np.int32)
    rb, q, _, _ = _prep(lengths, "f64", cfg=6, random_home=True)
    model = fdm.Model(rb, "f64", device=dev)
    got = model.joint_inertia(_t(q, "f64", dev), batch=batch, n=n).cpu().numpy()
    ref = oracle.crba(rb, q)
    for b in range(batch):
        scale = np.abs(ref[b]).max()
        assert np.abs(got[b] - ref[b]).max() <= 1e-13 * scale * max(1, n / 8), b


# ---------------- the building blocks on their own ----------------

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("reverse", [False, True])
def test_scan6(fdm, dev, dtype, reverse):
    lengths = np.array([1, 2, 3, 7, 8, 9, 31, 64, 65, 100, 128, 200, 256, 5], np.int64)
    b, c = synth.make_scan_elements(lengths, seed=17)
    off = synth.offsets_of(lengths)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        b, c = b.astype(np.float32).astype(np.float64), c.astype(np.float32).astype(np.float64)
    x = fdm.scan6(torch.from_numpy(b).to(dev, tdt), torch.from_numpy(c).to(dev, tdt),
                  torch.from_numpy(off).to(dev), max_len=int(lengths.max()), reverse=reverse).cpu().numpy()
    for s in range(len(lengths)):
        sl = slice(off[s], off[s + 1])
        ref = dense.scan_serial(b[sl], c[sl], reverse)
        tol = (1e-13 if dtype == "f64" else 1e-5) * np.sqrt(lengths[s])
        assert np.abs(x[sl] - ref).max() <= tol * (1 + np.abs(ref).max()), s


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_btd_solve6(fdm, dev, dtype):
    lengths = np.array([1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 33, 64, 100, 128, 129, 255, 256, 6], np.int64)
    d, u, r = synth.make_btd(lengths, k=6, seed=23)
    if dtype == "f32":
        d, u, r = (a.astype(np.float32).astype(np.float64) for a in (d, u, r))
    off = synth.offsets_of(lengths)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x, status = fdm.btd_solve6(torch.from_numpy(d).to(dev, tdt), torch.from_numpy(u).to(dev, tdt),
                               torch.from_numpy(r).to(dev, tdt), torch.from_numpy(off).to(dev),
                               max_len=int(lengths.max()))
    x = x.cpu().numpy().astype(np.float64)
    assert int(status.item()) == 0
    for s_ in range(len(lengths)):
        sl = slice(off[s_], off[s_ + 1])
        a = dense.btd_assemble(d[sl], u[sl])
        rv = r[sl].reshape(-1)

        def eta_of(xs):                       # normwise backward error of a solution
            return np.linalg.norm(a @ xs.reshape(-1) - rv) / (np.linalg.norm(a, 2) * np.linalg.norm(xs) +
                                                            np.linalg.norm(rv))
        # Odd-even elimination is block elimination with multipliers
        # E = U D^-1, and block elimination of an SPD matrix has a backward
        # error of order (1 + kappa^(1/2)) u rather than a size-only multiple of
        # u (Higham, Accuracy and Stability of Numerical Algorithms, block LU
        # of SPD matrices); here per level, L = ceil(log2 n) levels. The
        # oracle's plain evaluation of the paper's steps shows the same
        # growth (about 8e3 u on the 255-block system, kappa 2.5e6).
        levels = max(1, int(np.ceil(np.log2(lengths[s_]))))
        bound = 4.0 * levels * (1.0 + np.sqrt(np.linalg.cond(a)))
        eta_oee = eta_of(dense.oee_solve(d[sl], u[sl], r[sl])) / U["f64"]
        eta = eta_of(x[sl]) / U[dtype]
        print(f"btd {dtype} n={lengths[s_]}: backward error {eta:.1f} u (oracle's OEE {eta_oee:.1f} u), "
              f"bound {bound:.0f} u", flush=True)
        assert eta <= bound, (s_, lengths[s_], eta, bound)
        if dtype == "f64":                    # and LAPACK's x within the cap
            ref = dense.btd_solve_dense(d[sl], u[sl], r[sl])
            rel = np.linalg.norm(x[sl] - ref) / np.linalg.norm(ref)
            assert rel <= CAP[dtype], (s_, lengths[s_], rel)


def test_btd_solve6_reports_non_spd(fdm, dev):
    lengths = np.array([4], np.int64)
    d = np.tile(-np.eye(6), (4, 1, 1))
    u = np.zeros((4, 6, 6))
    r = np.ones((4, 6))
    _, status = fdm.btd_solve6(torch.from_numpy(d).to(dev), torch.from_numpy(u).to(dev),
                               torch.from_numpy(r).to(dev), torch.from_numpy(np.array([0, 4])).to(dev), max_len=4)
    assert int(status.item()) & 1


# ---------------- the batch's length bound (max_links) ----------------

@pytest.mark.parametrize("algo", ALGOS)
def test_length_bound_sizes_the_launch(fdm, dev, algo):
    """Robot ids into a model whose longest robot has 200 links: with max_links set to
    the batch's longest chain (30) every algorithm runs at that size and matches the
    oracle; ABIA is bit for bit the unbounded launch; a bound of 12 leaves the longer
    chains unsolved (NaN) and the others exact."""
    from paper_1609_06779_amd import _lib

    lengths = np.array([200, 30, 12, 7, 30, 25], np.int32)
    rb, _, _, _ = _prep(lengths, "f64", cfg=7)
    model = fdm.Model(rb, "f64", device=dev)
    ids = np.array([1, 2, 3, 4, 5, 1, 3, 2, 4, 5] * 3, np.int32)
    sub = rb.take(ids)
    q, qd, tau = synth.make_state(sub.n_links, cfg=7)
    off = sub.offsets
    tq, tqd, ttau = _t(q, "f64", dev), _t(qd, "f64", dev), _t(tau, "f64", dev)
    rid, toff = torch.from_numpy(ids).to(dev), torch.from_numpy(off).to(dev)
    ref = oracle.fd_exact(sub, q, qd, tau)
    got = model.forward(tq, tqd, ttau, batch=len(ids), algo=algo, robot_id=rid, offsets=toff, max_links=30)
    _check(got.cpu().numpy(), ref, off, "f64", f"{algo} bounded", algo)
    if algo == "abia":
        free = model.forward(tq, tqd, ttau, batch=len(ids), algo=algo, robot_id=rid, offsets=toff)
        assert torch.equal(got, free)
    short = model.forward(tq, tqd, ttau, batch=len(ids), algo=algo, robot_id=rid, offsets=toff,
                          max_links=12).cpu().numpy()
    for b, n in enumerate(sub.n_links):
        sl = slice(off[b], off[b + 1])
        if n > 12:
            assert np.all(np.isnan(short[sl])), b
        else:
            assert np.all(np.isfinite(short[sl])), b
    ok = sub.n_links <= 12
    keep = np.concatenate([np.arange(off[b], off[b + 1]) for b in np.nonzero(ok)[0]])
    sub_ok = sub.take(np.nonzero(ok)[0])
    _check(short[keep], ref[keep], sub_ok.offsets, "f64", f"{algo} short bound", algo)
    for bad in (-1, 257):
        with pytest.raises(_lib.FdError) as ei:
            model.forward(tq, tqd, ttau, batch=len(ids), algo=algo, robot_id=rid, offsets=toff, max_links=bad)
        assert ei.value.status == _lib.FD_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_every_chain_at_65536(fdm, dev, n):
    """65536 chains of n links (16 .. 128), FP64: every chain of every algorithm
    against the oracle (all host threads), within the cap; the chains above the
    target are counted and their error-model factor printed (diagnostics)."""
    from _errmodel import kappa

    batch = 65536
    lengths = synth.uniform_lengths(batch, n)
    rb, q, qd, tau = _prep(lengths, "f64", cfg=2)
    ref = oracle.fd_exact(rb, q, qd, tau, threads=0)
    off = rb.offsets
    model = fdm.Model(rb, "f64", device=dev)
    for algo in ALGOS:
        got = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, model=model)
        assert np.all(np.isfinite(got)), algo
        err = _check(got, ref, off, "f64", f"{algo} n={n} b={batch}", algo)
        over = np.nonzero(err > TARGET["f64"])[0]
        if len(over):
            k = kappa(algo, rb, q, n, over[:64])
            print(f"  {algo} n={n}: error / (kappa u) of the chains above the target: max "
                  f"{(err[over[:64]] / (k * U['f64'])).max():.2f}", flush=True)


@pytest.mark.parametrize("algo", ALGOS)
def test_non_finite_inputs_stay_in_their_chain(fdm, dev, algo):
    """A NaN or infinite entry makes its own chain's q-ddot non-finite and leaves
    every other chain of the batch bit for bit as in a clean run (chains share
    no arithmetic). The kernels branch on no input value, so nothing else moves."""
    lengths = np.full(10, 9, np.int32)
    rb, q, qd, tau = _prep(lengths, "f64", cfg=5)
    model = fdm.Model(rb, "f64", device=dev)
    clean = _forward(fdm, dev, rb, q, qd, tau, "f64", algo, model=model)
    q2, qd2, tau2 = q.copy(), qd.copy(), tau.copy()
    q2[3 * 9 + 4] = np.nan
    qd2[5 * 9 + 0] = np.inf
    tau2[7 * 9 + 8] = -np.inf
    dirty = _forward(fdm, dev, rb, q2, qd2, tau2, "f64", algo, model=model)
    for b in range(10):
        sl = slice(9 * b, 9 * b + 9)
        if b in (3, 5, 7):
            assert not np.all(np.isfinite(dirty[sl])), b
        else:
            np.testing.assert_array_equal(dirty[sl], clean[sl])


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("dtype,scale", [("f64", 1e2), ("f64", 1e5), ("f64", 1e7), ("f32", 50.0), ("f32", 1e5)])
def test_large_joint_angles(fdm, dev, algo, dtype, scale):
    """Joint angles far from zero (up to 1e7 rad, where the sine and cosine
    need a long argument reduction): every chain stays within the cap of the
    oracle, which evaluates the C library's sin and cos at the same angles."""
    lengths = np.full(29, 12, np.int32)
    rb, q, qd, tau = _prep(lengths, dtype, cfg=5)
    rng = np.random.default_rng(1609)
    q = q + scale * rng.uniform(-1.0, 1.0, q.shape)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
    ref = oracle.fd_exact(rb, q, qd, tau)
    got = _forward(fdm, dev, rb, q, qd, tau, dtype, algo)
    _check(got, ref, rb.offsets, dtype, f"{algo} {dtype} |q| ~ {scale:g}", algo)
