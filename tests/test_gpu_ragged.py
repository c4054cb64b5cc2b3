"""Ragged batches in one persistent launch: bit-for-bit the plain launch's
results for every grid size, and the oracle's within its bar."""
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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_persistent_equals_plain_and_oracle(dev, dtype):
    from paper_1609_06779_amd import fd

    lengths = synth.ragged_lengths(3001, 4, 256, cfg=3)
    lengths[:4] = [256, 4, 1, 255]
    rb = synth.make_robots(lengths, cfg=3)
    q, qd, tau = synth.make_state(lengths, cfg=3)
    if dtype == "f32":
        rb = rb.astype_rounded(np.float32)
        q, qd, tau = (a.astype(np.float32).astype(np.float64) for a in (q, qd, tau))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    off = rb.offsets
    model = fd.Model(rb, dtype, device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev, tdt) for a in (q, qd, tau))
    toff = torch.from_numpy(off).to(dev)
    plain = model.forward(tq, tqd, ttau, batch=len(lengths), algo="abia", offsets=toff)
    for grid in (0, 1, 7, 333):
        pers = model.forward_persistent(tq, tqd, ttau, batch=len(lengths), grid=grid, offsets=toff)
        assert torch.equal(pers, plain), grid
    pick = np.array([0, 1, 2, 3, 100, 1000, 3000])
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(off[b], off[b + 1]) for b in pick])
    ref = oracle.fd_exact(sub, q[idx], qd[idx], tau[idx])
    err = oracle.relative_error(plain.cpu().double().numpy()[idx], ref, sub.offsets)
    assert np.all(err <= CAP[dtype]), err


def test_persistent_skips_out_of_range_robot_ids(dev):
    from paper_1609_06779_amd import fd

    base = np.array([5, 9, 3], np.int32)
    rb = synth.make_robots(base, cfg=3)
    model = fd.Model(rb, "f64", device=dev)
    rid = np.array([0, 2, 7, 1, -1, 1], np.int32)          # 7 and -1 are not robots
    n = np.array([5, 3, 0, 9, 0, 9])
    off = synth.offsets_of(n)
    q, qd, tau = synth.make_state(n, cfg=3)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = torch.full((len(q),), 123.0, dtype=torch.float64, device=dev)
    model.forward_persistent(t(q), t(qd), t(tau), batch=6, robot_id=t(rid), offsets=t(off), out=out)
    plain = model.forward(t(q), t(qd), t(tau), batch=6, algo="abia", robot_id=t(rid), offsets=t(off))
    assert torch.equal(out, plain)


def test_auto_on_a_ragged_batch_takes_the_persistent_launch(dev):
    """AUTO on a batch with offsets, where the tuned table picks ABIA, runs the
    persistent length-sorted launch: its workspace size is the persistent one,
    and its q-ddot equals the plain ABIA launch bit for bit. Where the table
    picks another algorithm, AUTO equals that algorithm."""
    from paper_1609_06779_amd import fd, tune

    lengths = synth.ragged_lengths(65536, 4, 128, cfg=3)       # the tuned table picks ABIA at this size
    rb = synth.make_robots(lengths, cfg=3)
    q, qd, tau = synth.make_state(lengths, cfg=3)
    model = fd.Model(rb, "f64", device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev) for a in (q, qd, tau))
    toff = torch.from_numpy(rb.offsets).to(dev)
    batch = len(lengths)
    picked = tune.best_algo("f64", int(lengths.max()), batch)
    auto = model.forward(tq, tqd, ttau, batch=batch, algo="auto", offsets=toff)
    if picked == "abia":
        assert model.workspace_size(batch, "auto", offsets=toff) == model.persistent_workspace(batch, 0, offsets=toff).numel()
    ref = model.forward(tq, tqd, ttau, batch=batch, algo=picked, offsets=toff)
    assert torch.equal(auto, ref), picked


def test_full_size_ragged_batch_sampled(dev):
    """The ragged workload at full size (100000 chains, n ~ U{4..256}, each its own
    robot) in the launch the benchmark times (AUTO: the persistent length-sorted
    launch): 600 chains spread over every length band against the oracle, within
    the FP64 cap, and every output finite."""
    from paper_1609_06779_amd import fd

    lengths = synth.ragged_lengths(100000, 4, 256, cfg=3)
    rb = synth.make_robots(lengths, cfg=3)
    q, qd, tau = synth.make_state(lengths, cfg=3)
    off = rb.offsets
    model = fd.Model(rb, "f64", device=dev)
    tq, tqd, ttau = (torch.from_numpy(a).to(dev) for a in (q, qd, tau))
    toff = torch.from_numpy(off).to(dev)
    out = model.forward(tq, tqd, ttau, batch=len(lengths), algo="auto", offsets=toff).cpu().numpy()
    assert np.all(np.isfinite(out))
    rng = np.random.default_rng(31)
    order = np.argsort(lengths, kind="stable")
    pick = np.unique(np.concatenate([order[np.linspace(0, len(order) - 1, 300).astype(int)],
                                     rng.choice(len(lengths), 300, replace=False)]))
    sub = rb.take(pick)
    idx = np.concatenate([np.arange(off[b], off[b + 1]) for b in pick])
    ref = oracle.fd_exact(sub, q[idx], qd[idx], tau[idx])
    err = oracle.relative_error(out[idx], ref, sub.offsets)
    print(f"ragged 100000 sampled {len(pick)}: worst {err.max():.2e}", flush=True)
    assert np.all(err <= CAP["f64"]), err.max()
