"""Torch-facing binding of the C-ABI: device tensors in, device tensors out.

Every call hands raw device pointers and the current HIP stream to libfd.so;
nothing here computes. PyTorch only provides device memory and streams.
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib

_TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _alloc_on(stream):
    """Context for the default outputs and workspaces of a call: allocate them on the
    stream the call enqueues on, so the caching allocator does not hand their
    blocks to other work while that stream may still be writing them."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _dev_tensor(x, dtype, device, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not x.is_cuda:
        raise ValueError(f"{name} must live on the GPU (got {x.device})")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {x.dtype})")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


_TABLE_LOADED = False


def _load_tuning():
    """Hand the tuned AUTO table (measured on gfx950 by tune.py) to the library once."""
    global _TABLE_LOADED
    if not _TABLE_LOADED:
        from . import tune
        tune.load_table()
        _TABLE_LOADED = True


class Model:
    """A robot set uploaded to the GPU in one precision ('f64' or 'f32').

    ``robots`` needs the per-link arrays n_links, axis, home_rot, offset, mass,
    com, inertia and a gravity 3-vector (packed robot after robot); an optional
    ``parent`` array (parent of each link within its robot, -1 = base) makes
    the robots branched. Branched models run every path but the CFA (see the C header).
    """

    def __init__(self, robots, dtype: str = "f64", device=None):
        lib = _lib.load()
        _load_tuning()
        if dtype not in _lib.DTYPES:
            raise ValueError(f"dtype must be one of {list(_lib.DTYPES)}")
        self.dtype = dtype
        self.torch_dtype = _TORCH_DTYPE[dtype]
        self.device = torch.device(device if device is not None else "cuda")
        self.n_links = _c(robots.n_links, np.int32)
        # the common length when every robot has the same one (0 otherwise), for the size checks
        self._uniform_n = int(self.n_links[0]) if len(self.n_links) and np.all(self.n_links == self.n_links[0]) else 0
        self._keep = dict(axis=_c(robots.axis), home=_c(robots.home_rot), off=_c(robots.offset),
                          mass=_c(robots.mass), com=_c(robots.com), inertia=_c(robots.inertia))
        par = getattr(robots, "parent", None)
        self._keep["parent"] = None if par is None else _c(par, np.int32)
        starts = np.repeat(np.cumsum(self.n_links, dtype=np.int64) - self.n_links, self.n_links)
        self.branched = par is not None and bool(np.any(np.asarray(par) != np.arange(len(par)) - starts - 1))
        d = _lib.ModelDesc()
        dp = ctypes.POINTER(ctypes.c_double)
        d.num_robots = len(self.n_links)
        d.n_links = self.n_links.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.axis = self._keep["axis"].ctypes.data_as(dp)
        d.home_rot = self._keep["home"].ctypes.data_as(dp)
        d.offset = self._keep["off"].ctypes.data_as(dp)
        d.mass = self._keep["mass"].ctypes.data_as(dp)
        d.com = self._keep["com"].ctypes.data_as(dp)
        d.inertia = self._keep["inertia"].ctypes.data_as(dp)
        if self._keep["parent"] is not None:
            d.parent = self._keep["parent"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        for k in range(3):
            d.gravity[k] = float(robots.gravity[k])
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.fd_init(ctypes.byref(d), _lib.DTYPES[dtype], ctypes.byref(handle)), "fd_init")
        self._h = handle
        self._keep = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def max_links(self, algo: str = "auto") -> int:
        return int(_lib.load().fd_max_links(self._h, _lib.ALGOS[algo]))

    # ---- batches ----
    def _batch(self, batch: int, robot_id=None, offsets=None, max_links: int = 0, state=()) -> _lib.Batch:
        """The batch descriptor, after the size checks the library cannot make on
        raw pointers: robot_id needs `batch` entries, offsets `batch + 1`, and with
        no offsets on a model whose robots share one length n, every per-link
        array in `state` needs batch * n entries (per-chain offsets live on the
        device and are the caller's to keep within the arrays)."""
        if robot_id is not None and robot_id.numel() < batch:
            raise ValueError(f"robot_id has {robot_id.numel()} entries for a batch of {batch}")
        if offsets is not None and offsets.numel() < batch + 1:
            raise ValueError(f"offsets has {offsets.numel()} entries for a batch of {batch} (needs batch + 1)")
        uni = getattr(self, "_uniform_n", None)
        if uni is None:
            uni = int(self.n_links[0]) if len(self.n_links) and np.all(self.n_links == self.n_links[0]) else 0
        if offsets is None and uni:
            need = int(batch) * uni
            for name, t in state:
                if t is not None and t.numel() < need:
                    raise ValueError(f"{name} has {t.numel()} entries; {batch} chains of {uni} links need {need}")
        b = _lib.Batch()
        b.batch = int(batch)
        b.max_links = int(max_links)
        b.robot_id = _ptr(_dev_tensor(robot_id, torch.int32, self.device, "robot_id")).value if robot_id is not None else None
        b.offsets = _ptr(_dev_tensor(offsets, torch.int64, self.device, "offsets")).value if offsets is not None else None
        return b

    def _shape_batch(self, batch: int, ragged: bool, with_ids: bool, max_links: int) -> _lib.Batch:
        """A batch descriptor for the size and choice queries. They read no device
        memory (only whether robot_id and offsets are NULL matters), so a small
        device buffer of the model's stands in for both."""
        if getattr(self, "_marker", None) is None:
            self._marker = torch.zeros(1, dtype=torch.int64, device=self.device)
        b = _lib.Batch()
        b.batch = int(batch)
        b.max_links = int(max_links)
        b.robot_id = self._marker.data_ptr() if with_ids else None
        b.offsets = self._marker.data_ptr() if ragged else None
        return b

    def workspace_bytes(self, batch: int, algo: str = "auto", ragged: bool = False, with_ids: bool = False,
                        max_links: int = 0) -> int:
        """fd_workspace_size for a batch of this shape (chain offsets, robot ids or
        not), before any device buffer of it exists."""
        n = ctypes.c_size_t()
        b = self._shape_batch(batch, ragged, with_ids, max_links)
        _lib.check(_lib.load().fd_workspace_size(self._h, ctypes.byref(b), _lib.ALGOS[algo], ctypes.byref(n)),
                   "fd_workspace_size")
        return int(n.value)

    def auto_algo(self, batch: int, ragged: bool = False, with_ids: bool = False, max_links: int = 0):
        """(algorithm name, persistent launch?) that algo="auto" takes for a batch of this shape."""
        a, p = ctypes.c_int(), ctypes.c_int()
        b = self._shape_batch(batch, ragged, with_ids, max_links)
        _lib.check(_lib.load().fd_auto_algo(self._h, ctypes.byref(b), ctypes.byref(a), ctypes.byref(p)),
                   "fd_auto_algo")
        return {v: k for k, v in _lib.ALGOS.items()}[a.value], bool(p.value)

    def workspace_size(self, batch: int, algo: str = "auto", robot_id=None, offsets=None, max_links: int = 0) -> int:
        n = ctypes.c_size_t()
        b = self._batch(batch, robot_id, offsets, max_links)
        _lib.check(_lib.load().fd_workspace_size(self._h, ctypes.byref(b), _lib.ALGOS[algo], ctypes.byref(n)),
                   "fd_workspace_size")
        return int(n.value)

    def workspace(self, batch: int, algo: str = "auto", robot_id=None, offsets=None, max_links: int = 0,
                  stream=None):
        nbytes = self.workspace_size(batch, algo, robot_id, offsets, max_links)
        with _alloc_on(stream):
            return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)

    def forward(self, q, qd, tau, batch: int, algo: str = "auto", robot_id=None, offsets=None, out=None,
                workspace=None, stream=None, max_links: int = 0):
        """qdd = M(q)^-1 (tau - tau_bias(q, qd)) for every chain of the batch.
        max_links > 0 bounds the links of every chain (lane groups are sized to it;
        a longer chain is not solved and gets NaN)."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        qd = _dev_tensor(qd, dt, self.device, "qd")
        tau = _dev_tensor(tau, dt, self.device, "tau")
        # enter the stream's context only to allocate (it costs microseconds per call)
        with _alloc_on(stream) if (out is None or workspace is None) else contextlib.nullcontext():
            if out is None:
                out = torch.empty_like(q)
            _dev_tensor(out, dt, self.device, "out")
            b = self._batch(batch, robot_id, offsets, max_links,
                            state=(("q", q), ("qd", qd), ("tau", tau), ("out", out)))
            if workspace is None:
                workspace = self.workspace(batch, algo, robot_id, offsets, max_links, stream)
        _lib.check(_lib.load().fd_forward(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(tau), _ptr(out),
                                          _lib.ALGOS[algo], _ptr(workspace), workspace.numel(), _stream(stream)),
                   "fd_forward")
        return out

    def forward_noalloc(self, q, qd, tau, out, batch: int, algo: str = "auto", robot_id=None, offsets=None,
                        stream=None, max_links: int = 0):
        """fd_forward_noalloc: forward() with the library's own per-GPU scratch
        array as the workspace, so the call allocates nothing (out is required).
        Calls that overlap on one GPU share that array and race."""
        dt = self.torch_dtype
        for name, t in (("q", q), ("qd", qd), ("tau", tau), ("out", out)):
            _dev_tensor(t, dt, self.device, name)
        b = self._batch(batch, robot_id, offsets, max_links,
                        state=(("q", q), ("qd", qd), ("tau", tau), ("out", out)))
        _lib.check(_lib.load().fd_forward_noalloc(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(tau), _ptr(out),
                                                  _lib.ALGOS[algo], _stream(stream)), "fd_forward_noalloc")
        return out

    def persistent_workspace(self, batch: int, grid: int = 0, robot_id=None, offsets=None):
        n = ctypes.c_size_t()
        b = self._batch(batch, robot_id, offsets)
        _lib.check(_lib.load().fd_persistent_workspace_size(self._h, ctypes.byref(b), int(grid), ctypes.byref(n)),
                   "fd_persistent_workspace_size")
        return torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=self.device)

    def forward_persistent(self, q, qd, tau, batch: int, grid: int = 0, robot_id=None, offsets=None, out=None,
                           workspace=None, stream=None):
        """qdd for a (ragged) batch in one persistent launch, chains sorted by length on the device."""
        dt = self.torch_dtype
        for name, t in (("q", q), ("qd", qd), ("tau", tau)):
            _dev_tensor(t, dt, self.device, name)
        with _alloc_on(stream):
            out = torch.empty_like(q) if out is None else _dev_tensor(out, dt, self.device, "out")
            b = self._batch(batch, robot_id, offsets, state=(("q", q), ("qd", qd), ("tau", tau), ("out", out)))
            if workspace is None:
                workspace = self.persistent_workspace(batch, grid, robot_id, offsets)
        _lib.check(_lib.load().fd_forward_persistent(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(tau),
                                                     _ptr(out), int(grid), _ptr(workspace), workspace.numel(),
                                                     _stream(stream)), "fd_forward_persistent")
        return out

    def backward_workspace(self, batch: int, algo: str = "abia", robot_id=None, offsets=None, max_links: int = 0,
                           stream=None):
        n = ctypes.c_size_t()
        b = self._batch(batch, robot_id, offsets, max_links)
        _lib.check(_lib.load().fd_backward_workspace_size(self._h, ctypes.byref(b), _lib.ALGOS[algo],
                                                          ctypes.byref(n)), "fd_backward_workspace_size")
        with _alloc_on(stream):
            return torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=self.device)

    def backward(self, q, qd, qdd, grad_qdd, batch: int, algo: str = "abia", tau=None, robot_id=None, offsets=None,
                 grad_q=None, grad_qd=None, grad_tau=None, accumulate: bool = False, workspace=None, stream=None,
                 max_links: int = 0):
        """Vector-Jacobian product of forward dynamics at (q, qd, qdd = FD(q, qd, tau)):
        returns (grad_q, grad_qd, grad_tau) for the cotangent grad_qdd. ``algo`` is
        the factorisation of M^-1 that gives grad_tau = M^-1 grad_qdd; qdd None
        recomputes it from tau by the same algorithm."""
        dt = self.torch_dtype
        for name, t in (("q", q), ("qd", qd), ("grad_qdd", grad_qdd)):
            _dev_tensor(t, dt, self.device, name)
        if qdd is None and tau is None:
            raise ValueError("give qdd, or tau to recompute it")
        for name, t in (("qdd", qdd), ("tau", tau)):
            if t is not None:
                _dev_tensor(t, dt, self.device, name)
        with _alloc_on(stream):
            grad_q = torch.empty_like(q) if grad_q is None else _dev_tensor(grad_q, dt, self.device, "grad_q")
            grad_qd = torch.empty_like(q) if grad_qd is None else _dev_tensor(grad_qd, dt, self.device, "grad_qd")
            grad_tau = torch.empty_like(q) if grad_tau is None else _dev_tensor(grad_tau, dt, self.device, "grad_tau")
            b = self._batch(batch, robot_id, offsets, max_links,
                            state=(("q", q), ("qd", qd), ("tau", tau), ("qdd", qdd), ("grad_qdd", grad_qdd),
                                   ("grad_q", grad_q), ("grad_qd", grad_qd), ("grad_tau", grad_tau)))
            if workspace is None:
                workspace = self.backward_workspace(batch, algo, robot_id, offsets, max_links)
        _lib.check(_lib.load().fd_backward(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(tau), _ptr(qdd),
                                           _ptr(grad_qdd), _ptr(grad_q), _ptr(grad_qd), _ptr(grad_tau),
                                           _lib.ALGOS[algo], int(bool(accumulate)), _ptr(workspace),
                                           workspace.numel(), _stream(stream)), "fd_backward")
        return grad_q, grad_qd, grad_tau

    def euler_step(self, q, qd, qdd, dt: float, q_next=None, qd_next=None, stream=None):
        """qd_next = qd + dt qdd, q_next = q + dt qd_next (outputs may be the inputs)."""
        q_next = torch.empty_like(q) if q_next is None else q_next
        qd_next = torch.empty_like(q) if qd_next is None else qd_next
        _lib.check(_lib.load().fd_euler_step(_lib.DTYPES[self.dtype], q.numel(), float(dt), _ptr(q), _ptr(qd),
                                             _ptr(qdd), _ptr(q_next), _ptr(qd_next), _stream(stream)), "fd_euler_step")
        return q_next, qd_next

    def euler_step_backward(self, grad_q_next, grad_qd_next, dt: float, grad_q=None, grad_qd=None, grad_qdd=None,
                            stream=None):
        grad_q = torch.empty_like(grad_q_next) if grad_q is None else grad_q
        grad_qd = torch.empty_like(grad_q_next) if grad_qd is None else grad_qd
        grad_qdd = torch.empty_like(grad_q_next) if grad_qdd is None else grad_qdd
        _lib.check(_lib.load().fd_euler_step_backward(_lib.DTYPES[self.dtype], grad_q_next.numel(), float(dt),
                                                      _ptr(grad_q_next), _ptr(grad_qd_next), _ptr(grad_q),
                                                      _ptr(grad_qd), _ptr(grad_qdd), _stream(stream)),
                   "fd_euler_step_backward")
        return grad_q, grad_qd, grad_qdd

    def inverse(self, q, qd, qdd, batch: int, gravity: bool = True, robot_id=None, offsets=None, out=None,
                stream=None):
        """tau = M(q) qdd + tau_bias(q, qd) (qdd None = 0)."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        qd = _dev_tensor(qd, dt, self.device, "qd")
        if qdd is not None:
            _dev_tensor(qdd, dt, self.device, "qdd")
        out = torch.empty_like(q) if out is None else _dev_tensor(out, dt, self.device, "out")
        b = self._batch(batch, robot_id, offsets, state=(("q", q), ("qd", qd), ("qdd", qdd), ("out", out)))
        _lib.check(_lib.load().fd_inverse(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(qdd), int(bool(gravity)),
                                          _ptr(out), _stream(stream)), "fd_inverse")
        return out

    def joint_inertia(self, q, batch: int, n: int, robot_id=None, out=None, stream=None):
        """M(q) of every chain of a uniform batch, shape [batch, n, n]."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        if len(self.n_links) and int(self.n_links[0]) != n:      # uniform batches: every chain has n_links[0]
            raise ValueError(f"n = {n}, but the batch's chains have {int(self.n_links[0])} links")
        if out is None:
            out = torch.empty((batch, n, n), dtype=dt, device=self.device)
        elif _dev_tensor(out, dt, self.device, "out").numel() < batch * n * n:
            raise ValueError(f"out has {out.numel()} entries; {batch} matrices of {n} x {n} need {batch * n * n}")
        b = self._batch(batch, robot_id, None, state=(("q", q),))
        _lib.check(_lib.load().fd_joint_inertia(self._h, ctypes.byref(b), _ptr(q), _ptr(out), _stream(stream)),
                   "fd_joint_inertia")
        return out


def scan6(b, c, offsets, max_len: int, reverse: bool = False, out=None, stream=None):
    """x_i = B_i x_{i-1} + c_i per segment (reverse: x_i = B_i x_{i+1} + c_i)."""
    dtype = "f64" if b.dtype == torch.float64 else "f32"
    dt = _TORCH_DTYPE[dtype]
    dev = b.device
    _dev_tensor(b, dt, dev, "b")
    _dev_tensor(c, dt, dev, "c")
    _dev_tensor(offsets, torch.int64, dev, "offsets")
    if out is None:
        out = torch.empty_like(c)
    _lib.check(_lib.load().fd_scan6(_lib.DTYPES[dtype], offsets.numel() - 1, _ptr(offsets), int(max_len), _ptr(b),
                                    _ptr(c), int(bool(reverse)), _ptr(out), _stream(stream)), "fd_scan6")
    return out


def btd_solve6(d, u, r, offsets, max_len: int, out=None, status=None, stream=None):
    """Odd-even elimination solve of SPD block tri-diagonal systems with 6x6 blocks."""
    dtype = "f64" if d.dtype == torch.float64 else "f32"
    dt = _TORCH_DTYPE[dtype]
    dev = d.device
    for name, t in (("d", d), ("u", u), ("r", r)):
        _dev_tensor(t, dt, dev, name)
    _dev_tensor(offsets, torch.int64, dev, "offsets")
    if out is None:
        out = torch.empty_like(r)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    _lib.check(_lib.load().fd_btd_solve6(_lib.DTYPES[dtype], offsets.numel() - 1, _ptr(offsets), int(max_len),
                                         _ptr(d), _ptr(u), _ptr(r), _ptr(out), _ptr(status), _stream(stream)),
               "fd_btd_solve6")
    return out, status


class _ForwardDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, qd, tau, model, batch, algo, robot_id, offsets):
        qdd = model.forward(q.detach(), qd.detach(), tau.detach(), batch=batch, algo=algo, robot_id=robot_id,
                            offsets=offsets)
        ctx.model, ctx.batch, ctx.robot_id, ctx.offsets, ctx.algo = model, batch, robot_id, offsets, algo
        ctx.save_for_backward(q.detach(), qd.detach(), qdd)
        return qdd

    @staticmethod
    def backward(ctx, grad_qdd):
        q, qd, qdd = ctx.saved_tensors
        gq, gqd, gtau = ctx.model.backward(q, qd, qdd, grad_qdd.contiguous(), batch=ctx.batch, algo=ctx.algo,
                                           robot_id=ctx.robot_id, offsets=ctx.offsets)
        return gq, gqd, gtau, None, None, None, None, None


def forward_dynamics(model: Model, q, qd, tau, batch: int, algo: str = "auto", robot_id=None, offsets=None):
    """Differentiable qdd = FD(q, qd, tau): gradients come from fd_backward with the
    same algorithm (grad_tau = M^-1 grad_qdd by the factorisation that gave qdd)."""
    return _ForwardDynamics.apply(q, qd, tau, model, batch, algo, robot_id, offsets)


class _Rollout(torch.autograd.Function):
    """T semi-implicit Euler steps of forward dynamics; the backward pass keeps
    (q, qd) every ``every`` steps and recomputes each segment before reversing it."""

    @staticmethod
    def forward(ctx, q0, qd0, taus, model, batch, dt, every, algo):
        n_steps = taus.shape[0]
        q, qd = q0.detach().clone(), qd0.detach().clone()
        qdd = torch.empty_like(q)
        ws = model.workspace(batch, algo)
        checkpoints = []
        for t in range(n_steps):
            if t % every == 0:
                checkpoints.append((q.clone(), qd.clone()))
            model.forward(q, qd, taus[t], batch=batch, algo=algo, out=qdd, workspace=ws)
            model.euler_step(q, qd, qdd, dt, q_next=q, qd_next=qd)
        ctx.model, ctx.batch, ctx.dt, ctx.every, ctx.algo = model, batch, dt, every, algo
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(taus.detach())
        return q, qd

    @staticmethod
    def backward(ctx, gq_t, gqd_t):
        (taus,) = ctx.saved_tensors
        model, batch, dt, every, algo = ctx.model, ctx.batch, ctx.dt, ctx.every, ctx.algo
        n_steps = taus.shape[0]
        gq = gq_t.detach().clone().contiguous()
        gqd = gqd_t.detach().clone().contiguous()
        gtaus = torch.zeros_like(taus)
        gqdd = torch.empty_like(gq)
        fws = model.workspace(batch, algo)
        bws = model.backward_workspace(batch, algo)
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            t0 = seg * every
            t1 = min(n_steps, t0 + every)
            q, qd = ctx.checkpoints[seg]
            states = []
            q, qd = q.clone(), qd.clone()
            for t in range(t0, t1):                      # recompute the segment
                qdd = torch.empty_like(q)
                model.forward(q, qd, taus[t], batch=batch, algo=algo, out=qdd, workspace=fws)
                states.append((q, qd, qdd))
                q, qd = model.euler_step(q, qd, qdd, dt)
            for t in range(t1 - 1, t0 - 1, -1):          # reverse it
                qs, qds, qdds = states[t - t0]
                model.euler_step_backward(gq, gqd, dt, grad_q=gq, grad_qd=gqd, grad_qdd=gqdd)
                model.backward(qs, qds, qdds, gqdd, batch=batch, algo=algo, grad_q=gq, grad_qd=gqd,
                               grad_tau=gtaus[t], accumulate=True, workspace=bws)
        return gq, gqd, gtaus, None, None, None, None, None


def rollout(model: Model, q0, qd0, taus, batch: int, dt: float, every: int = 10, algo: str = "auto"):
    """Differentiable (q_T, qd_T) after T = taus.shape[0] semi-implicit Euler steps of
    forward dynamics with step dt, checkpointing (q, qd) every ``every`` steps."""
    return _Rollout.apply(q0, qd0, taus, model, batch, float(dt), int(every), algo)


class RolloutGraph:
    """A rollout of fixed shape (T semi-implicit Euler steps of forward dynamics,
    no gradient) recorded once into a HIP graph and replayed. For small batches a
    step is a few microseconds of kernel time, so launching 2 T kernels from the
    host costs more than running them; a replay submits them all at once.

    The graph owns its buffers: ``run`` copies (q0, qd0, taus) into them, replays
    and returns the graph's (q_T, qd_T), which the next ``run`` overwrites. The
    recorded path clears no memory and allocates nothing (the workspace is taken
    before recording)."""

    def __init__(self, model: Model, batch: int, steps: int, dt: float, algo: str = "abia", robot_id=None,
                 offsets=None, n_state: int = 0):
        if algo == "auto":
            raise ValueError("a recorded rollout needs a fixed algorithm (abia, jsiia or cfa)")
        if n_state <= 0:
            if offsets is not None or len(model.n_links) == 0 or np.any(model.n_links != model.n_links[0]):
                raise ValueError("give n_state (total links) for ragged batches")
            n_state = int(batch) * int(model.n_links[0])
        dev, dt_ = model.device, model.torch_dtype
        self.model, self.batch, self.steps, self.dt, self.algo = model, int(batch), int(steps), float(dt), algo
        self.robot_id, self.offsets = robot_id, offsets
        self.q = torch.zeros(n_state, dtype=dt_, device=dev)
        self.qd = torch.zeros_like(self.q)
        self.qdd = torch.zeros_like(self.q)
        self.taus = torch.zeros((self.steps, n_state), dtype=dt_, device=dev)
        self.ws = model.workspace(batch, algo, robot_id, offsets)
        side = torch.cuda.Stream(device=dev)           # torch records graphs after a warm-up off the main stream
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._steps()
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._steps()

    def _steps(self):
        m = self.model
        for t in range(self.steps):
            m.forward(self.q, self.qd, self.taus[t], batch=self.batch, algo=self.algo, robot_id=self.robot_id,
                      offsets=self.offsets, out=self.qdd, workspace=self.ws)
            m.euler_step(self.q, self.qd, self.qdd, self.dt, q_next=self.q, qd_next=self.qd)

    def run(self, q0, qd0, taus):
        """(q_T, qd_T) from (q0, qd0) under the torques taus [T, links]."""
        self.q.copy_(q0)
        self.qd.copy_(qd0)
        self.taus.copy_(taus)
        self.graph.replay()
        return self.q, self.qd
