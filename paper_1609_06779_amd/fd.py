"""Torch-facing binding of the C-ABI: device tensors in, device tensors out.

Every call hands raw device pointers and the current HIP stream to libfd.so;
nothing here computes. PyTorch only provides device memory and streams.
"""
from __future__ import annotations

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


def _dev_tensor(x, dtype, device, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (got {x.device})")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {x.dtype})")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class Model:
    """A robot set uploaded to the GPU in one precision ('f64' or 'f32').

    ``robots`` needs the per-link arrays n_links, axis, home_rot, offset, mass,
    com, inertia and a gravity 3-vector (packed robot after robot).
    """

    def __init__(self, robots, dtype: str = "f64", device=None):
        lib = _lib.load()
        if dtype not in _lib.DTYPES:
            raise ValueError(f"dtype must be one of {list(_lib.DTYPES)}")
        self.dtype = dtype
        self.torch_dtype = _TORCH_DTYPE[dtype]
        self.device = torch.device(device if device is not None else "cuda")
        self.n_links = _c(robots.n_links, np.int32)
        self._keep = dict(axis=_c(robots.axis), home=_c(robots.home_rot), off=_c(robots.offset),
                          mass=_c(robots.mass), com=_c(robots.com), inertia=_c(robots.inertia))
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
    def _batch(self, batch: int, robot_id=None, offsets=None) -> _lib.Batch:
        b = _lib.Batch()
        b.batch = int(batch)
        b.robot_id = _ptr(_dev_tensor(robot_id, torch.int32, self.device, "robot_id")).value if robot_id is not None else None
        b.offsets = _ptr(_dev_tensor(offsets, torch.int64, self.device, "offsets")).value if offsets is not None else None
        return b

    def workspace_size(self, batch: int, algo: str = "auto", robot_id=None, offsets=None) -> int:
        n = ctypes.c_size_t()
        b = self._batch(batch, robot_id, offsets)
        _lib.check(_lib.load().fd_workspace_size(self._h, ctypes.byref(b), _lib.ALGOS[algo], ctypes.byref(n)),
                   "fd_workspace_size")
        return int(n.value)

    def workspace(self, batch: int, algo: str = "auto", robot_id=None, offsets=None):
        nbytes = self.workspace_size(batch, algo, robot_id, offsets)
        return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)

    def forward(self, q, qd, tau, batch: int, algo: str = "auto", robot_id=None, offsets=None, out=None,
                workspace=None, stream=None):
        """qdd = M(q)^-1 (tau - tau_bias(q, qd)) for every chain of the batch."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        qd = _dev_tensor(qd, dt, self.device, "qd")
        tau = _dev_tensor(tau, dt, self.device, "tau")
        if out is None:
            out = torch.empty_like(q)
        _dev_tensor(out, dt, self.device, "out")
        b = self._batch(batch, robot_id, offsets)
        if workspace is None:
            workspace = self.workspace(batch, algo, robot_id, offsets)
        _lib.check(_lib.load().fd_forward(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(tau), _ptr(out),
                                          _lib.ALGOS[algo], _ptr(workspace), workspace.numel(), _stream(stream)),
                   "fd_forward")
        return out

    def inverse(self, q, qd, qdd, batch: int, gravity: bool = True, robot_id=None, offsets=None, out=None,
                stream=None):
        """tau = M(q) qdd + tau_bias(q, qd) (qdd None = 0)."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        qd = _dev_tensor(qd, dt, self.device, "qd")
        if qdd is not None:
            _dev_tensor(qdd, dt, self.device, "qdd")
        if out is None:
            out = torch.empty_like(q)
        b = self._batch(batch, robot_id, offsets)
        _lib.check(_lib.load().fd_inverse(self._h, ctypes.byref(b), _ptr(q), _ptr(qd), _ptr(qdd), int(bool(gravity)),
                                          _ptr(out), _stream(stream)), "fd_inverse")
        return out

    def joint_inertia(self, q, batch: int, n: int, robot_id=None, out=None, stream=None):
        """M(q) of every chain of a uniform batch, shape [batch, n, n]."""
        dt = self.torch_dtype
        q = _dev_tensor(q, dt, self.device, "q")
        if out is None:
            out = torch.empty((batch, n, n), dtype=dt, device=self.device)
        b = self._batch(batch, robot_id, None)
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
