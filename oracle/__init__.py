"""CPU oracle for batched forward dynamics of serial chains (and branched trees).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may call it; the library's product path never does. It shares
no code with the HIP path and imports nothing from it.

``fd`` is the plain definition qdd = M(q)^-1 (tau - tau_bias(q, qd))
(Sec. II-C, eq. (eq-motion), (tau-bias)): M by composite rigid bodies,
tau_bias by recursive Newton-Euler at zero acceleration, a dense Cholesky
solve. The C source (``fd_oracle.c``) is compiled with contraction off so that
its rounding follows the written order.

``dense`` holds numpy renderings of the paper's global matrix formulas and of
the building blocks (scan, odd-even elimination, the ABIA and CFA
factorisations) used to pin each step of the method.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("fd_oracle.c", "fd_oracle_cx.c", "fd_oracle_ld.c", "fd_core.inc",
                                          "fd_chain.h")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (plain -O2, no FMA contraction)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wno-unused-function", "-o", tmp, _SRCS[0], _SRCS[1], _SRCS[2], "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        model = [_d] * 7 + [_i32]
        lib.oracle_rnea_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _d, _d, ctypes.c_int, _d, ctypes.c_int]
        lib.oracle_crba_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _i64, _d, ctypes.c_int]
        lib.oracle_fd_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _d, _d, _d, ctypes.c_int]
        lib.oracle_fd_ld_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _d, _d, _d, ctypes.c_int]
        lib.oracle_fd_ld_batch.restype = ctypes.c_int
        lib.oracle_fk_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _d, _d, ctypes.c_int]
        lib.oracle_energy_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d, _d, _d, _d, ctypes.c_int]
        lib.oracle_link_rotation.argtypes = [_d, _d, ctypes.c_double, _d]
        lib.oracle_adjoint.argtypes = [_d, _d, ctypes.c_int, _d]
        lib.oracle_spatial_inertia.argtypes = [ctypes.c_double, _d, _d, _d]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_fd_jvp_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d] * 8 + [ctypes.c_int]
        lib.oracle_fd_jvp_batch.restype = ctypes.c_int
        lib.oracle_rnea_jvp_batch.argtypes = [ctypes.c_int, _i64, _i64] + model + [_d] * 6 + [ctypes.c_int, _d, ctypes.c_int]
        lib.oracle_rnea_jvp_batch.restype = ctypes.c_int
        for f in (lib.oracle_rnea_batch, lib.oracle_crba_batch, lib.oracle_fd_batch,
                  lib.oracle_fk_batch, lib.oracle_energy_batch):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, dtype=np.float64):
    return a.ctypes.data_as(_i64 if dtype == np.int64 else _d)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class _Model:
    """Contiguous float64 copies of a robot set's per-link arrays."""

    def __init__(self, robots):
        self.axis = _c(robots.axis)
        self.home_rot = _c(robots.home_rot)
        self.offset = _c(robots.offset)
        self.mass = _c(robots.mass)
        self.com = _c(robots.com)
        self.inertia = _c(robots.inertia)
        self.gravity = _c(robots.gravity)
        par = getattr(robots, "parent", None)
        self.parent = None if par is None else _c(par, np.int32)

    def args(self):
        return [_p(self.axis), _p(self.home_rot), _p(self.offset), _p(self.mass), _p(self.com),
                _p(self.inertia), _p(self.gravity),
                None if self.parent is None else self.parent.ctypes.data_as(_i32)]


def _offsets(robots, offsets):
    if offsets is None:
        n = np.asarray(robots.n_links, dtype=np.int64)
        offsets = np.zeros(len(n) + 1, np.int64)
        np.cumsum(n, out=offsets[1:])
    return _c(offsets, np.int64)


def _mstart(model_start):
    return None if model_start is None else _p(_c(model_start, np.int64), np.int64)


def max_threads() -> int:
    """Threads the last batch call ran with (all host cores unless a count was given)."""
    return int(_load().oracle_max_threads())


def fd(robots, q, qd, tau, offsets=None, model_start=None, threads: int = 0):
    """qdd for every chain. Chains whose M is not numerically SPD come back as NaN."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    q, qd, tau = _c(q), _c(qd), _c(tau)
    out = np.empty_like(q)
    ms = None if model_start is None else _c(model_start, np.int64)
    lib.oracle_fd_batch(len(off) - 1, _p(off, np.int64), None if ms is None else _p(ms, np.int64),
                        *m.args(), _p(q), _p(qd), _p(tau), _p(out), int(threads))
    return out


def fd_exact(robots, q, qd, tau, offsets=None, model_start=None, threads: int = 0):
    """``fd`` evaluated in long double (64-bit significand) from the same double
    inputs, rounded to double at the end: the forward-dynamics value to within
    about one unit in the last place of double wherever cond(M) stays below
    2^11, so a result compared with it is charged with its own error only."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    q, qd, tau = _c(q), _c(qd), _c(tau)
    out = np.empty_like(q)
    ms = None if model_start is None else _c(model_start, np.int64)
    lib.oracle_fd_ld_batch(len(off) - 1, _p(off, np.int64), None if ms is None else _p(ms, np.int64),
                           *m.args(), _p(q), _p(qd), _p(tau), _p(out), int(threads))
    return out


def rnea(robots, q, qd, qdd=None, gravity: bool = True, offsets=None, model_start=None, threads: int = 0):
    """Inverse dynamics tau = ID(q, qd, qdd) (qdd None = 0)."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    q, qd = _c(q), _c(qd)
    qa = None if qdd is None else _c(qdd)
    out = np.empty_like(q)
    ms = None if model_start is None else _c(model_start, np.int64)
    lib.oracle_rnea_batch(len(off) - 1, _p(off, np.int64), None if ms is None else _p(ms, np.int64),
                          *m.args(), _p(q), _p(qd), None if qa is None else _p(qa), int(bool(gravity)),
                          _p(out), int(threads))
    return out


def crba(robots, q, offsets=None, model_start=None, threads: int = 0):
    """Joint-space inertia matrices, one [n, n] array per chain."""
    lib = _load()
    off = _offsets(robots, offsets)
    n = np.diff(off)
    mstart = np.zeros(len(n) + 1, np.int64)
    np.cumsum(n * n, out=mstart[1:])
    m = _Model(robots)
    q = _c(q)
    out = np.empty(int(mstart[-1]))
    ms = None if model_start is None else _c(model_start, np.int64)
    lib.oracle_crba_batch(len(n), _p(off, np.int64), None if ms is None else _p(ms, np.int64),
                          *m.args(), _p(q), _p(mstart, np.int64), _p(out), int(threads))
    return [out[mstart[b]:mstart[b + 1]].reshape(int(n[b]), int(n[b])) for b in range(len(n))]


def fk(robots, q, offsets=None, threads: int = 0):
    """Base-frame rotation [N, 3, 3] and origin [N, 3] of every link frame."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    q = _c(q)
    rot = np.empty((len(q), 9))
    pos = np.empty((len(q), 3))
    lib.oracle_fk_batch(len(off) - 1, _p(off, np.int64), None, *m.args(), _p(q), _p(rot), _p(pos), int(threads))
    return rot.reshape(-1, 3, 3), pos


def energy(robots, q, qd, offsets=None, threads: int = 0):
    """(kinetic, potential) energy of every chain."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    q, qd = _c(q), _c(qd)
    b = len(off) - 1
    ke = np.empty(b)
    pe = np.empty(b)
    lib.oracle_energy_batch(b, _p(off, np.int64), None, *m.args(), _p(q), _p(qd), _p(ke), _p(pe), int(threads))
    return ke, pe


def fd_jvp(robots, q, qd, tau, dq, dqd, dtau, offsets=None, threads: int = 0):
    """(qdd, d qdd) with d qdd the derivative of forward dynamics along (dq, dqd, dtau),
    exact to rounding (complex step through the same arithmetic as ``fd``)."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    arrs = [_c(a) for a in (q, qd, tau, dq, dqd, dtau)]
    qdd = np.empty_like(arrs[0])
    dqdd = np.empty_like(arrs[0])
    lib.oracle_fd_jvp_batch(len(off) - 1, _p(off, np.int64), None, *m.args(), *[_p(a) for a in arrs], _p(qdd),
                            _p(dqdd), int(threads))
    return qdd, dqdd


def rnea_jvp(robots, q, qd, qdd, dq, dqd, dqdd, gravity: bool = True, offsets=None, threads: int = 0):
    """Derivative of tau = ID(q, qd, qdd) along (dq, dqd, dqdd) (complex step)."""
    lib = _load()
    off = _offsets(robots, offsets)
    m = _Model(robots)
    arrs = [_c(a) for a in (q, qd, qdd, dq, dqd, dqdd)]
    out = np.empty_like(arrs[0])
    lib.oracle_rnea_jvp_batch(len(off) - 1, _p(off, np.int64), None, *m.args(), *[_p(a) for a in arrs],
                              int(bool(gravity)), _p(out), int(threads))
    return out


def link_rotation(axis, home_rot, q):
    lib = _load()
    out = np.empty(9)
    lib.oracle_link_rotation(_p(_c(axis)), _p(_c(home_rot)), float(q), _p(out))
    return out.reshape(3, 3)


def adjoint(rot, pos, inverse: bool = False):
    lib = _load()
    out = np.empty(36)
    lib.oracle_adjoint(_p(_c(np.asarray(rot).reshape(9))), _p(_c(pos)), int(inverse), _p(out))
    return out.reshape(6, 6)


def spatial_inertia(mass, com, inertia6):
    lib = _load()
    out = np.empty(36)
    lib.oracle_spatial_inertia(float(mass), _p(_c(com)), _p(_c(inertia6)), _p(out))
    return out.reshape(6, 6)


def relative_error(x, ref, offsets):
    """Per-chain normwise relative error ||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d2 = np.add.reduceat((x - ref) ** 2, offsets[:-1]) if len(ref) else np.zeros(0)
    r2 = np.add.reduceat(ref ** 2, offsets[:-1]) if len(ref) else np.zeros(0)
    return np.sqrt(d2) / np.maximum(np.sqrt(r2), np.finfo(np.float64).tiny)
