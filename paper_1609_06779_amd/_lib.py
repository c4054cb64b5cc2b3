"""ctypes view of the C-ABI in include/fd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfd.so")

FD_OK, FD_ERR_INVALID_ARG, FD_ERR_UNSUPPORTED, FD_ERR_OUT_OF_MEMORY, FD_ERR_DEVICE, FD_ERR_WORKSPACE = 0, -1, -2, -3, -4, -5
ALGOS = {"abia": 0, "jsiia": 1, "cfa": 2, "auto": 3, "abia_scan": 4, "cfa_proj": 5}
DTYPES = {"f64": 0, "f32": 1}

# C-ABI entry points declared in include/fd.h
EXPORTS = ("fd_init", "fd_destroy", "fd_model_dtype", "fd_max_links", "fd_workspace_size", "fd_forward",
           "fd_persistent_workspace_size", "fd_forward_persistent",
           "fd_backward_workspace_size", "fd_backward", "fd_euler_step", "fd_euler_step_backward",
           "fd_inverse", "fd_joint_inertia", "fd_scan6", "fd_btd_solve6", "fd_set_auto_table", "fd_status_string",
           "fd_auto_algo", "fd_forward_noalloc", "fd_set_persistent_grid")
NOALLOC_SCRATCH_BYTES = 64 << 20          # FD_NOALLOC_SCRATCH_BYTES


class ModelDesc(ctypes.Structure):
    _fields_ = [
        ("num_robots", ctypes.c_int32),
        ("n_links", ctypes.POINTER(ctypes.c_int32)),
        ("axis", ctypes.POINTER(ctypes.c_double)),
        ("home_rot", ctypes.POINTER(ctypes.c_double)),
        ("offset", ctypes.POINTER(ctypes.c_double)),
        ("mass", ctypes.POINTER(ctypes.c_double)),
        ("com", ctypes.POINTER(ctypes.c_double)),
        ("inertia", ctypes.POINTER(ctypes.c_double)),
        ("gravity", ctypes.c_double * 3),
        ("parent", ctypes.POINTER(ctypes.c_int32)),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int32),
        ("robot_id", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
        ("max_links", ctypes.c_int32),
    ]


class FdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def load() -> ctypes.CDLL:
    """Load libfd.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1609_06779_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.fd_init.argtypes = [ctypes.POINTER(ModelDesc), ctypes.c_int, ctypes.POINTER(vp)]
    lib.fd_init.restype = ctypes.c_int
    lib.fd_destroy.argtypes = [vp]
    lib.fd_destroy.restype = None
    lib.fd_model_dtype.argtypes = [vp]
    lib.fd_model_dtype.restype = ctypes.c_int
    lib.fd_max_links.argtypes = [vp, ctypes.c_int]
    lib.fd_max_links.restype = i32
    lib.fd_workspace_size.argtypes = [vp, ctypes.POINTER(Batch), ctypes.c_int, ctypes.POINTER(sz)]
    lib.fd_workspace_size.restype = ctypes.c_int
    lib.fd_forward.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]
    lib.fd_forward.restype = ctypes.c_int
    lib.fd_forward_noalloc.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, vp, ctypes.c_int, vp]
    lib.fd_forward_noalloc.restype = ctypes.c_int
    lib.fd_persistent_workspace_size.argtypes = [vp, ctypes.POINTER(Batch), i32, ctypes.POINTER(sz)]
    lib.fd_persistent_workspace_size.restype = ctypes.c_int
    lib.fd_forward_persistent.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, vp, i32, vp, sz, vp]
    lib.fd_forward_persistent.restype = ctypes.c_int
    lib.fd_backward_workspace_size.argtypes = [vp, ctypes.POINTER(Batch), ctypes.c_int, ctypes.POINTER(sz)]
    lib.fd_backward_workspace_size.restype = ctypes.c_int
    lib.fd_backward.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                vp, sz, vp]
    lib.fd_backward.restype = ctypes.c_int
    lib.fd_euler_step.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    lib.fd_euler_step.restype = ctypes.c_int
    lib.fd_euler_step_backward.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    lib.fd_euler_step_backward.restype = ctypes.c_int
    lib.fd_inverse.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, ctypes.c_int, vp, vp]
    lib.fd_inverse.restype = ctypes.c_int
    lib.fd_joint_inertia.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp]
    lib.fd_joint_inertia.restype = ctypes.c_int
    lib.fd_scan6.argtypes = [ctypes.c_int, i32, vp, i32, vp, vp, ctypes.c_int, vp, vp]
    lib.fd_scan6.restype = ctypes.c_int
    lib.fd_btd_solve6.argtypes = [ctypes.c_int, i32, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.fd_btd_solve6.restype = ctypes.c_int
    lib.fd_set_auto_table.argtypes = [ctypes.c_int, vp]
    lib.fd_set_auto_table.restype = ctypes.c_int
    lib.fd_set_persistent_grid.argtypes = [ctypes.c_int, i32]
    lib.fd_set_persistent_grid.restype = ctypes.c_int
    lib.fd_auto_algo.argtypes = [vp, ctypes.POINTER(Batch), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.fd_auto_algo.restype = ctypes.c_int
    lib.fd_status_string.argtypes = [ctypes.c_int]
    lib.fd_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().fd_status_string(int(status)).decode()


def check(status: int, what: str) -> None:
    if status != FD_OK:
        raise FdError(status, what)
