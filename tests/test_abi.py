"""The C-ABI library loads, exports every entry point of include/fd.h and
rejects bad arguments before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_06779_amd import _lib, synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1609_06779_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert "fd_forward" in declared and "fd_init" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.fd_status_string(s)
    assert _lib.status_string(-5) == "workspace missing or too small"


def _desc(rb, keep):
    d = _lib.ModelDesc()
    dp = ctypes.POINTER(ctypes.c_double)
    arrs = {k: np.ascontiguousarray(getattr(rb, k), dtype=np.float64)
            for k in ("axis", "home_rot", "offset", "mass", "com", "inertia")}
    arrs["n"] = np.ascontiguousarray(rb.n_links, dtype=np.int32)
    keep.append(arrs)
    d.num_robots = len(rb.n_links)
    d.n_links = arrs["n"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    for k in ("axis", "home_rot", "offset", "mass", "com", "inertia"):
        setattr(d, k, arrs[k].ctypes.data_as(dp))
    for k in range(3):
        d.gravity[k] = rb.gravity[k]
    return d, arrs


@pytest.mark.parametrize("mutate", ["mass_zero", "mass_nan", "inertia_not_spd", "axis_zero",
                                    "rot_not_orthonormal", "n_zero", "n_too_long", "gravity_inf"])
def test_init_rejects_invalid_models(lib, mutate):
    rb = synth.make_robots([3, 2], seed=5)
    keep = []
    d, arrs = _desc(rb, keep)
    if mutate == "mass_zero":
        arrs["mass"][1] = 0.0
    elif mutate == "mass_nan":
        arrs["mass"][0] = np.nan
    elif mutate == "inertia_not_spd":
        arrs["inertia"][2] = [1.0, 1.0, 1.0, 2.0, 0.0, 0.0]
    elif mutate == "axis_zero":
        arrs["axis"][4] = 0.0
    elif mutate == "rot_not_orthonormal":
        arrs["home_rot"][0] = [2, 0, 0, 0, 1, 0, 0, 0, 1]
    elif mutate == "n_zero":
        arrs["n"][1] = 0
    elif mutate == "n_too_long":
        arrs["n"][0] = 100000
    elif mutate == "gravity_inf":
        d.gravity[2] = float("inf")
    out = ctypes.c_void_p()
    assert lib.fd_init(ctypes.byref(d), 0, ctypes.byref(out)) == _lib.FD_ERR_INVALID_ARG
    assert not out.value


@pytest.mark.parametrize("parents", [[0, 0, 1], [-1, 1, 0], [-1, 0, -2], [-1, 0, 3]])
def test_init_rejects_invalid_parents(lib, parents):
    """A parent must be an earlier link of the same robot, or the base (-1)."""
    rb = synth.make_robots([3, 2], seed=5)
    keep = []
    d, arrs = _desc(rb, keep)
    par = np.array(parents + [-1, 0], np.int32)
    keep.append(par)
    d.parent = par.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    out = ctypes.c_void_p()
    assert lib.fd_init(ctypes.byref(d), 0, ctypes.byref(out)) == _lib.FD_ERR_INVALID_ARG
    assert not out.value


def test_null_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.fd_init(None, 0, ctypes.byref(out)) == _lib.FD_ERR_INVALID_ARG
    b = _lib.Batch()
    b.batch = 4
    assert lib.fd_forward(None, ctypes.byref(b), None, None, None, None, 0, None, 0, None) == _lib.FD_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.fd_workspace_size(None, ctypes.byref(b), 0, ctypes.byref(n)) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_inverse(None, ctypes.byref(b), None, None, None, 1, None, None) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_scan6(0, -1, None, 8, None, None, 0, None, None) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_scan6(0, 0, None, 8, None, None, 0, None, None) == _lib.FD_OK
    assert lib.fd_scan6(7, 1, None, 8, None, None, 0, None, None) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_btd_solve6(0, 2, None, 8, None, None, None, None, None, None) == _lib.FD_ERR_INVALID_ARG
    fake = ctypes.c_void_p(8)   # never dereferenced: the length check fails first
    assert lib.fd_btd_solve6(0, 1, fake, 300, fake, fake, fake, fake, None, None) == _lib.FD_ERR_UNSUPPORTED
    assert lib.fd_max_links(None, 0) == 0


def test_binding_checks_array_sizes_before_any_launch():
    """The C ABI takes raw device pointers, so the binding checks what it can:
    robot_id and offsets entries for the batch, and per-link arrays of a
    uniform batch (batch * n entries). The checks run before the library is
    called, so they need no GPU."""
    torch = pytest.importorskip("torch")
    from paper_1609_06779_amd import fd

    class _Stub(fd.Model):
        def __init__(self, n_links):
            self.n_links = np.asarray(n_links, np.int32)
            self.device = torch.device("cuda:0")
            self._h = None

    m = _Stub([8, 8, 8])
    t = torch.empty(8 * 3)
    with pytest.raises(ValueError, match="robot_id"):
        m._batch(4, robot_id=torch.empty(3, dtype=torch.int32))
    with pytest.raises(ValueError, match="offsets"):
        m._batch(4, offsets=torch.empty(4, dtype=torch.int64))
    with pytest.raises(ValueError, match="q has 24 entries"):
        m._batch(4, state=(("q", t),))
    assert m._batch(3, state=(("q", t),)).batch == 3
    # robots of two lengths: the chain starts come from device offsets, so the
    # binding has no size to check and leaves the batch to the library
    assert _Stub([8, 5])._batch(2, state=(("q", torch.empty(1)),)).batch == 2


def test_choice_setters_check_their_arguments(lib):
    """The AUTO table and the default persistent grid are host-side settings:
    bad precisions, negative grids and table entries that name no algorithm
    (or AUTO itself) are refused; 0 and NULL restore the built-in choices."""
    assert lib.fd_set_persistent_grid(7, 0) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_set_persistent_grid(0, -1) == _lib.FD_ERR_INVALID_ARG
    assert lib.fd_set_persistent_grid(1, 512) == _lib.FD_OK
    assert lib.fd_set_persistent_grid(1, 0) == _lib.FD_OK
    table = np.zeros(257 * 21, np.int8)
    for bad in (_lib.ALGOS["auto"], 6, -1):
        table[300] = bad
        assert lib.fd_set_auto_table(0, table.ctypes.data_as(ctypes.c_void_p)) == _lib.FD_ERR_INVALID_ARG
    for good in (_lib.ALGOS["abia_scan"], _lib.ALGOS["cfa_proj"]):
        table[300] = good
        assert lib.fd_set_auto_table(0, table.ctypes.data_as(ctypes.c_void_p)) == _lib.FD_OK
    assert lib.fd_set_auto_table(0, None) == _lib.FD_OK
