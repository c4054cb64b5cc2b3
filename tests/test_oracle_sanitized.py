"""The oracle's C code under the address and undefined-behaviour sanitizers:
the library is rebuilt with -fsanitize=address,undefined into a temporary
directory and exercised (forward dynamics in double and long double, inverse
dynamics, M, the complex-step JVPs, chains and trees, ragged batches) in a
child process that preloads the sanitizer runtime; any report makes the child
fail. Host code only: nothing here touches a GPU."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r'''
import ctypes, sys
import numpy as np
sys.path.insert(0, {root!r})
import oracle
oracle._LIB = {lib!r}
from paper_1609_06779_amd import synth
rng = np.random.default_rng(3)
for lengths, tree in (([1, 2, 7, 16, 33], False), ([5, 9, 12], True)):
    if tree:
        rb = synth.make_tree_robots(lengths, seed=4, random_home=True)
    else:
        rb = synth.make_robots(lengths, seed=4, random_home=True)
    q, qd, tau = synth.make_state(lengths, seed=4)
    a = oracle.fd(rb, q, qd, tau)
    b = oracle.fd_exact(rb, q, qd, tau)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    oracle.rnea(rb, q, qd, a)
    oracle.crba(rb, q)
    oracle.fd_jvp(rb, q, qd, tau, rng.standard_normal(q.shape), rng.standard_normal(q.shape),
                  rng.standard_normal(q.shape))
print("ok")
'''


def _sanitizer_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_ub_sanitizers():
    asan = _sanitizer_runtime()
    if asan is None:
        pytest.skip("no address-sanitizer runtime for gcc")
    srcs = [os.path.join(os.path.dirname(oracle.__file__), f) for f in
            ("fd_oracle.c", "fd_oracle_cx.c", "fd_oracle_ld.c")]
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                        "-std=c11", "-o", lib, *srcs, "-lm"], check=True)
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env,
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0 and "ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
