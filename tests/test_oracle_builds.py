"""Builds of the CPU oracle other than the default one.

* The host-tuned build (-O3 -march=native, contraction still off) computes
  bitwise what the portable build computes: the CPU-baseline timing uses it.
* The whole pin suite passes under AddressSanitizer and
  UndefinedBehaviorSanitizer (the oracle's memory accesses and integer
  arithmetic are clean), run in a child process that preloads the ASan
  runtime.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
H = 0.01 * 2.0 * np.pi


def _results(lib):
    """A fixed set of oracle results from one loaded build."""
    import ctypes
    dp = ctypes.POINTER(ctypes.c_double)
    rng = np.random.default_rng(4)
    N, T = 24, 400
    ic = np.ascontiguousarray(np.vstack([rng.uniform(0, 2 * np.pi, (3, N)), rng.uniform(-2, 2, (3, N))]))
    w = np.ascontiguousarray(rng.standard_normal((6, N)))
    res = []
    for form, eps in ((6, 1e-2), (6, 1.0), (1, 0.3), (7, 0.1)):
        out = np.empty((9, N))
        st = np.empty((12, N))
        assert lib.oracle_ensemble(form, eps, H, T, N, ic.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                   out.ctypes.data_as(dp), st.ctypes.data_as(dp), 2) == 0
        res += [out, st]
    J = np.empty(N)
    dJ = np.empty((7, N))
    assert lib.oracle_J_grad_ensemble(6, 1e-2, H, 200, N, ic.ctypes.data_as(dp), J.ctypes.data_as(dp),
                                      dJ.ctypes.data_as(dp), 2) == 0
    L = np.empty(N)
    dL = np.empty((7, N))
    assert lib.oracle_ftle_grad_ensemble(6, 1e-2, H, 200, N, ic.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                         L.ctypes.data_as(dp), dL.ctypes.data_as(dp), 2) == 0
    return res + [J, dJ, L, dL]


def test_native_build_is_bitwise_equal(tmp_path):
    path = oracle.build(force=True, variant="native", out=str(tmp_path / "liboracle_native.so"))
    a = _results(oracle._load())
    b = _results(oracle.open_library(path))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.view(np.uint64), y.view(np.uint64))


def _preloads_in_place():
    return bool(os.environ.get("LD_PRELOAD")) or os.path.exists("/etc/ld.so.preload")


@pytest.mark.skipif(_preloads_in_place(), reason="another library is preloaded into every process here")
def test_pins_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    path = oracle.build(force=True, variant="sanitize", out=str(tmp_path / "liboracle_asan.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("the ASan runtime is not installed")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    env[oracle.LIB_ENV] = path
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")], env=env, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
