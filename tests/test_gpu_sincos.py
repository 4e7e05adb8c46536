"""The device's own sine and cosine, evaluated directly on the GPU.

The probe library runs the kernels' two sine/cosine routines on given
arguments.  The table-driven routine of the step loops must reproduce, bit for
bit, its replay by the table generator (every fused multiply-add rounded once,
the table offset taken from the same bits), and lie within 1.2e-16 of mpmath's
values; the polynomial routine of the initial conditions within 3e-16; the
kicks' z terms (cos z sin z, cos^2 z from the table at the doubled angle)
bit for bit their replay and within 6e-17 and 1.2e-16 of mpmath.  Both
are also held against numpy's libm over a large set of arguments: random ones
up to 1e6 (and near the magic-number rounding's limit), points at and beside
the midpoints between table nodes, where the rounding of q decides the node,
the nodes themselves, tiny and signed zeros; non-finite arguments give NaN."""
import ctypes
import importlib.util
import os

import numpy as np
import pytest

from gpu_util import gpu, need_gpu, print_case

pytestmark = gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1107_4107_amd", "csrc")


@pytest.fixture(scope="module")
def probe():
    need_gpu()
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1107_4107_amd", "libaw_probe.so"))
    lib.awp_sincos.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_void_p]
    lib.awp_sincos.restype = ctypes.c_int
    return lib


def _device(lib, x, form):
    import torch
    xd = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    s = torch.empty_like(xd)
    c = torch.empty_like(xd)
    torch.cuda.synchronize()
    assert lib.awp_sincos(xd.data_ptr(), s.data_ptr(), c.data_ptr(), xd.numel(), form, None) == 0
    torch.cuda.synchronize()
    return s.cpu().numpy(), c.cpu().numpy()


def _arguments(limit):
    rng = np.random.default_rng(11)
    k = np.arange(-6000, 6000)
    mid = (k + 0.5) * (np.pi / 2048)
    parts = [rng.uniform(-7.0, 7.0, 100_000), rng.uniform(-limit, limit, 100_000), rng.uniform(-1e-3, 1e-3, 10_000),
             mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf), k * (np.pi / 2048),
             np.array([0.0, -0.0, 5e-324, -5e-324, 1e-300, np.pi, -np.pi, 2 * np.pi, 1e5 * np.pi])]
    return np.concatenate(parts)


def _gen():
    spec = importlib.util.spec_from_file_location("gen_sincos_tab", os.path.join(CSRC, "gen_sincos_tab.py"))
    g = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(g)
    return g


def test_table_sincos_matches_its_model_and_mpmath(probe):
    print_case("table sincos")
    import mpmath as mp
    x = np.concatenate([_arguments(1e6), np.array([1e12, -1e12, 3.4e12])])
    s, c = _device(probe, x, 0)
    # numpy's libm over every argument (its own error is below an ulp of 1)
    assert np.max(np.abs(s - np.sin(x))) <= 2.5e-16
    assert np.max(np.abs(c - np.cos(x))) <= 2.5e-16
    # bitwise against the generator's replay, and within 1.2e-16 of mpmath, on a sample
    g = _gen()
    tab, ps, pc, inv, pa, pb, _, _ = g.constants()
    rng = np.random.default_rng(12)
    pick = np.concatenate([rng.choice(x.size, 1500, replace=False), np.arange(x.size - 12, x.size)])
    for i in pick:
        ms, mc = g.device_sincos(float(x[i]), tab, ps[0], pc, inv, pa, pb)
        assert s[i] == ms and c[i] == mc, (x[i], s[i], ms, c[i], mc)
        assert abs(s[i] - float(mp.sin(mp.mpf(float(x[i]))))) <= 1.2e-16
        assert abs(c[i] - float(mp.cos(mp.mpf(float(x[i]))))) <= 1.2e-16


def test_doubled_angle_z_terms_match_their_model_and_mpmath(probe):
    """The kicks' cos z sin z and cos^2 z (probe form 2) from the table at the
    doubled angle."""
    print_case("z terms")
    import mpmath as mp
    x = np.concatenate([_arguments(1e6), np.array([1e12, -1e12, 3.4e12])])
    zsz, z2 = _device(probe, x, 2)
    assert np.max(np.abs(zsz - np.cos(x) * np.sin(x))) <= 2.5e-16
    assert np.max(np.abs(z2 - np.cos(x) * np.cos(x))) <= 2.5e-16
    g = _gen()
    tab, _, _, inv, pa, pb, _, _ = g.constants()
    zs0, zc, _, _ = g.z_constants()
    rng = np.random.default_rng(14)
    pick = np.concatenate([rng.choice(x.size, 1500, replace=False), np.arange(x.size - 12, x.size)])
    for i in pick:
        ms, mc = g.device_zterms(float(x[i]), tab, zs0[0], zc, inv, pa, pb)
        assert zsz[i] == ms and z2[i] == mc, (x[i], zsz[i], ms, z2[i], mc)
        c, s_ = mp.cos(mp.mpf(float(x[i]))), mp.sin(mp.mpf(float(x[i])))
        assert abs(zsz[i] - float(c * s_)) <= 6e-17
        assert abs(z2[i] - float(c * c)) <= 1.2e-16


def test_polynomial_sincos_within_its_range(probe):
    print_case("polynomial sincos")
    import mpmath as mp
    x = _arguments(3e6)
    s, c = _device(probe, x, 1)
    assert np.max(np.abs(s - np.sin(x))) <= 4e-16
    assert np.max(np.abs(c - np.cos(x))) <= 4e-16
    rng = np.random.default_rng(13)
    for i in rng.choice(x.size, 1500, replace=False):
        assert abs(s[i] - float(mp.sin(mp.mpf(float(x[i]))))) <= 3e-16
        assert abs(c[i] - float(mp.cos(mp.mpf(float(x[i]))))) <= 3e-16


@pytest.mark.parametrize("form", [0, 1, 2])
def test_sincos_of_non_finite_arguments_is_nan(probe, form):
    print_case("sincos non-finite", form)
    s, c = _device(probe, np.array([np.inf, -np.inf, np.nan, 1.0]), form)
    assert np.all(np.isnan(s[:3])) and np.all(np.isnan(c[:3]))
    if form == 2:
        assert s[3] == pytest.approx(np.sin(1.0) * np.cos(1.0), abs=3e-16)
        assert c[3] == pytest.approx(np.cos(1.0) ** 2, abs=3e-16)
    else:
        assert s[3] == pytest.approx(np.sin(1.0), abs=3e-16) and c[3] == pytest.approx(np.cos(1.0), abs=3e-16)
