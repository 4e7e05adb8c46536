"""The C-ABI library: it loads, exports every function include/aw.h declares,
its ctypes mirrors match the C struct layouts, and the host-side validation
rejects bad descriptors before touching a device.  CPU only."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1107_4107_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aw_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _abi.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.EXPORTS)


def test_probe_library_loads():
    """The probes (FP64 peak and clock for the benchmark; the device sine and
    cosine for the tests) are built beside libaw.so and check their arguments
    before touching a device."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1107_4107_amd", "libaw_probe.so"))
    assert hasattr(lib, "awp_fma_peak") and hasattr(lib, "awp_sincos")
    lib.awp_fma_peak.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    out = (ctypes.c_double * 5)()
    assert lib.awp_fma_peak(0, 1000, out) == 2      # argument check, no device touched
    assert lib.awp_fma_peak(1, 1000, None) == 2
    lib.awp_sincos.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_void_p]
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below returns before any launch
    assert lib.awp_sincos(fake, fake, fake, -1, 0, None) == 2
    assert lib.awp_sincos(fake, fake, fake, 10, 3, None) == 2
    assert lib.awp_sincos(fake, fake, fake, 10, -1, None) == 2
    assert lib.awp_sincos(None, fake, fake, 10, 0, None) == 2
    assert lib.awp_sincos(None, None, None, 0, 1, None) == 0


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "aw.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(aw_ensemble), sizeof(aw_tuning), sizeof(aw_image_spec));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(aw_ensemble, n_steps), offsetof(aw_ensemble, nx),
         offsetof(aw_ensemble, n_orbits), offsetof(aw_ensemble, chi_threshold), offsetof(aw_ensemble, flags));
  printf("%zu %zu\\n", offsetof(aw_image_spec, key_axis), offsetof(aw_image_spec, lo));
  printf("%zu %zu\\n", offsetof(aw_ensemble, energy), offsetof(aw_ensemble, window));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    E, T, S = _abi.AwEnsemble, _abi.AwTuning, _abi.AwImageSpec
    got = [ctypes.sizeof(E), ctypes.sizeof(T), ctypes.sizeof(S), E.n_steps.offset, E.nx.offset,
           E.n_orbits.offset, E.chi_threshold.offset, E.flags.offset, S.key_axis.offset, S.lo.offset,
           E.energy.offset, E.window.offset]
    assert [int(v) for v in out] == got


def _ens(**kw):
    from paper_1107_4107_amd import Ensemble
    return Ensemble(**{**dict(eps=1e-2, n_steps=10, nx=8, ny=8), **kw}).to_c()


@pytest.mark.parametrize("kw,status", [
    (dict(M=4), _abi.AW_EUNSUPPORTED),
    (dict(map_form=3), _abi.AW_EINVAL),
    (dict(n_steps=0), _abi.AW_EINVAL),
    (dict(h=0.0), _abi.AW_EINVAL),
    (dict(eps=float("nan")), _abi.AW_EINVAL),
    (dict(axis=(3, 3)), _abi.AW_EINVAL),
    (dict(axis=(3, 6)), _abi.AW_EINVAL),
    (dict(nx=0), _abi.AW_EINVAL),
    (dict(ic_kind="explicit", n_orbits=5), _abi.AW_EINVAL),  # no ic array
    (dict(chi_threshold=float("nan")), _abi.AW_EINVAL),
    (dict(ic_kind="sphere", n_orbits=4, energy=1.0, eps=1.0), _abi.AW_EINVAL),      # E <= 2|eps|
    (dict(ic_kind="sphere", n_orbits=4, energy=15.0, eps=1.0, window=(0.5, 0.2, -1, 1)), _abi.AW_EINVAL),
    (dict(ic_kind="sphere", n_orbits=4, energy=15.0, eps=1.0, window=(-4.0, 0.2, -1, 1)), _abi.AW_EINVAL),
    (dict(stay_in_window=True, window=(0, 1, -1.5, 1)), _abi.AW_EINVAL),
])
def test_host_validation_rejects_bad_descriptors(kw, status):
    lib = _abi.load()
    e = _ens(**kw)
    outs = _abi.ptr_array([None])
    st = lib.aw_map_ensemble(ctypes.byref(e), 1, None, outs, None, None, None, None)
    assert st == status
    assert lib.aw_last_error()


def test_bad_tuning_is_rejected():
    lib = _abi.load()
    e = _ens()
    for t in [(100, 1, 1, 8, 0), (256, 3, 1, 8, 0), (256, 1, 3, 8, 0), (256, 1, 1, 3, 0), (256, 1, 1, 32, 0),
              (256, 1, 1, 8, 0, 3), (256, 1, 1, 8, 0, -1)]:
        tun = _abi.AwTuning(*t)
        st = lib.aw_map_ensemble(ctypes.byref(e), 1, None, _abi.ptr_array([None]), None, None,
                                 ctypes.byref(tun), None)
        assert st == _abi.AW_EINVAL, t


def test_batched_ensembles_must_share_form():
    lib = _abi.load()
    arr = (_abi.AwEnsemble * 2)(_ens(), _ens(map_form="stdmap"))
    st = lib.aw_map_ensemble(arr, 2, None, _abi.ptr_array([None, None]), None, None, None, None)
    assert st == _abi.AW_EINVAL


def test_grad_workspace_size():
    lib = _abi.load()
    e = _ens(ic_kind="explicit", n_orbits=1000, n_steps=10_000)
    nb = ctypes.c_size_t()
    assert lib.aw_indicator_grad_workspace(ctypes.byref(e), 100, ctypes.byref(nb)) == 0
    # 100 checkpoints + the final state + the states kept in one segment (every
    # 4th step and the last: 25 for segments that start on a multiple of 4,
    # floor((100 + 2)/4) + 1 = 26 for any start), 6 doubles per orbit each.
    assert nb.value == 8 * 6 * 1000 * (100 + 1 + 26)
    assert lib.aw_indicator_grad_workspace(ctypes.byref(e), 0, ctypes.byref(nb)) == _abi.AW_EINVAL
    # one segment: ceil(T/4) kept states at most (+1 for a start off the multiples of 4)
    assert lib.aw_indicator_grad_workspace(ctypes.byref(e), 10_000, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 6 * 1000 * (1 + 1 + 2501)
    # the store-free sweep: checkpoints and the final state only
    assert lib.aw_indicator_grad_reversible_workspace(ctypes.byref(e), 100, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 6 * 1000 * (100 + 1)
    assert lib.aw_indicator_grad_reversible_workspace(ctypes.byref(e), 0, ctypes.byref(nb)) == _abi.AW_EINVAL


def test_kept_step_slots_cover_every_segment():
    """The slot of a kept step, (g >> 2) - (g0 >> 2), stays below the slot count
    the workspace query reserves, floor((ck + 2)/4) + 1, for every segment
    start and length, and distinct kept steps of a segment get distinct slots."""
    for ck in range(1, 40):
        bound = (ck + 2) // 4 + 1
        for g0 in range(0, 64):
            g1 = g0 + ck
            kept = [g for g in range(g0, g1) if (g + 1) % 4 == 0 or g == g1 - 1]
            slots = [(g >> 2) - (g0 >> 2) for g in kept]
            assert len(set(slots)) == len(slots) and min(slots) >= 0 and max(slots) < bound, (ck, g0)


def test_ftle_grad_workspace_and_validation():
    """Workspace of the FTLE gradient: 12 doubles (state and tangent) per orbit
    per checkpoint and per kept step of a segment (none for the store-free
    sweep), and the rescale exponents; bad calls are refused on the host
    before any device work."""
    lib = _abi.load()
    e = _ens(ic_kind="explicit", n_orbits=1000, n_steps=10_000)
    nb = ctypes.c_size_t()
    assert lib.aw_ftle_grad_reversible_workspace(ctypes.byref(e), 100, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 12 * 1000 * (100 + 1) + 2 * 1000 * (10_000 // 8)
    assert lib.aw_ftle_grad_workspace(ctypes.byref(e), 100, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 12 * 1000 * (100 + 1 + 26) + 2 * 1000 * (10_000 // 8)
    assert lib.aw_ftle_grad_workspace(ctypes.byref(e), 0, ctypes.byref(nb)) == _abi.AW_EINVAL
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    # not EXPLICIT
    g = _ens()
    assert lib.aw_ftle_grad(ctypes.byref(g), None, fake, None, 100, None, fake, fake, fake, 1 << 40, None,
                            None) == _abi.AW_EINVAL
    # no tangent start
    assert lib.aw_ftle_grad(ctypes.byref(e), fake, None, None, 100, None, fake, fake, fake, 1 << 40, None,
                            None) == _abi.AW_EINVAL
    # workspace too small
    assert lib.aw_ftle_grad(ctypes.byref(e), fake, fake, None, 100, None, fake, fake, fake, nb.value - 8, None,
                            None) == _abi.AW_EWORKSPACE
    # no gradient outputs
    assert lib.aw_ftle_grad(ctypes.byref(e), fake, fake, None, 100, None, None, fake, fake, 1 << 40, None,
                            None) == _abi.AW_EINVAL
    assert lib.aw_last_error()


def test_step_op_counts_match_the_stage_structure():
    """Per map step: 9 kicks and 10 drifts for the 6th-order triple jump, 7
    and 8 for Y6; the counts are those of the kernel's formulas in the rotated
    frame u = x + y, v = x - y.  A kick takes the sincos of u and v from the
    4096-entry table (8 fma, 4 mul, 1 add each) and cos^2 z, cos z sin z from
    the same table at the doubled angle (9 fma, 3 mul, 1 add); the rest of a
    kick is 3 fma, 2 mul and 1 add, plus 8 fma and 6 mul for the tangent; a
    drift 3 fma, 6 with the tangent; the J accumulator 3 fma, 3 subtractions
    and a doubling."""
    from paper_1107_4107_amd import step_op_counts
    sc_f, sc_m, sc_a = 8, 4, 1
    zt_f, zt_m, zt_a = 9, 3, 1
    kick_t = (2 * sc_f + zt_f + 3 + 8, 2 * sc_m + zt_m + 2 + 6, 2 * sc_a + zt_a + 1)
    kick_n = (2 * sc_f + zt_f + 3, 2 * sc_m + zt_m + 2, 2 * sc_a + zt_a + 1)
    f, m, a = step_op_counts("s6", True)
    assert (f, m, a) == (9 * kick_t[0] + 10 * 6 + 3, 9 * kick_t[1], 9 * kick_t[2] + 4)
    assert 2 * f + m + a == 985
    f, m, a = step_op_counts("y6", True)   # 7 kicks, 8 drifts
    assert (f, m, a) == (7 * kick_t[0] + 8 * 6 + 3, 7 * kick_t[1], 7 * kick_t[2] + 4)
    f1, m1, a1 = step_op_counts("stdmap", True)
    assert (f1, m1, a1) == (kick_t[0] + 6 + 3, kick_t[1], kick_t[2] + 4)
    f0, m0, a0 = step_op_counts("s6", False)
    assert (f0, m0, a0) == (9 * kick_n[0] + 10 * 3 + 3, 9 * kick_n[1], 9 * kick_n[2] + 4)


def test_y6_weights_agree_between_the_two_derivations():
    """The HIP library's weights of the 7-stage composition (generated offline
    with mpmath) and the oracle's (Newton's method in long double at load time)
    are derived independently from the order conditions; they must agree to
    a few ulps."""
    import numpy as np

    import oracle
    text = open(os.path.join(ROOT, "paper_1107_4107_amd", "csrc", "aw_y6_coef.h")).read()
    vals = re.search(r"AW_Y6_W\[4\] = \{([^}]*)\}", text).group(1).split(",")
    hip = np.array([float.fromhex(v.strip()) for v in vals])
    orc = oracle.y6_weights()
    np.testing.assert_allclose(hip, orc, rtol=4e-16, atol=0)


def test_ensemble_size():
    lib = _abi.load()
    assert lib.aw_ensemble_size(ctypes.byref(_ens(nx=7, ny=5))) == 35
    assert lib.aw_ensemble_size(ctypes.byref(_ens(ic_kind="box", n_orbits=123))) == 123
    assert lib.aw_ensemble_size(ctypes.byref(_ens(nx=0))) == -1


@pytest.mark.parametrize("gen,header", [("gen_sincos.py", "aw_sincos_coef.h"), ("gen_sincos_tab.py", "aw_sincos_tab.h")])
def test_generated_headers_are_current(gen, header):
    """The committed constant headers of the device sine/cosine are exactly
    what their generators write (the generators also replay the device
    arithmetic against mpmath and record the error in the header)."""
    csrc = os.path.join(ROOT, "paper_1107_4107_amd", "csrc")
    out = subprocess.run(["python3", os.path.join(csrc, gen)], capture_output=True, text=True, timeout=300,
                         cwd=csrc, check=True).stdout
    assert out == open(os.path.join(csrc, header)).read()


def test_table_sincos_error_bound():
    """The table-driven sine and cosine of the step loops, replayed by its
    generator with exactly rounded FMAs over arguments up to 1e6 and around
    the table's interval edges, stay within 1.2e-16 of the true values (half
    an ulp of 1 plus the rotation's rounding); the polynomial form of the
    initial conditions and the energy within 2.5e-16 on its reduced range."""
    import re
    csrc = os.path.join(ROOT, "paper_1107_4107_amd", "csrc")
    tab = open(os.path.join(csrc, "aw_sincos_tab.h")).read()
    m = re.search(r"max abs error sin ([0-9.e+-]+), cos ([0-9.e+-]+)", tab)
    assert m and float(m.group(1)) <= 1.2e-16 and float(m.group(2)) <= 1.2e-16
    m = re.search(r"max abs error cos\^2 z ([0-9.e+-]+), cos z sin z ([0-9.e+-]+)", tab)
    assert m and float(m.group(1)) <= 1.2e-16 and float(m.group(2)) <= 6e-17
    assert "#define AW_TAB_N 4096" in tab
    poly = open(os.path.join(csrc, "aw_sincos_coef.h")).read()
    errs = [float(x) for x in re.findall(r"double Horner max abs error ([0-9.e+-]+)", poly)]
    assert len(errs) == 2 and max(errs) <= 2.5e-16


def test_doubled_angle_z_terms_error_bound():
    """The kicks' z terms, cos^2 z and cos z sin z, from the table at the
    doubled angle (sincos_tab's reduction of z, node 2q, short polynomials for
    sin(2r)/2 and cos(2r)/2), replayed with exactly rounded FMAs, lie within
    1.2e-16 and 6e-17 of mpmath's values: over random arguments up to 1e5, the
    edges of the reduced interval (where q rounds either way), the nodes, far
    arguments and signed zeros.  Against libm's cos z * cos z and
    cos z * sin z they agree to 2.5e-16."""
    import importlib.util
    import random
    import mpmath as mp
    spec = importlib.util.spec_from_file_location(
        "gen_sincos_tab", os.path.join(ROOT, "paper_1107_4107_amd", "csrc", "gen_sincos_tab.py"))
    g = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(g)
    tab, _, _, inv, pa, pb, _, _ = g.constants()
    zs0, zc, errzs, errzc = g.z_constants()
    assert errzs < 1e-7 and errzc < 1e-14
    rnd = random.Random(21)
    edge = [float((k + 0.5) * mp.pi / 2048) for k in range(-5000, 5000, 37)]
    zs = [rnd.uniform(-10.0, 10.0) for _ in range(400)] + [rnd.uniform(-1e5, 1e5) for _ in range(300)]
    zs += edge + [math.nextafter(x, math.inf) for x in edge] + [math.nextafter(x, -math.inf) for x in edge]
    zs += [k * float(mp.pi) / 2048 for k in range(-60, 60)] + [0.0, -0.0, 1e-300, 1e12, -3e12]
    for z in zs:
        zsz, z2 = g.device_zterms(z, tab, zs0[0], zc, inv, pa, pb)
        cz, sz = mp.cos(mp.mpf(z)), mp.sin(mp.mpf(z))
        assert abs(z2 - float(cz * cz)) <= 1.2e-16, z
        assert abs(zsz - float(cz * sz)) <= 6e-17, z
        assert abs(z2 - math.cos(z) * math.cos(z)) <= 2.5e-16 and abs(zsz - math.cos(z) * math.sin(z)) <= 2.5e-16


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits non-zero
    before touching a device."""
    res = subprocess.run(["python3", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_image_workspace_query():
    """The library scratch of one image call, from the host alone: none for a
    single IC-grid ensemble or a single unbatched propagation; per-orbit
    histogram items plus sort buffers, growing with the ensemble; batch tables
    for several ensembles; invalid descriptors refused like the call itself."""
    from paper_1107_4107_amd import ImageSpec
    lib = _abi.load()
    nb = ctypes.c_size_t()

    def ws(ens, spec):
        arr = (_abi.AwEnsemble * len(ens))(*ens)
        st = lib.aw_image_workspace(arr, len(ens), ctypes.byref(spec.to_c()) if spec else None, ctypes.byref(nb))
        return st, nb.value

    assert ws([_ens()], ImageSpec(kind="ic_grid", W=8, H=8)) == (0, 0)
    assert ws([_ens()], None) == (0, 0)
    p0 = ImageSpec(kind="hist_p0", field=6, W=64, H=64)
    st, small = ws([_ens(ic_kind="box", n_orbits=1000)], p0)
    assert st == 0 and small >= 1000 * (4 + 8 + 2 + 8)
    st, big = ws([_ens(ic_kind="box", n_orbits=100_000)], p0)
    assert st == 0 and big >= 100_000 * (4 + 8 + 2 + 8) and big > small
    st, vdir = ws([_ens(ic_kind="box", n_orbits=100_000)], ImageSpec(kind="hist_vdir", W=64, H=64))
    assert st == 0 and 100_000 * (4 + 2) <= vdir < big          # no values to carry
    st, two = ws([_ens(), _ens(nx=16, ny=16)], None)
    assert st == 0 and two > 0                                  # descriptors and work items
    assert ws([_ens(M=4)], p0)[0] == _abi.AW_EUNSUPPORTED
    assert ws([_ens(ic_kind="box", n_orbits=10)], ImageSpec(kind="hist_p0", W=0, H=8))[0] == _abi.AW_EINVAL
    assert lib.aw_image_workspace(None, 1, None, ctypes.byref(nb)) == _abi.AW_EINVAL


def test_graph_create_refuses_bad_requests_on_the_host():
    """aw_graph_create validates everything before it allocates or captures:
    a bad descriptor, a missing spec, explicit initial conditions or a bad
    tuning return an error with no graph handed out."""
    lib = _abi.load()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    imgs = _abi.ptr_array([fake])
    spec = _abi.AwImageSpec(0, _abi.OUT_CHI, 8, 8, (3, 4), (0.0, 0.0), (1.0, 1.0))
    cases = [
        ((_abi.AwEnsemble * 1)(_ens(M=4)), ctypes.byref(spec), None, _abi.AW_EUNSUPPORTED),
        ((_abi.AwEnsemble * 1)(_ens()), None, None, _abi.AW_EINVAL),
        ((_abi.AwEnsemble * 1)(_ens(ic_kind="explicit", n_orbits=64)), ctypes.byref(spec), None, _abi.AW_EINVAL),
        ((_abi.AwEnsemble * 1)(_ens()), ctypes.byref(spec), ctypes.byref(_abi.AwTuning(100, 1, 1, 8, 0, 0)),
         _abi.AW_EINVAL),
    ]
    for ens, sp, tun, status in cases:
        out = ctypes.c_void_p(0x1234)
        st = lib.aw_graph_create(ens, 1, sp, imgs, None, None, tun, ctypes.byref(out))
        assert st == status, (st, status)
        assert out.value is None
        assert lib.aw_last_error()


def test_accumulation_chunks_fit_the_scratch(tmp_path):
    """The histogram accumulation's chunk size and the scratch bound it is
    sized by (aw_hist.hpp), compiled for the host: the chunk is a multiple
    of 4096 of at least 16384 items; ceil(N / chunk) never exceeds
    acc_bound(N, T), which never decreases with N (scratch sized for the
    largest ensemble of a call serves the smaller ones); and for tile
    populations from uniform to a single crowded tile, the chunks (one at
    least per tile) and the partial tiles of tiles of several chunks fit
    T + ceil(N / chunk) and 2 ceil(N / chunk)."""
    src = tmp_path / "chunks.cpp"
    src.write_text(r"""
#include <cstdio>
#include <cstdint>
#include <vector>
#include "aw_hist.hpp"
using namespace aw;
static int64_t nch(int64_t c, int64_t ch) { return c == 0 ? 1 : (c + ch - 1) / ch; }
int main() {
  const int64_t Ts[] = {1, 2, 6, 8, 64, 192, 256, 1024, 4096, 8192};
  uint64_t s = 12345;
  auto rnd = [&]() { s = s * 6364136223846793005ull + 1442695040888963407ull; return s >> 11; };
  for (int64_t T : Ts) {
    int64_t prev = -1;
    for (int64_t N = 0; N < (int64_t(1) << 31); N = N < 100000 ? N + 997 : N + N / 7 + 1) {
      const int64_t ch = acc_chunk(N, T), b = acc_bound(N > 0 ? N : 1, T), k = (N + ch - 1) / ch;
      if (ch < ACC_CHUNK_MIN || ch % ACC_ROUND) { printf("chunk %lld T %lld N %lld\n", (long long)ch, (long long)T, (long long)N); return 1; }
      if (k > b) { printf("bound T %lld N %lld: %lld > %lld\n", (long long)T, (long long)N, (long long)k, (long long)b); return 1; }
      if (b < prev) { printf("bound decreases at T %lld N %lld\n", (long long)T, (long long)N); return 1; }
      prev = b;
      if (T > 1024 && N > 50000000) continue;
      for (int shape = 0; shape < 3; ++shape) {   // uniform, one crowded tile, random shares
        std::vector<int64_t> c(T, 0);
        if (shape == 0) for (int64_t t = 0; t < T; ++t) c[t] = N / T + (t < N % T ? 1 : 0);
        else if (shape == 1) c[rnd() % T] = N;
        else { int64_t left = N; for (int64_t t = 0; t + 1 < T && left > 0; ++t) { int64_t x = (int64_t)(rnd() % (uint64_t)(left + 1)); c[t] = x; left -= x; } c[T - 1] += left; }
        int64_t chunks = 0, parts = 0;
        for (int64_t t = 0; t < T; ++t) { const int64_t q = nch(c[t], ch); chunks += q; if (q > 1) parts += q; }
        if (chunks > T + k || parts > 2 * k || parts > 2 * b) { printf("fit T %lld N %lld shape %d\n", (long long)T, (long long)N, shape); return 1; }
        if (shape == 0 && N > 0 && 2 * ((N + T - 1) / T) <= (N + 255) / 256 && parts != 0) { printf("uniform split T %lld N %lld\n", (long long)T, (long long)N); return 1; }
      }
    }
  }
  printf("ok\n");
  return 0;
}
""")
    exe = tmp_path / "chunks"
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    csrc = os.path.join(ROOT, "paper_1107_4107_amd", "csrc")
    subprocess.run([hipcc, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", csrc, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
