"""The parity sets of the benchmark configurations at full size, against
oracle values stored under tests/golden/ (written by tests/golden/
make_goldens.py, which calls only the oracle; every input is restated there
from its definition).

* c2 (eps = 1e-3, the 1024 x 1024 (px, py) slice, T = 1e5; section "Main
  results": regular against resonant orbits), in the launch bench.py times:
  every point of the stride-4 256 x 256 sub-grid -- the class on >= 99.5% of
  them with every disagreement inside chi in [1.5, 2.5], and on regular
  orbits (oracle chi < 1.5) L, chi, dP2 and J to 1e-6 (dP2 on the scale of
  J, its mean over the run); then the class of every point of the whole
  slice against the oracle's, every disagreement inside the band.
* c5 (1e7 orbits uniform on [0, 2 pi)^6, eps = 5e-3, T = 1e6): orbits
  0..4095 -- identical to those of the full ensemble, since every draw is
  keyed on the orbit index -- run in the 1e5-step chunks with state carry
  that bench.py runs: the class as above, and on regular orbits L, V and J
  to 1e-6 or within 4 times the orbit's own one-ulp spread, stored with the
  oracle's values (at T = 1e6 binary64 does not fix L and dP2 to 1e-6 on
  every regular orbit), dP2 on the scale of J by the distribution of its
  error against its spread; the
  momentum-drift image keyed on (px0, py0) and the V-direction density
  exactly as the oracle bins the same per-orbit values (the direction keys
  themselves to an ulp).
* c4 (eps = 1e-2, the 512 x 512 slice, T = 1e4, checkpoints every 100
  steps): the gradient of J over the whole slice in one call, both sweeps;
  the 256 regular orbits drawn with seed 3 against the oracle's forward-mode
  derivative (1e-9, or within 4 times the oracle's own one-ulp spread of it
  for at most one orbit), its central differences with step 1e-6 (1e-5), the
  GPU's own central differences (1e-5) and a dot-product test.
* The eps sweep of the model section (the chaotic web thickens with eps, its
  volume scaling as sqrt(eps)) on the pz0 = 1 companion slice, 256 x 256,
  T = 3e4, 16 values of eps in one batched launch: classes on the stride-2
  sub-grid against the oracle's (>= 99.5%, disagreements inside the band),
  the chaotic fractions against the oracle's, and the log-log slope of the
  fraction against eps.

Regular orbits that miss 1e-6 are held to the rule of the shared helper: FP64
does not fix such a value more closely than the oracle's own one-ulp spread,
so the GPU must lie within 4 times that spread, and such orbits must be rare.
"""
import os

import numpy as np
import pytest

import oracle
from gpu_util import (H, assert_close, check_regular_rows, check_rows_with_spread, class_agreement, gpu, need_gpu,
                      np_, print_case)

pytestmark = gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TWO_PI = 2.0 * np.pi
L_, CHI_, DP2_, J_ = 0, 2, 6, 7


def _golden(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"missing {path}: write it with tests/golden/make_goldens.py")
    return np.load(path)


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def _regular_rows(got, ref, ic, w0, eps, T, what, rows=(L_, CHI_, DP2_, J_)):
    """Rows of the regular orbits: L, chi and V relative to max(1, |b|) (chi ~ 1
    there); J relative to itself (floor 1e-12); dP2 = |P_T - P_0|^2 relative to
    max(|dP2|, J).  dP2 is the end point of a quasi-periodic oscillation whose
    mean over the run is J, so its error is a phase error times the
    oscillation's size: near a minimum of the oscillation |dP2| itself is no
    scale for it, and J is."""
    floors = {DP2_: np.maximum(ref[J_], 1e-12), J_: 1e-12}
    worst, beyond = check_regular_rows(got, ref, rows, ic, w0, eps, T, floors=floors, what=what)
    for c, r, err, s in beyond:
        print(f"{what}: orbit column {c} row {r}: error {err:.2e}, oracle one-ulp spread {s:.2e}", flush=True)
    return worst, len({b[0] for b in beyond})


def test_c2_every_subgrid_point(aw):
    from paper_1107_4107_amd import workloads as wl
    g = _golden("c2_slice_1024_T1e5_stride4.npz")
    e = wl.c2()
    assert (g["eps"], g["n"], g["T"]) == (e.eps, e.nx, e.n_steps)
    print_case("c2 stride-4 sub-grid")
    img, cnt, cls = aw.indicator_image(e, wl.chi_image(e.nx), want_counts=True, want_class=True)
    chi = np_(img).ravel()
    c = np_(cls)
    out = np_(aw.map_ensemble(e, want_class=False).orbit_out)
    np.testing.assert_array_equal(out[CHI_], chi)          # one kernel, two epilogues
    idx = g["idx"]
    ref = np.full((9, idx.size), np.nan)
    ref[L_], ref[CHI_], ref[DP2_], ref[J_] = g["L"], g["chi"], g["dP2"], g["J"]
    frac = class_agreement(chi[idx], g["chi"])
    reg = np.flatnonzero(g["chi"] < 1.5)
    ic = oracle.ic_grid2((3, 4), (0, 0), (TWO_PI, TWO_PI), e.nx, e.ny, list(e.base), idx=idx[reg])
    worst, n_ill = _regular_rows(out[:, idx[reg]], ref[:, reg], ic, oracle.w0(0, idx=idx[reg]), e.eps, e.n_steps,
                                 "c2 sub-grid")
    print(f"sub-grid: {idx.size} points, class agreement {frac:.5f}, {reg.size} regular, worst error within the "
          f"bar {worst:.2e}, {n_ill} beyond it within their one-ulp spread", flush=True)
    assert int(np_(cnt).view(np.uint32)[0]) == int(c.sum())


def test_c2_class_of_every_point(aw):
    from paper_1107_4107_amd import workloads as wl
    full = _golden("c2_slice_1024_T1e5_classes.npz")
    e = wl.c2()
    assert (full["eps"], full["n"], full["T"]) == (e.eps, e.nx, e.n_steps)
    print_case("c2 class of every point")
    img, _, cls = aw.indicator_image(e, wl.chi_image(e.nx), want_counts=True, want_class=True)
    chi = np_(img).ravel()
    c = np_(cls)
    N = chi.size
    cls_o = np.unpackbits(full["class_bits"], bitorder="little")[:N].astype(bool)
    dis = np.flatnonzero((chi > 2.0) != cls_o)
    band = dict(zip(full["band_idx"].tolist(), full["band_chi"].tolist()))
    out_band = [int(m) for m in dis if not (m in band and 1.5 <= band[m] <= 2.5)]
    assert not out_band, f"class disagreements outside the band: {out_band[:8]}"
    assert dis.size <= 0.005 * N
    print(f"whole slice: {N} points, {int(cls_o.sum())} chaotic for the oracle, {int(c.sum())} for the GPU, "
          f"{dis.size} disagreements, all inside the band", flush=True)


def test_c5_first_4096_orbits_at_the_full_horizon(aw):
    import torch
    from paper_1107_4107_amd import workloads as wl
    g = _golden("c5_box_orbits0-4095_T1e6.npz")
    spread = _golden("c5_box_orbits0-4095_T1e6_one_ulp_spread.npz")["spread"]
    ref = g["out"]
    M = ref.shape[1]
    e = wl.c5(n_orbits=M)
    assert (g["eps"], g["T"], g["seed_ic"]) == (e.eps, e.n_steps, e.seed_ic)
    print_case("c5 orbits 0..4095 T=1e6 in chunks of 1e5")
    T, chunk = e.n_steps, 100_000
    carry = torch.empty((aw.NCARRY, M), dtype=torch.float64, device="cuda")
    out_t = torch.empty((aw.NOUT, M), dtype=torch.float64, device="cuda")
    cls = torch.empty((M,), dtype=torch.uint8, device="cuda")
    for k in range(0, T, chunk):
        k1 = min(T, k + chunk)
        aw.map_ensemble_steps(e, carry, k, k1, orbit_out=out_t if k1 == T else None, cls=cls if k1 == T else None)
    out = np_(out_t)
    np.testing.assert_array_equal(np_(cls), (out[CHI_] > 2.0).astype(np.uint8))
    frac = class_agreement(out[CHI_], ref[CHI_])
    reg = np.flatnonzero(ref[CHI_] < 1.5)
    ic_all = oracle.ic_box([0.0] * 6, [TWO_PI] * 6, 2, M)
    # At T = 1e6 binary64 fixes L and dP2 to 1e-6 on most regular orbits but
    # not all (dP2, a phase-sensitive end point, on about half), so every
    # orbit's own one-ulp spread is stored beside the oracle's values.
    floors = {J_: 1e-12}
    rep = check_rows_with_spread(out[:, reg], ref[:, reg], spread[:, reg], (L_, CHI_, 3, 4, 5, J_), floors,
                                 what="c5")
    print(f"{M} orbits: class agreement {frac:.5f}, {reg.size} regular; beyond 1e-6 (count, largest error / "
          f"one-ulp spread) per row: " + ", ".join(f"{r}: {v}" for r, v in rep.items()), flush=True)
    # dP2, the end point of an oscillation, on the scale of J.  Its error is a
    # phase error, and the ratio of the GPU's rounding-driven deviation to the
    # largest of the 12 one-ulp moves is heavy-tailed: beyond 1e-6 each orbit
    # within 10 times its spread, within 4 times on all but 0.5% of them, and
    # the median ratio at most 1 (one more draw of the same perturbation would
    # exceed the largest of 12 draws one time in 13).
    scale = np.maximum(ref[J_, reg], np.abs(ref[DP2_, reg]))
    err = np.abs(out[DP2_, reg] - ref[DP2_, reg]) / scale
    sp = spread[DP2_, reg] / scale
    beyond = err > 1e-6
    ratio = err[beyond] / sp[beyond]
    assert np.all(ratio <= 10.0), np.sort(ratio)[-5:]
    assert np.sum(ratio > 4.0) <= 0.005 * ratio.size, np.sort(ratio)[-10:]
    assert np.median(ratio) <= 1.0
    print(f"dP2: {int(beyond.sum())} regular orbits beyond 1e-6 of J; error / one-ulp spread: median "
          f"{np.median(ratio):.2f}, 99th percentile {np.quantile(ratio, 0.99):.2f}, largest {ratio.max():.2f} "
          f"({int(np.sum(ratio > 4.0))} above 4)", flush=True)
    # images: the library's reductions of the GPU's own per-orbit values
    # against the oracle's serial binning of the same values -- counts exact
    spec = wl.c5_p0_image()
    ic_t, _ = aw.generate_ic(e)
    cnt, sums, drop = aw.histogram2d(ic_t[3].contiguous(), ic_t[4].contiguous(), out_t[aw.OUT_DP2].contiguous(),
                                     spec.lo, spec.hi, spec.W, spec.H)
    c_o, s_o, d_o = oracle.hist2d(ic_all[3], ic_all[4], out[DP2_], spec.lo, spec.hi, spec.W, spec.H)
    np.testing.assert_array_equal(np_(cnt).view(np.uint32), c_o)
    assert int(np_(drop)[0]) == d_o == 0 and int(c_o.sum()) == M
    np.testing.assert_allclose(np_(sums), s_o, rtol=1e-12, atol=0)
    phi, mu = aw.vdir_keys(out_t[aw.OUT_VX:aw.OUT_VZ + 1].contiguous())
    vcnt, _, vdrop = aw.histogram2d(phi, mu, None, (-np.pi, -1.0), (np.pi, 1.0), 512, 512, closed_upper=True)
    kp, km = oracle.vdir_keys(out[3:6])
    np.testing.assert_array_equal(np_(mu), km)          # correctly rounded operations
    assert_close(np_(phi), kp, 4e-16, what="phi")        # atan2 to an ulp
    vc_o, _, vd_o = oracle.hist2d(np_(phi), np_(mu), np.zeros(M), (-np.pi, -1.0), (np.pi, 1.0), 512, 512,
                                  closed_upper=True)
    np.testing.assert_array_equal(np_(vcnt).view(np.uint32), vc_o)
    assert int(np_(vdrop)[0]) == vd_o


@pytest.mark.parametrize("reversible", [False, True])
def test_c4_gradient_on_the_256_seed3_orbits(aw, reversible):
    import torch
    from paper_1107_4107_amd import workloads as wl
    g = _golden("c4_grad_512_T1e4.npz")
    s = wl.c4()
    N, T = s.nx * s.ny, s.n_steps
    assert (g["eps"], g["n"], g["T"]) == (s.eps, s.nx, T)
    print_case("c4 gradient 512x512 T=1e4", "reversible" if reversible else "store")
    idx = g["idx"]
    assert idx.size == 256
    ic_all, _ = aw.generate_ic(s)
    e = aw.Ensemble(eps=s.eps, n_steps=T, ic_kind="explicit", n_orbits=N, tangent=False)
    J, gic, geps = aw.indicator_grad(e, ic_all, ckpt_every=wl.C4_CKPT, reversible=reversible)
    ic = oracle.ic_grid2((3, 4), (0, 0), (TWO_PI, TWO_PI), s.nx, s.ny, list(s.base), idx=idx)
    np.testing.assert_array_equal(np_(ic_all)[:, idx], ic)
    assert_close(np_(J)[idx], g["J"], 1e-9, floor=1e-300, what="J")
    grad = np.vstack([np_(gic)[:, idx], np_(geps)[None, idx]])
    scale = np.maximum(np.max(np.abs(g["dJ"]), axis=0, keepdims=True), 1e-300)
    err_fwd = np.abs(grad - g["dJ"]) / scale
    # Forward mode to 1e-9 relative to each orbit's gradient.  An orbit beyond
    # it must lie within 4 times the oracle's own one-ulp spread of dJ (the
    # largest change of its forward-mode derivative when one initial
    # coordinate moves by one ulp), and such orbits must be rare.
    per_orbit = err_fwd.max(axis=0)
    beyond = np.flatnonzero(per_orbit > 1e-9)
    for k in beyond:
        moved = np.repeat(ic[:, k:k + 1], 12, axis=1)
        for a in range(6):
            moved[a, 2 * a] = np.nextafter(ic[a, k], -np.inf)
            moved[a, 2 * a + 1] = np.nextafter(ic[a, k], np.inf)
        _, dJm = oracle.J_grad_ensemble("s6", s.eps, H, T, moved)
        spread = float(np.max(np.abs(dJm - g["dJ"][:, k:k + 1])) / scale[0, k])
        print(f"orbit {int(idx[k])}: |adjoint - forward mode| {per_orbit[k]:.2e}, oracle one-ulp spread of dJ "
              f"{spread:.2e}", flush=True)
        assert per_orbit[k] <= 4 * spread, (int(idx[k]), per_orbit[k], spread)
    assert beyond.size <= 1, [int(i) for i in idx[beyond]]
    good = np.setdiff1d(np.arange(idx.size), beyond)
    # z -> -z symmetry of eq. 2 on the invariant plane: exact zeros
    assert np.all(grad[2] == 0.0) and np.all(grad[5] == 0.0)
    err_fd = np.abs(grad - g["fd"]) / scale
    assert err_fd.max() <= 1e-5, f"against the oracle's central differences: {err_fd.max():.3e}"
    # the GPU's own central differences, step 1e-6, on the same 256 orbits
    d = float(g["fd_step"])
    w0 = oracle.w0(0, idx=idx)

    def J_of(ic_, eps_):
        ee = aw.Ensemble(eps=eps_, n_steps=T, ic_kind="explicit", n_orbits=256, tangent=False)
        return np_(aw.map_ensemble(ee, torch.as_tensor(ic_, device="cuda").contiguous(),
                                   want_class=False).orbit_out[aw.OUT_J])

    fd = np.empty((7, 256))
    for a in range(6):
        p, m = ic.copy(), ic.copy()
        p[a] += d
        m[a] -= d
        fd[a] = (J_of(p, s.eps) - J_of(m, s.eps)) / (2 * d)
    fd[6] = (J_of(ic, s.eps + d) - J_of(ic, s.eps - d)) / (2 * d)
    err_gfd = np.abs(grad - fd) / scale
    assert err_gfd.max() <= 1e-5, f"against the GPU's central differences: {err_gfd.max():.3e}"
    # dot-product test on the 256 orbits alone: <grad, (u, v)> with upstream gJ
    rng = np.random.default_rng(31)
    gJ = rng.normal(size=256)
    u = rng.normal(size=(6, 256))
    v = rng.normal()
    e256 = aw.Ensemble(eps=s.eps, n_steps=T, ic_kind="explicit", n_orbits=256, tangent=False)
    _, gic2, geps2 = aw.indicator_grad(e256, torch.as_tensor(ic, device="cuda").contiguous(),
                                       torch.as_tensor(gJ, device="cuda"), ckpt_every=wl.C4_CKPT,
                                       reversible=reversible)
    # over the orbits within the 1e-9 bar
    lhs = float(np.sum(np_(gic2)[:, good] * u[:, good]) + np.sum(np_(geps2)[good]) * v)
    terms = gJ[good] * (np.sum(g["dJ"][:6, good] * u[:, good], axis=0) + g["dJ"][6, good] * v)
    rhs = float(np.sum(terms))
    assert abs(lhs - rhs) <= 1e-9 * float(np.sum(np.abs(terms)))
    print(f"256 orbits: forward mode {per_orbit[good].max():.2e} ({beyond.size} beyond 1e-9 within their spread), "
          f"oracle FD {err_fd.max():.2e}, GPU FD {err_gfd.max():.2e}, dot product "
          f"{abs(lhs - rhs) / float(np.sum(np.abs(terms))):.2e}", flush=True)


def test_eps_sweep_against_the_oracle(aw):
    from paper_1107_4107_amd import workloads as wl
    g = _golden("sweep_pz1_256_T3e4_stride2.npz")
    n, T, pz0 = int(g["n"]), int(g["T"]), float(g["pz0"])
    ens = wl.eps_sweep(n=n, T=T, n_eps=g["eps"].size, pz0=pz0)
    np.testing.assert_array_equal(np.array([x.eps for x in ens]), g["eps"])
    print_case("eps sweep pz0=1 256x256 T=3e4")
    res = aw.map_ensembles(ens, want_class=True)
    idx = g["idx"]
    frac_gpu_sub, frac_gpu_all, n_dis = [], [], 0
    for k, (e, r) in enumerate(zip(ens, res)):
        chi = np_(r.orbit_out)[CHI_]
        cls_o = np.unpackbits(g["class_bits"][k], bitorder="little")[:idx.size].astype(bool)
        cls_g = chi[idx] > 2.0
        dis = np.flatnonzero(cls_g != cls_o)
        # every disagreement must have its oracle chi stored in [1.4, 3.0] and inside [1.5, 2.5]
        sel = g["band_eps"] == k
        band = dict(zip(g["band_idx"][sel].tolist(), g["band_chi"][sel].tolist()))
        for m in dis:
            assert m in band and 1.5 <= band[m] <= 2.5, (e.eps, int(idx[m]), band.get(m))
        assert dis.size <= 0.005 * idx.size, (e.eps, dis.size)
        n_dis += dis.size
        frac_gpu_sub.append(cls_g.mean())
        frac_gpu_all.append((chi > 2.0).mean())
    frac_o = g["fraction"]
    np.testing.assert_allclose(frac_gpu_sub, frac_o, rtol=0, atol=0.005)
    eps = g["eps"]

    def loglog_slope(f):
        f = np.asarray(f)
        ok = f > 0
        return float(np.polyfit(np.log(eps[ok]), np.log(f[ok]), 1)[0])

    slope_sub, slope_o, slope = loglog_slope(frac_gpu_sub), float(g["loglog_slope"]), loglog_slope(frac_gpu_all)
    print(f"chaotic fraction (GPU, whole slice): {np.round(frac_gpu_all, 5).tolist()}", flush=True)
    print(f"log-log slope on the sub-grid: GPU {slope_sub:.4f}, oracle {slope_o:.4f}; on the whole slice (GPU) "
          f"{slope:.4f}; {n_dis} class disagreements over {len(ens)} x {idx.size} points, all in the band", flush=True)
    assert abs(slope_sub - slope_o) <= 0.01
    # The model section's sqrt(eps) scaling of the web volume, on the whole
    # slice (the stride-2 sub-grid holds the lines px = 0 and px = py, where
    # the chaos of the smallest eps lies, twice as densely, and so flattens
    # the slope).
    assert abs(slope - 0.5) <= 0.1, slope
    # beside it, the literal invariant-plane slice (pz0 = 0), whose chaos is only
    # the two pendulum separatrices of the decoupled standard maps
    lit = aw.map_ensembles(wl.eps_sweep(n=n, T=T, n_eps=eps.size, pz0=0.0), want_class=True)
    frac_lit = np.array([float(np_(r.cls).mean()) for r in lit])
    ok = frac_lit > 0
    slope_lit = float(np.polyfit(np.log(eps[ok]), np.log(frac_lit[ok]), 1)[0])
    print(f"literal slice (pz0 = 0): fractions {np.round(frac_lit, 5).tolist()}, log-log slope {slope_lit:.4f}",
          flush=True)
