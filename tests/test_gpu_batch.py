"""Batched persistent launches and HIP graphs.

One persistent launch over many ensembles (different eps, grid sizes and
horizons) must give per-orbit results bitwise equal to separate launches; a
captured graph replayed several times, with other GPU work between replays,
must reproduce the eager result every time; the 64-ensemble batch of the
eps sweep is checked against the oracle on sampled orbits."""
import numpy as np
import pytest

import oracle
from gpu_util import H, assert_close, class_agreement, gpu, need_gpu, np_, print_case

pytestmark = gpu


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def _mixed(aw):
    from paper_1107_4107_amd import workloads as wl
    spec = [(1e-4, 33, 700), (3e-3, 64, 300), (1e-2, 128, 1000), (5e-2, 17, 50), (1e-1, 96, 411), (2e-2, 1, 9)]
    return [wl.slice_ensemble(e, n, T) for e, n, T in spec]


@pytest.mark.parametrize("tun", [None, (64, 1, 1, 8, 7), (128, 2, 1, 4, 0), (512, 1, 1, 8, 0)])
def test_batched_equals_separate(aw, tun):
    print_case("batched vs separate", tun)
    ens = _mixed(aw)
    t = aw.Tuning(block=tun[0], orbits_per_lane=tun[1], unroll=tun[2], renorm_every=tun[3],
                  persistent_wgs=tun[4]) if tun else None
    batch = aw.map_ensembles(ens, want_state=True, tuning=t)
    for e, b in zip(ens, batch):
        s = aw.map_ensemble(e, want_state=True)
        np.testing.assert_array_equal(np_(b.orbit_out), np_(s.orbit_out))
        np.testing.assert_array_equal(np_(b.state), np_(s.state))
        np.testing.assert_array_equal(np_(b.cls), np_(s.cls))


def test_batched_equals_separate_y6(aw):
    """The same for the 7-stage 6th-order composition (its own stage pattern)."""
    import dataclasses
    print_case("batched vs separate y6")
    ens = [dataclasses.replace(e, map_form="y6") for e in _mixed(aw)]
    batch = aw.map_ensembles(ens, want_state=True)
    for e, b in zip(ens, batch):
        s = aw.map_ensemble(e, want_state=True)
        np.testing.assert_array_equal(np_(b.orbit_out), np_(s.orbit_out))
        np.testing.assert_array_equal(np_(b.state), np_(s.state))


def test_graph_replays_match_eager(aw):
    import torch
    print_case("graph replays")
    ens = _mixed(aw)[:5]
    # One image spec per graph, so the batch shares one grid size; eps and T differ.
    same = [aw.Ensemble(eps=e.eps, n_steps=e.n_steps, nx=48, ny=40, base=e.base) for e in ens]
    sp = aw.ImageSpec(kind="ic_grid", field=aw.OUT_CHI, W=48, H=40)
    eager = [aw.indicator_image(e, sp) for e in same]
    imgs = [torch.full((40, 48), -1.0, dtype=torch.float64, device="cuda") for _ in same]
    cnts = [torch.full((1,), 12345, dtype=torch.int32, device="cuda") for _ in same]
    g = aw.Graph(same, sp, imgs, cnts)
    for rep in range(3):
        for im in imgs:
            im.fill_(-1.0)
        g.launch()
        torch.cuda.synchronize()
        for k in range(len(same)):
            np.testing.assert_array_equal(np_(imgs[k]), np_(eager[k][0]))
            assert int(np_(cnts[k]).view(np.uint32)[0]) == int(np_(eager[k][1]).view(np.uint32)[0])
        # unrelated eager work between replays
        aw.map_ensemble(ens[rep])
        x = torch.randn(1000, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    g.close()


def test_eps_sweep_batch_against_oracle(aw):
    """The 64-ensemble eps sweep (eps_k = 10^(-4+3k/63), grids 128^2..1024^2,
    T in {1e4, 3e4, 1e5}) at 1/100 of its horizons in one persistent launch;
    12 orbits of every ensemble against the oracle."""
    print_case("eps sweep T/100")
    from paper_1107_4107_amd import workloads as wl
    ens = wl.c3(t_scale=0.01)
    res = aw.map_ensembles(ens, want_class=True)
    rng = np.random.default_rng(5)
    chi_g, chi_o = [], []
    for e, r in zip(ens, res):
        N = e.nx * e.ny
        idx = np.sort(rng.choice(N, 12, replace=False))
        ic = oracle.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), e.nx, e.ny, list(e.base), idx=idx)
        out_o = oracle.ensemble("s6", e.eps, H, e.n_steps, ic, oracle.w0(0, idx=idx))
        out = np_(r.orbit_out)[:, idx]
        reg = out_o[2] < 1.5
        assert_close(out[0, reg], out_o[0, reg], 1e-6, what=f"L eps={e.eps:.2e}")
        chi_g.append(out[2])
        chi_o.append(out_o[2])
    class_agreement(np.concatenate(chi_g), np.concatenate(chi_o), min_frac=0.99)


def test_graph_over_mixed_grids(aw):
    """W = H = 0: every ensemble images on its own grid inside one graph."""
    import torch
    print_case("graph mixed grids")
    ens = _mixed(aw)
    spec = aw.ImageSpec(kind="ic_grid", field=aw.OUT_DP2, W=0, H=0)
    imgs = [torch.empty((e.ny, e.nx), dtype=torch.float64, device="cuda") for e in ens]
    cnts = [torch.empty((1,), dtype=torch.int32, device="cuda") for e in ens]
    g = aw.Graph(ens, spec, imgs, cnts)
    eager_imgs, eager_cnts, _ = aw.indicator_images(ens, spec)
    for _ in range(2):
        g.launch()
        torch.cuda.synchronize()
        for a, b, c, d in zip(imgs, eager_imgs, cnts, eager_cnts):
            np.testing.assert_array_equal(np_(a), np_(b))
            np.testing.assert_array_equal(np_(c), np_(d))
    g.close()


def test_web_thickens_with_eps(aw):
    """Model section: with growing perturbation the Arnold web becomes
    thicker.  The chaotic fraction (chi > 2) of the p_z0 = 1 slice, from one
    batched launch over 8 eps values, must not decrease with eps beyond
    sampling noise, and must grow overall."""
    print_case("web thickens")
    from paper_1107_4107_amd import workloads as wl
    ens = wl.eps_sweep(n=128, T=10_000, n_eps=8, pz0=1.0)
    spec = aw.ImageSpec(kind="ic_grid", field=aw.OUT_CHI, W=0, H=0)
    _, cnts, _ = aw.indicator_images(ens, spec)
    frac = np.array([int(np_(c).view(np.uint32)[0]) for c in cnts]) / (128 * 128)
    print("chaotic fractions", frac, flush=True)
    noise = 3 * np.sqrt(np.maximum(frac, 1.0 / 16384) / 16384)
    assert np.all(np.diff(frac) >= -noise[1:]), frac
    assert frac[-1] > frac[0] + 0.01
