"""The paper's own experiments (section "Main results", Figs. 2-3): fixed
energy on the momentum sphere, eps = 1, the density F of the direction of the
mean velocity V, zooms and the "remained within the area" selection.

Parity: initial positions bitwise, momenta to a few ulps (they take a cosine,
a sine and Hp), states to 1e-12 at T = 50 at E = 400, window decisions equal
except for orbits that pass within 1e-9 of an edge.  Physics: the qualitative
facts the paper states about Fig. 2 (parity with its figures is unpinned:
they are not printed)."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import H, assert_close, gpu, need_gpu, np_, print_case

pytestmark = gpu


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def _oracle_ic(e, idx=None):
    return oracle.ic_sphere(e.energy, e.eps, e.window[:2], e.window[2:], e.box_lo[:3], e.box_hi[:3], e.seed_ic,
                            n_orbits=None if idx is not None else e.n_orbits, idx=idx)


def test_sphere_initial_conditions(aw):
    print_case("sphere ic")
    from paper_1107_4107_amd import workloads as wl
    for e in (wl.sphere_ensemble(400.0, 20000), wl.sphere_ensemble(15.0, 20000, window=(0.3, 1.2, -0.4, 0.1))):
        ic, _ = aw.generate_ic(e)
        g = np_(ic)
        o = _oracle_ic(e)
        np.testing.assert_array_equal(g[:3], o[:3])
        # a cosine, a sine and Hp each within a few ulps: relative to |P|
        assert_close(g[3:], o[3:], 1e-15, floor=math.sqrt(2 * e.energy), what="P")
        Hs = [oracle.energy(g[:, n], 1.0) for n in range(0, 20000, 101)]
        np.testing.assert_allclose(Hs, e.energy, rtol=1e-14)


def test_states_at_E400(aw):
    """Weak regime of Fig. 2 (E = 400, |P| ~ 28): states after 50 steps."""
    print_case("E=400 states")
    from paper_1107_4107_amd import workloads as wl
    e = wl.sphere_ensemble(400.0, 4096, T=50, tangent=True)
    r = aw.map_ensemble(e, want_state=True)
    ic = _oracle_ic(e)                       # the oracle draws its own (ulp-level equal) states
    out_o, st_o = oracle.ensemble("s6", 1.0, H, 50, ic, oracle.w0(0, 4096), want_state=True)
    assert_close(np_(r.state)[:6], st_o[:6], 1e-12, what="state")
    assert_close(np_(r.orbit_out)[3:6], out_o[3:6], 1e-12, what="V")


def test_window_decisions(aw):
    """Fig. 3 zoom: orbits are kept only while the direction of P stays in the
    window; decisions must agree unless an orbit came within 1e-9 of an edge."""
    print_case("window flags")
    from paper_1107_4107_amd import workloads as wl
    e = wl.fig3_zoom(n_orbits=4096, T=1000)
    r = aw.map_ensemble(e)
    ic = _oracle_ic(e)
    _, left, margin = oracle.ensemble_window("s6", 1.0, H, 1000, ic, oracle.w0(0, 4096), e.window)
    g = (np_(r.cls) >> 1) & 1
    dis = g != left
    assert not (dis & (np.abs(margin) > 1e-9)).any(), (dis.sum(), margin[dis][:5])
    assert 0.05 < left.mean() < 0.95


def test_zoomed_direction_density(aw):
    """F on a zoom window, with and without the stay-in-window selection."""
    print_case("zoom density")
    from paper_1107_4107_amd import workloads as wl
    e = wl.fig3_zoom(n_orbits=50_000, T=300)
    spec = wl.sphere_image(128, 64, e.window)
    img, cnt, _ = aw.indicator_image(e, spec)
    c = np_(cnt).view(np.uint32)
    ic = _oracle_ic(e)
    out_o, left, margin = oracle.ensemble_window("s6", 1.0, H, 300, ic, oracle.w0(0, 50_000), e.window)
    keep = left == 0
    safe = np.abs(margin) > 1e-9
    assert c.sum() <= keep.sum() + (~safe).sum()
    phi, mu = oracle.vdir_keys(out_o[3:6][:, keep & safe])
    co, _, _ = oracle.hist2d(phi, mu, np.zeros(phi.size), (e.window[0], e.window[2]), (e.window[1], e.window[3]),
                             128, 64, closed_upper=True)
    diff = np.abs(c.astype(np.int64) - co.astype(np.int64))
    assert diff.sum() <= (~safe).sum() + 2 * 4, diff.sum()   # unsafe orbits and edge items only
    norm = 1.0 / (50_000 * ((e.window[1] - e.window[0]) / 128) * ((e.window[3] - e.window[2]) / 64))
    assert_close(np_(img), c * norm, 1e-14, floor=0.0)


def test_fig2_web_structure(aw):
    """Section "Main results", Fig. 2 (E = 400, eps_eff = 0.005, Delta t = 50 T):
    the uniform initial density stays uniform almost everywhere (regular
    motion keeps V near P(0)), and the primary resonances m = (1, -1, 0) and
    (1, 1, 0), i.e. Vx = Vy (phi = pi/4, -3 pi/4) and Vx = -Vy (phi = -pi/4,
    3 pi/4), show as bright lines with a dark zone beside them.  So do the
    other primary resonances of eq. 2's Fourier form, m = (1, +-1, +-2): on
    the sphere m . V = 0 is the circle mu = -s2 c / sqrt(4 + c^2) with
    c = cos phi + s1 sin phi, and the bins it crosses hold at least twice the
    median count (away from the (1, +-1, 0) lines and from mu = 0, where the
    circles meet)."""
    print_case("fig 2 structure")
    from paper_1107_4107_amd import workloads as wl
    N = 2_000_000
    e = wl.fig2(n_orbits=N)
    spec = wl.sphere_image(512, 256)
    img, cnt, _ = aw.indicator_image(e, spec)
    F = np_(img)
    c = np_(cnt).view(np.uint32)
    assert c.sum() == N
    uniform = 1.0 / (4 * math.pi)
    # density against phi, averaged over the mu rows |mu| < 0.7 (~2000 counts a column)
    mu_c = -1.0 + (np.arange(256) + 0.5) * 2.0 / 256
    prof = F[np.abs(mu_c) < 0.7].mean(axis=0)
    phi = -math.pi + (np.arange(512) + 0.5) * 2 * math.pi / 512
    med = np.median(prof)
    print(f"median density / uniform = {med / uniform:.4f}", flush=True)
    assert abs(med / uniform - 1.0) < 0.1
    for c0 in (math.pi / 4, -3 * math.pi / 4, -math.pi / 4, 3 * math.pi / 4):
        near = np.abs(phi - c0) < 0.02
        ring = (np.abs(phi - c0) > 0.03) & (np.abs(phi - c0) < 0.08)
        print(f"resonance phi={c0:+.3f}: line max / median = {prof[near].max() / med:.3f}, "
              f"side min / median = {prof[ring].min() / med:.3f}", flush=True)
        assert prof[near].max() > 1.3 * med
        assert prof[ring].min() < 0.9 * med
    cmed = np.median(c)
    far_from_lines = np.min([np.abs((phi - c0 + math.pi) % (2 * math.pi) - math.pi)
                             for c0 in (math.pi / 4, -3 * math.pi / 4, -math.pi / 4, 3 * math.pi / 4)], axis=0) > 0.15
    for s1 in (1, -1):
        for s2 in (1, -1):
            cc = np.cos(phi) + s1 * np.sin(phi)
            mu_r = -s2 * cc / np.sqrt(4 + cc * cc)
            cols = far_from_lines & (np.abs(mu_r) > 0.1)
            on = (np.abs(mu_c[:, None] - mu_r[None, :]) < 1.5 / 256) & cols[None, :]
            ratio = c[on].mean() / cmed
            print(f"resonance m=(1,{s1:+d},{2 * s2:+d}): mean count on the circle / median = {ratio:.3f}", flush=True)
            assert ratio > 2.0


def _cloud(aw, n, T):
    from paper_1107_4107_amd import workloads as wl
    return wl.fig4_cloud(n_orbits=n, T=T)


def _oracle_cloud(e):
    return oracle.ic_cloud(e.energy, e.eps, e.cloud, e.box_lo[:3], e.box_hi[:3], e.seed_ic, n_orbits=e.n_orbits)


def test_cloud_initial_conditions(aw):
    """Fig. 4's cloud at W: the rejection draw of X takes the same attempt on
    both sides (its test is far from 0 for all but a vanishing few orbits),
    the velocities agree to a few ulps and H = E."""
    print_case("cloud ic")
    e = _cloud(aw, 20000, 10)
    g = np_(aw.generate_ic(e)[0])
    o = _oracle_cloud(e)
    same_x = np.all(g[:3] == o[:3], axis=0)
    assert same_x.mean() >= 0.9999
    assert_close(g[3:5, same_x], o[3:5, same_x], 2e-15, floor=math.sqrt(2 * e.energy), what="vx, vy")
    # vz = sqrt(R) with R = 2 (E - Hp) - vx^2 - vy^2 a difference of terms ~ 2E:
    # R agrees to a few ulps of 2E, vz itself only to that divided by 2 sqrt(R).
    assert np.all(np.sign(g[5, same_x]) == np.sign(o[5, same_x]))
    assert_close(g[5, same_x] ** 2, o[5, same_x] ** 2, 1e-13, floor=1.0, what="vz^2")
    Hs = [oracle.energy(g[:, n], 1.0) for n in range(0, 20000, 97)]
    np.testing.assert_allclose(Hs, e.energy, rtol=1e-14)


def test_window_density_accumulates_over_windows(aw):
    """F averaged over consecutive windows (Fig. 4): the per-window direction
    counts of V added over 4 windows of 100 steps, against the oracle's window
    velocities binned the same way.  Both sides start from their own draws of
    the cloud (equal to ulps) in a chaotic region, so items within 1e-4 of a
    bin width from an edge may fall either side; splitting the windows over two
    calls changes nothing."""
    import torch
    print_case("window density")
    e = _cloud(aw, 4096, 400)
    w = math.pi / 4
    spec = aw.ImageSpec(kind="hist_vdir", W=64, H=64, lo=(w - 0.6, -0.6), hi=(w + 0.6, 0.6))
    N = e.n_orbits
    carry = torch.empty((aw.NCARRY, N), dtype=torch.float64, device="cuda")
    cnt = torch.zeros((64, 64), dtype=torch.int32, device="cuda")
    aw.window_density(e, carry, 0, 4, 100, spec, cnt)
    c1 = np_(cnt).view(np.uint32).copy()
    carry1 = np_(carry).copy()
    carry2 = torch.empty_like(carry)
    cnt2 = torch.zeros_like(cnt)
    aw.window_density(e, carry2, 0, 1, 100, spec, cnt2)
    aw.window_density(e, carry2, 100, 3, 100, spec, cnt2)
    np.testing.assert_array_equal(np_(cnt2).view(np.uint32), c1)
    np.testing.assert_array_equal(np_(carry2)[:20], carry1[:20])
    V = oracle.window_velocities("s6", 1.0, H, _oracle_cloud(e), 4, 100)
    co = np.zeros((64, 64), dtype=np.int64)
    amb = 0
    for k in range(4):
        phi, mu = oracle.vdir_keys(V[k])
        ck, _, _ = oracle.hist2d(phi, mu, np.zeros(N), (w - 0.6, -0.6), (w + 0.6, 0.6), 64, 64, closed_upper=True)
        co += ck
        fi = (phi - (w - 0.6)) / 1.2 * 64
        fj = (mu + 0.6) / 1.2 * 64
        amb += int(np.sum((np.abs(fi - np.round(fi)) < 1e-4) | (np.abs(fj - np.round(fj)) < 1e-4)))
    diff = np.abs(c1.astype(np.int64) - co)
    print(f"window counts: {c1.sum()} binned, |diff| sum {diff.sum()}, edge items {amb}", flush=True)
    assert c1.sum() > 0.5 * 4 * N
    assert diff.sum() <= 2 * amb + 4


def test_window_density_merges_crowded_tiles(aw):
    """The window density of 2e5 cloud orbits on a 64 x 64 zoom (four tiles):
    a window puts more items into a tile than one accumulation chunk holds, so
    its counts go through the chunk merge, and they are added to a buffer that
    already holds counts.  Against the oracle's window velocities binned the
    same way, with the edge-item allowance of the test above."""
    import torch
    print_case("window density, crowded tiles")
    e = _cloud(aw, 200_000, 200)
    w = math.pi / 4
    lo, hi = (w - 0.6, -0.6), (w + 0.6, 0.6)
    spec = aw.ImageSpec(kind="hist_vdir", W=64, H=64, lo=lo, hi=hi)
    N = e.n_orbits
    carry = torch.empty((aw.NCARRY, N), dtype=torch.float64, device="cuda")
    base = np.random.default_rng(5).integers(0, 1000, (64, 64)).astype(np.int32)
    cnt = torch.as_tensor(base).cuda()
    aw.window_density(e, carry, 0, 2, 100, spec, cnt)
    c1 = np_(cnt).astype(np.int64) - base
    V = oracle.window_velocities("s6", 1.0, H, _oracle_cloud(e), 2, 100)
    co = np.zeros((64, 64), dtype=np.int64)
    amb, crowded = 0, 0
    for k in range(2):
        phi, mu = oracle.vdir_keys(V[k])
        ck, _, _ = oracle.hist2d(phi, mu, np.zeros(N), lo, hi, 64, 64, closed_upper=True)
        co += ck
        crowded = max(crowded, int(ck.reshape(2, 32, 2, 32).sum(axis=(1, 3)).max()))
        fi = (phi - lo[0]) / 1.2 * 64
        fj = (mu - lo[1]) / 1.2 * 64
        amb += int(np.sum((np.abs(fi - np.round(fi)) < 1e-4) | (np.abs(fj - np.round(fj)) < 1e-4)))
    diff = np.abs(c1 - co)
    print(f"largest tile of a window {crowded} items; |diff| sum {diff.sum()}, edge items {amb}", flush=True)
    assert crowded > 16_384
    assert diff.sum() <= 2 * amb + 4
