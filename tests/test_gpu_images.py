"""GPU parity of the image reductions (section "Main results": the indicator
image over a slice of initial conditions, the momentum-drift image keyed on
the initial momenta, and the density F of the direction of V on the sphere).

Counts are integers decided by floating-point bin edges; both sides compute
the bin with the same IEEE operations on bitwise-equal keys where the keys
are initial conditions, so those counts must be bitwise equal.  Keys that
come out of the propagation (V) agree only to ~1e-12, so an item within
1e-9 of a bin edge may fall on either side: per bin the count difference must
be covered by such ambiguous items."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import H, assert_close, gpu, need_gpu, np_, print_case

pytestmark = gpu
TWO_PI = 2 * math.pi


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def tensor(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("N,W,H_", [(300_001, 512, 512), (54_321, 37, 23), (1, 64, 32), (0, 8, 8),
                                    (3_000_001, 1024, 512), (20_000, 4096, 2048)])
def test_histogram2d_matches_oracle(aw, N, W, H_):
    """Counts bitwise and sums to 1e-12 against the oracle.  The cases span
    one and several 32 x 32 tiles, ragged images, no items, per-tile rows of
    more than one scan chunk (3e6 items: 367 count blocks) and the largest
    image (4096 x 2048: 8192 tiles)."""
    print_case("hist2d", N, W, H_)
    rng = np.random.default_rng(N + W)
    a = rng.uniform(-0.3, 6.6, N)
    b = rng.uniform(-0.2, 6.5, N)
    v = rng.normal(size=N)
    if N > 10:
        a[:3] = [0.0, TWO_PI, np.nan]        # left edge kept, right edge dropped, NaN dropped
        b[:3] = [1.0, 1.0, 1.0]
    c, s, d = aw.histogram2d(tensor(a), tensor(b), tensor(v), (0, 0), (TWO_PI, TWO_PI), W, H_)
    co, so, do = oracle.hist2d(a, b, v, (0, 0), (TWO_PI, TWO_PI), W, H_)
    np.testing.assert_array_equal(np_(c).view(np.uint32), co)
    assert int(np_(d)[0]) == do
    # The order of the additions inside a bin is the device's (LDS atomics),
    # so a sum is fixed only up to rounding relative to the sum of the
    # magnitudes of its terms, which is the bound applied.
    _, sabs, _ = oracle.hist2d(a, b, np.abs(v), (0, 0), (TWO_PI, TWO_PI), W, H_)
    err = np.abs(np_(s) - so)
    bad = ~(err <= 1e-12 * np.maximum(sabs, 1e-300))
    assert not bad.any(), f"sums: {bad.sum()} bins beyond 1e-12 of their sum of |v|; worst {err[bad].max()}"


def _crowded_keys(rng, N, W, H_, tiles):
    """Keys with 90% of the items spread over the given 32 x 32-bin tiles
    (equal shares) and the rest uniform over the image and a little beyond."""
    a = rng.uniform(-0.3, 6.6, N)
    b = rng.uniform(-0.2, 6.5, N)
    crowd = np.nonzero(rng.random(N) < 0.9)[0]
    which = rng.integers(0, len(tiles), crowd.size)
    wa, wb = TWO_PI / W, TWO_PI / H_
    for k, (tx, ty) in enumerate(tiles):
        m = crowd[which == k]
        a[m] = (tx * 32 + rng.uniform(0, min(32, W - tx * 32), m.size)) * wa
        b[m] = (ty * 32 + rng.uniform(0, min(32, H_ - ty * 32), m.size)) * wb
    return a, b


@pytest.mark.parametrize("N,W,H_,tiles", [(2_000_003, 512, 512, [(5, 3)]),
                                          (40_000, 64, 64, [(0, 0), (1, 1)]),
                                          (16_384, 32, 32, [(0, 0)]), (16_385, 32, 32, [(0, 0)]),
                                          (1_000_000, 1024, 512, [(0, 0), (31, 15), (7, 9), (8, 9), (20, 2)])])
def test_histogram2d_crowded_tiles_match_oracle(aw, N, W, H_, tiles):
    """Items crowding into a few tiles: the accumulation splits each tile's
    range into chunks of at least 16384 items, one workgroup each, and adds
    the partial tiles of a tile in chunk order.  One tile of 1.8e6 items
    (about 110 chunks), two of about 2e4 (two chunks each), one tile of
    exactly one chunk and of one chunk plus an item, five crowded tiles of
    a large image.  Counts bitwise, sums within 1e-12 of their sum of |v|."""
    print_case("hist2d crowded", N, W, H_, len(tiles))
    rng = np.random.default_rng(N + 7 * W)
    a, b = _crowded_keys(rng, N, W, H_, tiles)
    if N == 16_384 or N == 16_385:   # every item in the single tile
        a = rng.uniform(0.0, TWO_PI, N)
        b = rng.uniform(0.0, TWO_PI, N)
        a[a >= TWO_PI] = 0.0
        b[b >= TWO_PI] = 0.0
    v = rng.normal(size=N)
    c, s, d = aw.histogram2d(tensor(a), tensor(b), tensor(v), (0, 0), (TWO_PI, TWO_PI), W, H_)
    co, so, do = oracle.hist2d(a, b, v, (0, 0), (TWO_PI, TWO_PI), W, H_)
    per_tile = np.add.reduceat(np.add.reduceat(co.astype(np.int64), np.arange(0, H_, 32), axis=0),
                               np.arange(0, W, 32), axis=1)
    print(f"largest tile {per_tile.max()} items", flush=True)
    if N > 16_384:
        assert per_tile.max() > 16_384                # the case has a tile of several chunks
    np.testing.assert_array_equal(np_(c).view(np.uint32), co)
    assert int(np_(d)[0]) == do
    _, sabs, _ = oracle.hist2d(a, b, np.abs(v), (0, 0), (TWO_PI, TWO_PI), W, H_)
    err = np.abs(np_(s) - so)
    bad = ~(err <= 1e-12 * np.maximum(sabs, 1e-300))
    assert not bad.any(), f"sums: {bad.sum()} bins beyond 1e-12 of their sum of |v|; worst {err[bad].max()}"
    c2, s2, d2 = aw.histogram2d(tensor(a), tensor(b), None, (0, 0), (TWO_PI, TWO_PI), W, H_)
    assert s2 is None
    np.testing.assert_array_equal(np_(c2).view(np.uint32), co)
    assert int(np_(d2)[0]) == do


def test_histogram2d_without_values_and_closed_edges(aw):
    print_case("hist2d closed")
    a = np.array([-np.pi, np.pi, 0.0, np.pi, 3.0])
    b = np.array([-1.0, 1.0, 0.0, -1.0, np.nextafter(1.0, 2.0)])   # the last is above the range
    c, s, d = aw.histogram2d(tensor(a), tensor(b), None, (-np.pi, -1.0), (np.pi, 1.0), 16, 8, closed_upper=True)
    co, _, do = oracle.hist2d(a, b, np.zeros(5), (-np.pi, -1.0), (np.pi, 1.0), 16, 8, closed_upper=True)
    assert s is None
    np.testing.assert_array_equal(np_(c).view(np.uint32), co)
    assert int(np_(d)[0]) == do
    assert co[7, 15] == 1 and co[0, 15] == 1 and do == 1   # phi = pi lands in the last column


def test_vdir_keys(aw):
    print_case("vdir keys")
    rng = np.random.default_rng(7)
    V = rng.normal(size=(3, 10000))
    V[:, 0] = 0.0
    V[:, 1] = [-1.0, 0.0, 0.0]  # phi = pi
    phi, mu = aw.vdir_keys(tensor(V))
    po, mo = oracle.vdir_keys(V)
    np.testing.assert_array_equal(np_(mu), mo)   # same correctly rounded operations
    p = np_(phi)
    assert np.isnan(p[0]) and np.isnan(po[0])
    assert_close(p[1:], po[1:], 4e-16, what="phi")


def test_ic_grid_image_is_the_orbit_row(aw):
    print_case("ic grid image")
    e = aw.Ensemble(eps=1e-2, n_steps=1000, nx=64, ny=64)
    for field in (aw.OUT_CHI, aw.OUT_DP2):
        img, cnt, cls = aw.indicator_image(e, aw.ImageSpec(kind="ic_grid", field=field, W=64, H=64),
                                           want_counts=True, want_class=True)
        ref = aw.map_ensemble(e)
        np.testing.assert_array_equal(np_(img).ravel(), np_(ref.orbit_out)[field])
        np.testing.assert_array_equal(np_(cls), np_(ref.cls))
        assert int(np_(cnt).view(np.uint32)[0]) == int(np_(ref.cls).sum())


def _box(aw, N, T):
    from paper_1107_4107_amd import workloads
    return workloads.c5(n_orbits=N, T=T)


def test_momentum_drift_image(aw):
    """HIST_P0: counts depend only on the initial momenta (bitwise equal on both
    sides); per-bin means of |P_T - P_0|^2 to 1e-9 at T = 50."""
    print_case("hist p0")
    from paper_1107_4107_amd import workloads
    N, T = 200_003, 50
    e = _box(aw, N, T)
    spec = workloads.c5_p0_image()
    img, cnt, _ = aw.indicator_image(e, spec)
    ic = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, N)
    out = oracle.ensemble("s6", e.eps, H, T, ic, oracle.w0(e.seed_tangent, N), nthreads=0)
    mean_o, cnt_o, drop_o = oracle.hist_p0(ic, out[6], (3, 4), (0, 0), (TWO_PI, TWO_PI), 512, 512)
    np.testing.assert_array_equal(np_(cnt).view(np.uint32), cnt_o)
    assert drop_o == 0
    assert_close(np_(img), mean_o, 1e-9, floor=1e-12, what="mean dP2")


def test_momentum_drift_image_crowded(aw):
    """HIST_P0 with the initial momenta in a narrow box, so that a few tiles
    hold every item and the mean image goes through the chunk merge: counts
    bitwise, per-bin means of |P_T - P_0|^2 to 1e-9 at T = 50."""
    import dataclasses
    print_case("hist p0 crowded")
    from paper_1107_4107_amd import workloads
    N, T = 200_003, 50
    e = _box(aw, N, T)
    lo, hi = list(e.box_lo), list(e.box_hi)
    lo[3], hi[3], lo[4], hi[4] = 1.0, 1.2, 2.0, 2.2
    e = dataclasses.replace(e, box_lo=lo, box_hi=hi)
    spec = workloads.c5_p0_image()
    img, cnt, _ = aw.indicator_image(e, spec)
    ic = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, N)
    out = oracle.ensemble("s6", e.eps, H, T, ic, oracle.w0(e.seed_tangent, N), nthreads=0)
    mean_o, cnt_o, drop_o = oracle.hist_p0(ic, out[6], (3, 4), (0, 0), (TWO_PI, TWO_PI), 512, 512)
    per_tile = np.add.reduceat(np.add.reduceat(cnt_o.astype(np.int64), np.arange(0, 512, 32), axis=0),
                               np.arange(0, 512, 32), axis=1)
    assert per_tile.max() > 2 * 16_384
    np.testing.assert_array_equal(np_(cnt).view(np.uint32), cnt_o)
    assert drop_o == 0
    assert_close(np_(img), mean_o, 1e-9, floor=1e-12, what="mean dP2")


def _ambiguous_ok(cnt, cnt_o, phi, mu, W, Hh, tol=1e-9):
    """Count differences must be explained by items within tol of a bin edge."""
    diff = cnt.astype(np.int64) - cnt_o.astype(np.int64)
    if not diff.any():
        return 0
    fi = (phi + np.pi) / (2 * np.pi) * W
    fj = (mu + 1.0) / 2.0 * Hh
    amb = (np.abs(fi - np.round(fi)) < tol * W) | (np.abs(fj - np.round(fj)) < tol * Hh)
    slack = np.zeros_like(diff)
    ii = np.clip(np.floor(fi[amb]).astype(int), 0, W - 1)
    jj = np.clip(np.floor(fj[amb]).astype(int), 0, Hh - 1)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            np.add.at(slack, (np.clip(jj + dj, 0, Hh - 1), np.clip(ii + di, 0, W - 1)), 1)
    assert np.all(np.abs(diff) <= slack), "count differences not explained by edge items"
    return int(np.abs(diff).sum())


def test_direction_density_image(aw):
    """HIST_VDIR: the density F of V/|V| on the sphere, in equal-area bins."""
    print_case("hist vdir")
    from paper_1107_4107_amd import workloads
    N, T = 200_003, 50
    e = _box(aw, N, T)
    spec = workloads.c5_vdir_image()
    img, cnt, _ = aw.indicator_image(e, spec)
    ic = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, N)
    out = oracle.ensemble("s6", e.eps, H, T, ic, oracle.w0(e.seed_tangent, N))
    dens_o, cnt_o, drop_o = oracle.hist_vdir(out[3:6], 512, 512)
    c = np_(cnt).view(np.uint32)
    assert c.sum() == N - drop_o
    phi, mu = oracle.vdir_keys(out[3:6])
    _ambiguous_ok(c, cnt_o, phi, mu, 512, 512)
    norm = 1.0 / (N * (2 * np.pi / 512) * (2.0 / 512))
    assert_close(np_(img), c * norm, 1e-14, floor=0.0, what="density")


def test_large_ensemble_histogram_full_size(aw):
    """The 1e7-orbit ensemble (uniform on [0, 2 pi)^6, eps = 5e-3) through the
    full image path at a reduced horizon: counts bitwise against the oracle's
    histogram of the initial momenta, sum of count*mean equal to the sum of the
    per-orbit drifts, and 64 sampled orbits against the oracle."""
    print_case("hist p0 1e7")
    from paper_1107_4107_amd import workloads
    N, T = 10_000_000, 200
    e = _box(aw, N, T)
    spec = workloads.c5_p0_image()
    img, cnt, _ = aw.indicator_image(e, spec)
    c = np_(cnt).view(np.uint32)
    ic_p = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, N)
    cnt_o, _, drop_o = oracle.hist2d(ic_p[3], ic_p[4], np.zeros(N), (0, 0), (TWO_PI, TWO_PI), 512, 512)
    np.testing.assert_array_equal(c, cnt_o)
    del ic_p
    r = aw.map_ensemble(e, want_class=False)
    dp2 = np_(r.orbit_out[6])
    assert abs(float(np.sum(np_(img) * c)) - float(np.sum(dp2))) <= 1e-10 * float(np.sum(dp2))
    idx = np.sort(np.random.default_rng(2).choice(N, 64, replace=False))
    ic = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, idx=idx)
    out_o = oracle.ensemble("s6", e.eps, H, T, ic, oracle.w0(e.seed_tangent, idx=idx))
    out = np_(r.orbit_out)[:, idx]
    reg = out_o[2] < 1.5
    assert_close(out[0, reg], out_o[0, reg], 1e-6, what="L")
    assert_close(out[6, reg], out_o[6, reg], 1e-6, floor=1e-9, what="dP2")
