"""The host library on the GPU: graphs of histogram images, library scratch
per stream, reserved scratch, and batch-table staging under a backlog.

* A graph of HIST_P0 / HIST_VDIR images (propagation, sort and accumulation)
  replays the eager result several times, with unrelated GPU work and host
  synchronisation between the replays.
* Image calls on two streams at once (each stream has its own scratch) give
  the results of the same calls run one after the other.
* After aw_reserve() of the queried workspace the calls give the same results.
* Many batched calls queued without synchronising (the pinned staging of
  their tables is reused only once its copies are done) give the result of one.
Counts are compared bit for bit; per-bin means, whose float sums depend on
the order of LDS atomics, within 1e-12 relative (every value is >= 0)."""
import numpy as np
import pytest

from gpu_util import gpu, need_gpu, np_, print_case

pytestmark = gpu


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def _boxes(aw, sizes, T):
    from paper_1107_4107_amd import workloads as wl
    out = []
    for k, N in enumerate(sizes):
        e = wl.c5(n_orbits=N, T=T)
        e.eps = 5e-3 * (1 + k)
        out.append(e)
    return out


def _same_image(a, b, what):
    a, b = np_(a), np_(b)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0, err_msg=what)


@pytest.mark.parametrize("kind", ["hist_p0", "hist_vdir"])
@pytest.mark.parametrize("n_ens", [1, 3])
def test_graph_of_histogram_images_replays_eager(aw, kind, n_ens):
    import torch
    print_case("graph hist", kind, n_ens)
    ens = _boxes(aw, [20_011, 4_099, 65_536][:n_ens], 40)
    spec = aw.ImageSpec(kind=kind, field=aw.OUT_DP2, W=96, H=80)
    eager_i, eager_c, _ = aw.indicator_images(ens, spec)
    torch.cuda.synchronize()
    imgs = [torch.full((80, 96), -1.0, dtype=torch.float64, device="cuda") for _ in ens]
    cnts = [torch.full((80, 96), -7, dtype=torch.int32, device="cuda") for _ in ens]
    g = aw.Graph(ens, spec, imgs, cnts)
    for rep in range(3):
        for im, c in zip(imgs, cnts):
            im.fill_(-1.0)
            c.fill_(-7)
        g.launch()
        torch.cuda.synchronize()
        for k in range(n_ens):
            np.testing.assert_array_equal(np_(cnts[k]), np_(eager_c[k]))
            _same_image(imgs[k], eager_i[k], f"replay {rep} ensemble {k}")
        # unrelated eager work, including other image calls on the same stream
        aw.indicator_images(_boxes(aw, [3000], 10), spec)
        x = torch.randn(4096, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    g.close()


def test_two_streams_at_once(aw):
    import torch
    print_case("two streams")
    spec = aw.ImageSpec(kind="hist_p0", field=aw.OUT_DP2, W=128, H=128)
    a = _boxes(aw, [150_001, 70_000], 200)
    b = _boxes(aw, [90_007], 300)
    ref_a = aw.indicator_images(a, spec)
    ref_b = aw.indicator_images(b, spec)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(2):
        with torch.cuda.stream(s1):
            got_a = aw.indicator_images(a, spec)
        with torch.cuda.stream(s2):
            got_b = aw.indicator_images(b, spec)
        torch.cuda.synchronize()
        for got, ref in ((got_a, ref_a), (got_b, ref_b)):
            for k in range(len(got[0])):
                np.testing.assert_array_equal(np_(got[1][k]), np_(ref[1][k]))
                _same_image(got[0][k], ref[0][k], "two streams")


def test_reserved_scratch(aw):
    import torch
    print_case("reserve")
    ens = _boxes(aw, [50_000, 30_000], 60)
    spec = aw.ImageSpec(kind="hist_vdir", W=64, H=64)
    nb = aw.image_workspace_bytes(ens, spec)
    # one u32 bin per orbit of every ensemble, one u16 sorted slot per item of the larger one
    assert nb >= 4 * 80_000 + 2 * 50_000
    ref = aw.indicator_images(ens, spec)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        aw.reserve(nb)
        got = aw.indicator_images(ens, spec)
    torch.cuda.synchronize()
    for k in range(len(ens)):
        np.testing.assert_array_equal(np_(got[1][k]), np_(ref[1][k]))
        np.testing.assert_array_equal(np_(got[0][k]), np_(ref[0][k]))   # density = count x norm


def test_batched_calls_queued_without_waiting(aw):
    import torch
    print_case("staging backlog")
    from paper_1107_4107_amd import workloads as wl
    ens = [wl.slice_ensemble(e, n, T) for e, n, T in [(1e-3, 64, 3000), (2e-2, 33, 2000), (5e-2, 48, 2500)]]
    ref = aw.map_ensembles(ens)
    torch.cuda.synchronize()
    outs = [aw.map_ensembles(ens) for _ in range(12)]   # queued back to back
    torch.cuda.synchronize()
    for res in outs:
        for r, q in zip(res, ref):
            np.testing.assert_array_equal(np_(r.orbit_out), np_(q.orbit_out))
