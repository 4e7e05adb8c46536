"""The default benchmark workload at full size, in the launch configuration
bench.py times: eps = 1e-3, the 1024 x 1024 (px, py) slice, T = 1e5, the chi
image, the class map and the chaotic count in one call.  96 sampled orbits --
half drawn at random, half among those the GPU classes chaotic -- are run by
the oracle at the full horizon: regular orbits' chi to 1e-6, every class
disagreement inside the band chi in [1.5, 2.5]."""
import numpy as np
import pytest

import oracle
from gpu_util import H, assert_close, gpu, need_gpu, np_, print_case

pytestmark = gpu


def test_default_workload_full_size():
    need_gpu()
    import paper_1107_4107_amd as aw
    from paper_1107_4107_amd import workloads as wl
    print_case("1024x1024 T=1e5")
    e = wl.c2()
    N = e.nx * e.ny
    img, cnt, cls = aw.indicator_image(e, wl.chi_image(e.nx), want_counts=True, want_class=True)
    chi = np_(img).ravel()
    c = np_(cls)
    np.testing.assert_array_equal(c, (chi > 2.0).astype(np.uint8))
    assert int(np_(cnt).view(np.uint32)[0]) == int(c.sum())
    rng = np.random.default_rng(11)
    chaotic = np.flatnonzero(c)
    idx = np.unique(np.concatenate([rng.choice(N, 48, replace=False),
                                    rng.choice(chaotic, min(48, chaotic.size), replace=False)]))
    ic = oracle.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), e.nx, e.ny, list(e.base), idx=idx)
    out_o = oracle.ensemble("s6", e.eps, H, e.n_steps, ic, oracle.w0(0, idx=idx))
    chi_o = out_o[2]
    reg = chi_o < 1.5
    assert_close(chi[idx][reg], chi_o[reg], 1e-6, what="chi (regular)")
    dis = (chi[idx] > 2.0) != (chi_o > 2.0)
    assert not (dis & ~((chi_o >= 1.5) & (chi_o <= 2.5))).any(), chi_o[dis]
    print(f"sampled {idx.size}: {reg.sum()} regular, {dis.sum()} class disagreements in band; "
          f"chaotic fraction {c.mean():.5f}", flush=True)
