"""Two lanes per orbit (tangent-free intermediate and time-window launches):
lane 2m holds u and p_u, lane 2m + 1 holds v and p_v in the rotated frame,
and every value is rounded as with one lane per orbit, so the carried states,
the window counts and the final outputs must be bitwise equal to the
one-lane kernel's.  The ensembles are chaotic (eps = 1 at E = 15, and
eps = 5e-2 on the torus), so any difference in rounding would grow into a
visible one; their sizes leave a ragged last block and a half-filled wave."""
import dataclasses

import numpy as np
import pytest

from gpu_util import gpu, need_gpu, np_, print_case

pytestmark = gpu


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def test_window_density_two_lanes_equals_one_lane(aw):
    import torch
    from paper_1107_4107_amd import workloads as wl
    print_case("window density, two lanes per orbit")
    e = wl.fig4_cloud(n_orbits=3001, T=1000)
    spec = aw.ImageSpec(kind="hist_vdir", W=96, H=64)
    res = {}
    for lpo in (1, 2, 0):
        t = aw.Tuning(lanes_per_orbit=lpo)
        carry = torch.full((aw.NCARRY, e.n_orbits), -1.0, dtype=torch.float64, device="cuda")
        cnt = torch.zeros((64, 96), dtype=torch.int32, device="cuda")
        aw.window_density(e, carry, 0, 3, 50, spec, cnt, tuning=t)       # from the initial conditions
        aw.window_density(e, carry, 150, 4, 50, spec, cnt, tuning=t)     # from the carry
        res[lpo] = (np_(cnt).copy(), np_(carry).copy())
    assert res[1][0].sum() > 0
    for lpo in (2, 0):
        np.testing.assert_array_equal(res[lpo][0], res[1][0], err_msg=f"counts, lanes per orbit {lpo}")
        np.testing.assert_array_equal(res[lpo][1], res[1][1], err_msg=f"carry, lanes per orbit {lpo}")


@pytest.mark.parametrize("form", ["s6", "stdmap", "y6"])
def test_chunked_run_two_lanes_equals_one_lane(aw, form):
    import torch
    from paper_1107_4107_amd import workloads as wl
    print_case("chunked run, two lanes per orbit", form)
    e = dataclasses.replace(wl.c5(n_orbits=1037, T=300), eps=5e-2, map_form=form, tangent=False)
    ref = aw.map_ensemble(e, want_state=True, want_class=False)
    outs = {}
    for lpo in (1, 2):
        t = aw.Tuning(lanes_per_orbit=lpo)
        carry = torch.full((aw.NCARRY, e.size), -1.0, dtype=torch.float64, device="cuda")
        out = torch.empty((aw.NOUT, e.size), dtype=torch.float64, device="cuda")
        st = torch.empty((12, e.size), dtype=torch.float64, device="cuda")
        aw.map_ensemble_steps(e, carry, 0, 100, tuning=t)
        c100 = np_(carry).copy()
        aw.map_ensemble_steps(e, carry, 100, 251, tuning=t)
        c251 = np_(carry).copy()
        aw.map_ensemble_steps(e, carry, 251, 300, orbit_out=out, state=st, tuning=t)
        outs[lpo] = (c100, c251, np_(out), np_(st))
    for a, b, what in zip(outs[2], outs[1], ("carry at 100", "carry at 251", "outputs", "state")):
        np.testing.assert_array_equal(a, b, err_msg=what)
    out2, st2 = outs[2][2], outs[2][3]
    np.testing.assert_array_equal(out2[3:], np_(ref.orbit_out)[3:])   # L, lambda, chi are NaN without tangent
    np.testing.assert_array_equal(st2[:6], np_(ref.state)[:6])
