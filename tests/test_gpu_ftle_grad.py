"""GPU parity of the second-order adjoint: the gradient of the tangent growth
L = ln(|w_T| / |w_0|) (the FTLE before its division by T h) with respect to
the initial state and eps.

References: the oracle's forward-over-forward derivatives (pinned against
finite differences and mpmath third derivatives), central differences of the
GPU's own forward L, and the autograd wrapper.  Bars: on regular orbits
(oracle chi < 1.5) the seven derivatives to 1e-8 of the orbit's largest
derivative and L to 1e-9 at T = 1000 (a relative change of 1e-15 in the
initial state alone moves the oracle's derivatives by up to 1.6e-10 there;
measured: 6.6e-10 and 1.9e-11);
results bitwise independent of the checkpoint interval."""
import numpy as np
import pytest

import oracle
from gpu_util import H, gpu, need_gpu, np_, print_case

pytestmark = gpu


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def _slice_ic(n, pz0, idx):
    return oracle.ic_grid2((3, 4), (0.0, 0.0), (2 * np.pi, 2 * np.pi), n, n, [0.0, 0.0, 0.0, 0.0, 0.0, pz0], idx=idx)


def _explicit(aw, eps, T, N, form="s6"):
    return aw.Ensemble(eps=eps, n_steps=T, map_form=form, ic_kind="explicit", n_orbits=N, tangent=True)


def _per_orbit_close(g, o, rel, what):
    """|g - o| <= rel * max_c |o_c| for every orbit (columns = orbits)."""
    scale = np.maximum(np.max(np.abs(o), axis=0), 1e-300)
    err = np.max(np.abs(g - o), axis=0) / scale
    print(f"{what}: max rel err {err.max():.3e}, median {np.median(err):.3e}", flush=True)
    assert np.all(err <= rel), (what, np.sort(err)[-5:])


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("pz0", [0.0, 1.0])
def test_ftle_gradient_matches_oracle(aw, pz0):
    """256 orbits of the eps = 1e-2 slice (and its pz0 = 1 companion), T = 1000,
    checkpoints every 100 steps."""
    print_case("ftle grad vs oracle", pz0)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(128 * 128, 256, replace=False))
    ic = _slice_ic(128, pz0, idx)
    w0 = oracle.w0(0, idx=idx)
    T, eps = 1000, 1e-2
    Lo, dLo = oracle.ftle_grad_ensemble("s6", eps, H, T, ic, w0)
    e = _explicit(aw, eps, T, 256)
    L, gic, geps = aw.ftle_grad(e, _to_dev(ic), _to_dev(w0), ckpt_every=100)
    g = np.vstack([np_(gic), np_(geps)[None]])
    chi = Lo / np.log(1 + T * H)
    reg = chi < 1.5
    assert reg.sum() > 100
    print(f"L: max abs err {np.max(np.abs(np_(L)[reg] - Lo[reg])):.3e}", flush=True)
    assert np.max(np.abs(np_(L)[reg] - Lo[reg])) < 1e-9
    _per_orbit_close(g[:, reg], dLo[:, reg], 1e-8, "dL (regular)")


@pytest.mark.parametrize("form", ["stdmap", "s2", "s4", "y6"])
def test_ftle_gradient_other_forms(aw, form):
    print_case("ftle grad form", form)
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 9, 64)
    w0 = oracle.w0(4, 64)
    T, eps = 200, 2e-2
    Lo, dLo = oracle.ftle_grad_ensemble(form, eps, H, T, ic, w0)
    L, gic, geps = aw.ftle_grad(_explicit(aw, eps, T, 64, form), _to_dev(ic), _to_dev(w0), ckpt_every=30)
    g = np.vstack([np_(gic), np_(geps)[None]])
    assert np.max(np.abs(np_(L) - Lo)) < 1e-10
    reg = Lo / np.log(1 + T * H) < 1.5
    assert reg.sum() > 16
    _per_orbit_close(g[:, reg], dLo[:, reg], 1e-8, f"dL {form}")


def test_ftle_gradient_against_gpu_differences(aw):
    """Central differences (step 1e-6) of the GPU forward kernel's own L."""
    import torch
    print_case("ftle grad vs gpu fd")
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 13, 64)
    T, eps, d = 400, 1e-2, 1e-6
    e = _explicit(aw, eps, T, 64)
    icd = _to_dev(ic)
    L, gic, geps = aw.ftle_grad(e, icd)                   # seeded tangent start, as map_ensemble
    g = np.vstack([np_(gic), np_(geps)[None]])

    def Lf(x, ep):
        ee = aw.Ensemble(eps=ep, n_steps=T, ic_kind="explicit", n_orbits=64, tangent=True)
        return np_(aw.map_ensemble(ee, x, want_class=False).orbit_out[aw.OUT_L])

    # The forward kernel steps in the rotated frame (x + y, x - y), the adjoint
    # in (x, y): the same map, rounded differently, so L agrees to rounding on
    # the regular orbits (the chaotic ones amplify it).
    reg = np_(L) / np.log(1 + T * H) < 1.5
    np.testing.assert_allclose(np_(L)[reg], Lf(icd, eps)[reg], rtol=1e-10, atol=0)
    fd = np.empty((7, 64))
    for c in range(6):
        dp = icd.clone()
        dp[c] += d
        dm = icd.clone()
        dm[c] -= d
        fd[c] = (Lf(dp, eps) - Lf(dm, eps)) / (2 * d)
    fd[6] = (Lf(icd, eps + d) - Lf(icd, eps - d)) / (2 * d)
    assert reg.sum() > 16
    _per_orbit_close(g[:, reg], fd[:, reg], 2e-6, "dL vs differences")
    torch.cuda.synchronize()


def test_ftle_gradient_independent_of_checkpoints(aw):
    """Ragged horizon (T = 333, not a multiple of 8 or of the interval): the
    result does not depend on the checkpoint interval, bit for bit, among the
    intervals that are multiples of 4 and the one-segment run (the same
    states are kept: every 4th step and the last); other intervals keep more
    states and agree to rounding."""
    print_case("ftle grad checkpoints")
    ic = _to_dev(oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 3, 300))
    e = _explicit(aw, 3e-2, 333, 300)
    ref = aw.ftle_grad(e, ic, ckpt_every=333)
    for ck in (4, 8, 64, 100, 332, 1000):
        got = aw.ftle_grad(e, ic, ckpt_every=ck)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(np_(a), np_(b))
    for ck in (1, 7, 37):
        got = aw.ftle_grad(e, ic, ckpt_every=ck)
        np.testing.assert_array_equal(np_(got[0]), np_(ref[0]))      # L is the forward pass's
        g = np.vstack([np_(got[1]), np_(got[2])[None]])
        r = np.vstack([np_(ref[1]), np_(ref[2])[None]])
        scale = np.max(np.abs(r), axis=0, keepdims=True)
        assert np.max(np.abs(g - r) / scale) <= 1e-11, ck


@pytest.mark.parametrize("reversible", [False, True])
def test_ftle_gradient_integrable_limit(aw, reversible):
    """At eps = 0 the map is free flight, X += t P: L takes the closed form
    ln(|dX0 + T h dP0|^2 + |dP0|^2)/2 - ln|w0|^2/2, which does not depend on the
    initial state.  Every kick and its derivatives are then exactly zero, so
    the state gradient vanishes exactly.  dL/deps does not: to first order
    the tangent picks up the Hessian kick, and the oracle's forward-over-forward
    derivative gives it (1e-9 relative)."""
    print_case("ftle grad eps=0", reversible)
    T, N = 300, 32
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 19, N)
    w0 = oracle.w0(0, N)
    L, gic, geps = aw.ftle_grad(_explicit(aw, 0.0, T, N), _to_dev(ic), _to_dev(w0), ckpt_every=40,
                                reversible=reversible)
    th = T * H
    Lc = 0.5 * np.log(np.sum((w0[0:3] + th * w0[3:6]) ** 2, axis=0) + np.sum(w0[3:6] ** 2, axis=0)) \
        - 0.5 * np.log(np.sum(w0 ** 2, axis=0))
    np.testing.assert_allclose(np_(L), Lc, rtol=1e-11, atol=0)
    assert np.all(np_(gic) == 0.0)
    _, dLo = oracle.ftle_grad_ensemble("s6", 0.0, H, T, ic, w0)
    assert np.all(dLo[:6] == 0.0)
    assert np.max(np.abs(dLo[6])) > 1e-3          # not zero at eps = 0
    np.testing.assert_allclose(np_(geps), dLo[6], rtol=1e-9, atol=0)


def test_ftle_gradient_edge_cases(aw):
    """T = 1 (one step, no rescale), T = 8 (the last step is a rescale step),
    one orbit, and an empty ensemble."""
    import torch
    print_case("ftle grad edges")
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 17, 5)
    w0 = oracle.w0(0, 5)
    for T in (1, 8, 9):
        Lo, dLo = oracle.ftle_grad_ensemble("s6", 0.1, H, T, ic, w0)
        L, gic, geps = aw.ftle_grad(_explicit(aw, 0.1, T, 5), _to_dev(ic), _to_dev(w0), ckpt_every=4)
        _per_orbit_close(np.vstack([np_(gic), np_(geps)[None]]), dLo, 1e-12, f"T={T}")
        np.testing.assert_allclose(np_(L), Lo, rtol=0, atol=1e-14)
    one = aw.ftle_grad(_explicit(aw, 0.1, 20, 1), _to_dev(ic[:, :1]), _to_dev(w0[:, :1]))
    Lo, dLo = oracle.ftle_grad_ensemble("s6", 0.1, H, 20, ic[:, :1], w0[:, :1])
    _per_orbit_close(np.vstack([np_(one[1]), np_(one[2])[None]]), dLo, 1e-12, "one orbit")
    empty = torch.empty((6, 0), dtype=torch.float64, device="cuda")
    L0, g0, e0 = aw.ftle_grad(_explicit(aw, 0.1, 20, 0), empty, empty)
    assert L0.shape == (0,) and g0.shape == (6, 0) and e0.shape == (0,)


@pytest.mark.parametrize("reversible", [False, True])
def test_ftle_autograd(aw, reversible):
    """IndicatorL: the backward of sum(c * L) equals the adjoint with upstream
    gradient c; the eps gradient is the sum of the per-orbit contributions."""
    import torch
    print_case("ftle autograd", reversible)
    ic = _to_dev(oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 23, 128))
    x = ic.t().contiguous().requires_grad_(True)
    eps = torch.tensor(2e-2, dtype=torch.float64, requires_grad=True)
    L = aw.IndicatorL.apply(x, eps, 300, H, "s6", 100, 0, reversible)
    c = torch.linspace(-1.0, 2.0, 128, dtype=torch.float64, device="cuda")
    (L * c).sum().backward()
    e = _explicit(aw, 2e-2, 300, 128)
    _, gic, geps = aw.ftle_grad(e, ic, grad_L=c, reversible=reversible)
    np.testing.assert_allclose(np_(x.grad), np_(gic).T, rtol=1e-14, atol=1e-14)
    assert abs(float(eps.grad) - float(geps.sum())) <= 1e-12 * max(1.0, abs(float(eps.grad)))


def test_ftle_gradient_full_size(aw):
    """The gradient workload at full size, in the configuration the benchmark
    times: the 512 x 512 slice, eps = 1e-2, T = 1e4, checkpoints every 100
    steps, all 262144 orbits in one call.  64 regular orbits drawn with seed 3
    against the oracle's forward-over-forward derivatives.  Bars: dL to 1e-6
    of the orbit's largest derivative and L to 1e-7 -- at this horizon a
    relative change of 1e-15 in the initial state alone moves the oracle's dL
    by up to 6e-8 and L by 2.4e-9 on these orbits."""
    print_case("ftle gradient 512x512 T=1e4")
    from paper_1107_4107_amd import workloads as wl
    s = wl.c4()
    N, T = s.nx * s.ny, s.n_steps
    ic_all, _ = aw.generate_ic(s)
    e = _explicit(aw, s.eps, T, N)
    L, gic, geps = aw.ftle_grad(e, ic_all, ckpt_every=wl.C4_CKPT)
    rng = np.random.default_rng(3)
    cand = np.sort(rng.choice(N, 160, replace=False))
    ic = oracle.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), s.nx, s.ny, list(s.base), idx=cand)
    w0 = oracle.w0(0, idx=cand)
    Lo, dLo = oracle.ftle_grad_ensemble("s6", s.eps, H, T, ic, w0)
    reg = Lo / np.log(1 + T * H) < 1.5
    pick = np.flatnonzero(reg)[:64]
    assert pick.size == 64
    Lg = np_(L)[cand[pick]]
    print(f"L: max abs err {np.max(np.abs(Lg - Lo[pick])):.3e}", flush=True)
    assert np.max(np.abs(Lg - Lo[pick])) < 1e-7
    g = np.vstack([np_(gic)[:, cand[pick]], np_(geps)[None, cand[pick]]])
    _per_orbit_close(g, dLo[:, pick], 1e-6, "dL full size")
    assert np.all(np.isfinite(np_(gic))) and np.all(np.isfinite(np_(geps)))


def test_adjoints_do_not_depend_on_the_block_size(aw):
    """Blocks of 64, 128, 256 and 512 (the default) threads, which fill the
    4096-entry sine/cosine table in 64 down to 8 passes and split the ensemble
    differently, give bitwise the same gradients, for both adjoints."""
    print_case("adjoint block sizes")
    ic = _to_dev(oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 29, 300))
    e = _explicit(aw, 2e-2, 200, 300)
    ej = aw.Ensemble(eps=2e-2, n_steps=200, ic_kind="explicit", n_orbits=300, tangent=False)
    ref_f = aw.ftle_grad(e, ic, ckpt_every=50)
    ref_j = aw.indicator_grad(ej, ic, ckpt_every=50)
    for b in (64, 128, 256):
        t = aw.Tuning(block=b)
        got_f = aw.ftle_grad(e, ic, ckpt_every=50, tuning=t)
        got_j = aw.indicator_grad(ej, ic, ckpt_every=50, tuning=t)
        for a, r in zip(got_f + got_j, ref_f + ref_j):
            np.testing.assert_array_equal(np_(a), np_(r))


@pytest.mark.parametrize("pz0", [0.0, 1.0])
def test_reversible_ftle_gradient_matches_oracle(aw, pz0):
    """The store-free sweep (each segment swept back from the next checkpoint,
    rescales undone with the recorded exponents) at the bars of the
    recompute-and-store sweep, and close to it."""
    print_case("reversible ftle grad vs oracle", pz0)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(128 * 128, 256, replace=False))
    ic = _slice_ic(128, pz0, idx)
    w0 = oracle.w0(0, idx=idx)
    T, eps = 1000, 1e-2
    Lo, dLo = oracle.ftle_grad_ensemble("s6", eps, H, T, ic, w0)
    e = _explicit(aw, eps, T, 256)
    L, gic, geps = aw.ftle_grad(e, _to_dev(ic), _to_dev(w0), ckpt_every=100, reversible=True)
    g = np.vstack([np_(gic), np_(geps)[None]])
    reg = Lo / np.log(1 + T * H) < 1.5
    assert np.max(np.abs(np_(L)[reg] - Lo[reg])) < 1e-9
    _per_orbit_close(g[:, reg], dLo[:, reg], 1e-8, "reversible dL (regular)")
    _, gs, es = aw.ftle_grad(e, _to_dev(ic), _to_dev(w0), ckpt_every=100)
    _per_orbit_close(g[:, reg], np.vstack([np_(gs), np_(es)[None]])[:, reg], 1e-9, "reversible vs store")


@pytest.mark.parametrize("form,T,ck", [("stdmap", 200, 30), ("y6", 200, 64), ("s6", 1, 4), ("s6", 8, 3), ("s6", 9, 9),
                                       ("s6", 333, 1)])
def test_reversible_ftle_gradient_forms_and_edges(aw, form, T, ck):
    print_case("reversible ftle grad", form, T, ck)
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 9, 64)
    w0 = oracle.w0(4, 64)
    eps = 2e-2
    Lo, dLo = oracle.ftle_grad_ensemble(form, eps, H, T, ic, w0)
    L, gic, geps = aw.ftle_grad(_explicit(aw, eps, T, 64, form), _to_dev(ic), _to_dev(w0), ckpt_every=ck,
                                reversible=True)
    g = np.vstack([np_(gic), np_(geps)[None]])
    reg = Lo / np.log(1 + T * H) < 1.5 if T > 50 else np.ones(64, dtype=bool)
    assert reg.sum() > 16
    _per_orbit_close(g[:, reg], dLo[:, reg], 1e-8, f"reversible dL {form} T={T}")


def test_reversible_ftle_gradient_full_size(aw):
    """Full size (512 x 512, eps = 1e-2, T = 1e4, checkpoints every 100
    steps), store-free sweep: 64 regular orbits (seed 3) against the oracle at
    the bars of the store sweep (dL 1e-6, L 1e-7)."""
    print_case("reversible ftle gradient 512x512 T=1e4")
    from paper_1107_4107_amd import workloads as wl
    s = wl.c4()
    N, T = s.nx * s.ny, s.n_steps
    ic_all, _ = aw.generate_ic(s)
    e = _explicit(aw, s.eps, T, N)
    L, gic, geps = aw.ftle_grad(e, ic_all, ckpt_every=wl.C4_CKPT, reversible=True)
    rng = np.random.default_rng(3)
    cand = np.sort(rng.choice(N, 160, replace=False))
    ic = oracle.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), s.nx, s.ny, list(s.base), idx=cand)
    w0 = oracle.w0(0, idx=cand)
    Lo, dLo = oracle.ftle_grad_ensemble("s6", s.eps, H, T, ic, w0)
    reg = Lo / np.log(1 + T * H) < 1.5
    pick = np.flatnonzero(reg)[:64]
    assert pick.size == 64
    assert np.max(np.abs(np_(L)[cand[pick]] - Lo[pick])) < 1e-7
    g = np.vstack([np_(gic)[:, cand[pick]], np_(geps)[None, cand[pick]]])
    _per_orbit_close(g, dLo[:, pick], 1e-6, "reversible dL full size")
