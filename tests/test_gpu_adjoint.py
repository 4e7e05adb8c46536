"""The hand-written adjoint of J = (1/T) sum_k |P_k - P_0|^2 (the
step-averaged momentum drift of the model section) against the oracle's
forward-mode derivatives (1e-9 relative on regular orbits), central finite
differences of the GPU's own J (step 1e-6, 1e-5 relative), a dot-product test,
and the exact zeros of the z -> -z symmetry on the invariant plane.  The
full-size slice (512 x 512, T = 1e4) is checked against stored oracle values
in test_gpu_parity_sets.py."""
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


def tensor(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _regular_ics(n, seed, eps, T, pz=True):
    rng = np.random.default_rng(seed)
    ic = np.empty((6, 0))
    while ic.shape[1] < n:
        c = np.vstack([rng.uniform(0, 2 * np.pi, (3, 4 * n)), rng.uniform(0.3, 2.0, (3, 4 * n))])
        if not pz:
            c[2] = 0.0
            c[5] = 0.0
        out = oracle.ensemble("s6", eps, H, T, c, oracle.w0(0, c.shape[1]))
        ic = np.hstack([ic, c[:, out[2] < 1.5]])
    return ic[:, :n]


def _grad_rel(g, ref, rel):
    # relative to the size of each orbit's gradient vector
    scale = np.maximum(np.max(np.abs(ref), axis=0, keepdims=True), 1e-300)
    err = np.abs(g - ref) / scale
    assert err.max() <= rel, f"max rel err {err.max():.3e}"


@pytest.mark.parametrize("form,T,ck", [("s6", 500, 50), ("s6", 537, 100), ("stdmap", 800, 64), ("s4", 300, 300)])
def test_adjoint_matches_forward_mode(aw, form, T, ck):
    print_case("adjoint vs forward mode", form, T, ck)
    eps = 1e-2
    ic = _regular_ics(64, 1, eps, T)
    e = aw.Ensemble(eps=eps, n_steps=T, map_form=form, ic_kind="explicit", n_orbits=64, tangent=False)
    J, gic, geps = aw.indicator_grad(e, tensor(ic), ckpt_every=ck)
    Jo, dJo = oracle.J_grad_ensemble(form, eps, H, T, ic)
    assert_close(np_(J), Jo, 1e-11, floor=1e-300, what="J")
    g = np.vstack([np_(gic), np_(geps)[None, :]])
    _grad_rel(g, dJo, 1e-9)


def test_adjoint_independent_of_checkpoints(aw):
    """The gradient does not depend on the checkpoint interval, bit for bit,
    among the intervals that are multiples of 4 and one segment (the forward
    pass then keeps the step states itself and the backward pass skips its
    recompute), with a ragged last segment: the same states are kept, those
    of every 4th step and of the last.  Other intervals also keep the end of
    every segment, and agree to rounding."""
    print_case("adjoint checkpoints")
    ic = tensor(oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 4, 200))
    e = aw.Ensemble(eps=3e-2, n_steps=333, ic_kind="explicit", n_orbits=200, tangent=False)
    ref = aw.indicator_grad(e, ic, ckpt_every=333)
    for ck in (4, 8, 64, 100, 332, 1000):
        got = aw.indicator_grad(e, ic, ckpt_every=ck)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(np_(a), np_(b))
    for ck in (1, 7, 37):
        got = aw.indicator_grad(e, ic, ckpt_every=ck)
        np.testing.assert_array_equal(np_(got[0]), np_(ref[0]))      # J is the forward pass's
        _grad_rel(np.vstack([np_(got[1]), np_(got[2])[None]]), np.vstack([np_(ref[1]), np_(ref[2])[None]]), 1e-11)


def test_adjoint_dot_product(aw):
    """<dL/dic, u> + dL/deps * v = sum_n gJ_n (dJ_n . (u_n, v)) for random gJ, u, v."""
    print_case("dot product")
    eps, T = 2e-2, 400
    ic = _regular_ics(32, 2, eps, T)
    rng = np.random.default_rng(9)
    gJ = rng.normal(size=32)
    e = aw.Ensemble(eps=eps, n_steps=T, ic_kind="explicit", n_orbits=32, tangent=False)
    _, gic, geps = aw.indicator_grad(e, tensor(ic), tensor(gJ), ckpt_every=37)
    _, dJo = oracle.J_grad_ensemble("s6", eps, H, T, ic)
    u = rng.normal(size=(6, 32))
    v = rng.normal()
    lhs = float(np.sum(np_(gic) * u) + np.sum(np_(geps)) * v)
    rhs = float(np.sum(gJ * (np.sum(dJo[:6] * u, axis=0) + dJo[6] * v)))
    assert abs(lhs - rhs) <= 1e-9 * max(abs(rhs), 1e-12)


def test_adjoint_against_finite_differences(aw):
    print_case("finite differences")
    eps, T, d = 1e-2, 1000, 1e-6
    ic = _regular_ics(16, 3, eps, T)
    e = aw.Ensemble(eps=eps, n_steps=T, ic_kind="explicit", n_orbits=16, tangent=False)
    _, gic, geps = aw.indicator_grad(e, tensor(ic), ckpt_every=100)
    g = np.vstack([np_(gic), np_(geps)[None, :]])

    def J_of(ic_, eps_):
        ee = aw.Ensemble(eps=eps_, n_steps=T, ic_kind="explicit", n_orbits=16, tangent=False)
        return np_(aw.map_ensemble(ee, tensor(ic_), want_class=False).orbit_out[aw.OUT_J])

    fd = np.empty((7, 16))
    for c in range(6):
        p, m = ic.copy(), ic.copy()
        p[c] += d
        m[c] -= d
        fd[c] = (J_of(p, eps) - J_of(m, eps)) / (2 * d)
    fd[6] = (J_of(ic, eps + d) - J_of(ic, eps - d)) / (2 * d)
    scale = np.max(np.abs(g), axis=0, keepdims=True)
    assert np.max(np.abs(g - fd) / scale) < 1e-5


def test_symmetry_zeros_on_the_invariant_plane(aw):
    print_case("symmetry zeros")
    ic = _regular_ics(16, 4, 1e-2, 300, pz=False)
    e = aw.Ensemble(eps=1e-2, n_steps=300, ic_kind="explicit", n_orbits=16, tangent=False)
    _, gic, _ = aw.indicator_grad(e, tensor(ic), ckpt_every=30)
    g = np_(gic)
    assert np.all(g[2] == 0.0) and np.all(g[5] == 0.0)


@pytest.mark.parametrize("reversible", [False, True])
def test_integrable_limit_gradient_is_zero(aw, reversible):
    """At eps = 0 every kick adds exactly zero, so P_k = P_0 at every step, J = 0
    for every initial state, and its whole gradient vanishes exactly (d/deps
    too: J is of second order in eps)."""
    print_case("adjoint eps=0", reversible)
    ic = oracle.ic_box([0.0] * 6, [2 * np.pi] * 6, 9, 64)
    e = aw.Ensemble(eps=0.0, n_steps=200, ic_kind="explicit", n_orbits=64, tangent=False)
    J, gic, geps = aw.indicator_grad(e, tensor(ic), ckpt_every=30, reversible=reversible)
    assert np.all(np_(J) == 0.0)
    assert np.all(np_(gic) == 0.0) and np.all(np_(geps) == 0.0)


@pytest.mark.parametrize("reversible", [False, True])
def test_autograd_function(aw, reversible):
    import torch
    print_case("autograd", reversible)
    eps, T = 1e-2, 300
    ic = _regular_ics(8, 5, eps, T)
    x = tensor(ic.T.copy()).requires_grad_(True)
    ep = torch.tensor(eps, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.arange(1, 9, dtype=torch.float64, device="cuda")
    J = aw.IndicatorJ.apply(x, ep, T, H, "s6", 100, reversible)
    (J * w).sum().backward()
    _, dJo = oracle.J_grad_ensemble("s6", eps, H, T, ic)
    gx = np_(x.grad).T
    _grad_rel(gx, dJo[:6] * np.arange(1, 9), 1e-9)
    ref = float(np.sum(dJo[6] * np.arange(1, 9)))
    assert abs(float(ep.grad) - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("form,T,ck", [("s6", 500, 50), ("s6", 537, 100), ("stdmap", 800, 64), ("y6", 400, 37),
                                       ("s6", 300, 1)])
def test_reversible_adjoint_matches_forward_mode(aw, form, T, ck):
    """The store-free sweep (segments swept back from the next checkpoint by
    inverting the steps) against the oracle's forward mode, at the same 1e-9
    bar, and against the recompute-and-store sweep to rounding."""
    print_case("reversible adjoint", form, T, ck)
    eps = 1e-2
    ic = _regular_ics(64, 1, eps, T)
    e = aw.Ensemble(eps=eps, n_steps=T, map_form=form, ic_kind="explicit", n_orbits=64, tangent=False)
    J, gic, geps = aw.indicator_grad(e, tensor(ic), ckpt_every=ck, reversible=True)
    Jo, dJo = oracle.J_grad_ensemble(form, eps, H, T, ic)
    assert_close(np_(J), Jo, 1e-11, floor=1e-300, what="J")
    g = np.vstack([np_(gic), np_(geps)[None, :]])
    _grad_rel(g, dJo, 1e-9)
    _, gic_s, geps_s = aw.indicator_grad(e, tensor(ic), ckpt_every=ck)
    _grad_rel(g, np.vstack([np_(gic_s), np_(geps_s)[None, :]]), 1e-11)
