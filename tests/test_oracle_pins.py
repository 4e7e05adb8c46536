"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every test here runs on the CPU.  Each pin is chosen so that a plausible slip
in the oracle (a dropped term or sign in the force or the Hessian, a wrong
composition coefficient, a transposed tangent column, a wrong accumulator)
makes at least one of them fail:

* the integrable limit eps = 0 (model section, after eq. 1), in closed form;
* the derivatives of eq. 2 against complex-step / mpmath differentiation of
  the formula as printed;
* the Hamiltonian flow of eqs. 1-2 integrated by SciPy's DOP853, and the
  order of convergence of each map form towards it;
* symplecticity (section "Computational method") and time reversibility;
* the reduction of the invariant plane z = p_z = 0 to two textbook Chirikov
  standard maps;
* the finite-time Lyapunov exponent at the hyperbolic and elliptic fixed
  points of eq. 2, in closed form;
* forward-mode derivatives of J against central finite differences;
* histogram counts against numpy's histogram2d, and the equal-area property
  of the direction binning;
* twenty steps of S6, S4 and the standard map redone at 50 digits from the
  definitions, the force by mpmath differentiation of the printed eq. 2 and
  the tangent by 50-digit central differences (state and L);
* reversibility and symplecticity on random initial states, eps, h and forms
  drawn by hypothesis.
"""
import json
import os

import mpmath
import numpy as np
import pytest
from scipy.integrate import solve_ivp

H_PAPER = 0.01 * 2.0 * np.pi  # h = 10^-2 T with T = 2 pi (section "Computational method")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# ---------------------------------------------------------------- helpers
def hp_literal(x, y, z):
    """Eq. 2 exactly as printed; works for complex arguments."""
    return np.cos(x) * np.cos(y) * (1 + np.cos(2 * z))


def grad_complex_step(X):
    """Gradient of eq. 2 by complex-step differentiation (exact to rounding)."""
    d = 1e-30
    g = np.empty(3)
    for a in range(3):
        Z = np.array(X, dtype=complex)
        Z[a] += 1j * d
        g[a] = hp_literal(*Z).imag / d
    return g


def flow_rhs(eps):
    def f(t, s):
        g = grad_complex_step(s[:3])
        return np.concatenate([s[3:], -eps * g])
    return f


def exact_flow(s0, eps, t):
    sol = solve_ivp(flow_rhs(eps), (0.0, t), s0, method="DOP853", rtol=1e-13, atol=1e-13)
    assert sol.success
    return sol.y[:, -1]


# ---------------------------------------------------------------- composition constants
def test_triple_jump_order_conditions(orc):
    """Triple-jump weights satisfy the order conditions of the composition:
    2 g1 + g0 = 1 with 2 g1^3 + g0^3 = 0 (4th order) and 2 d1 + d0 = 1 with
    2 d1^5 + d0^5 = 0 (6th order)."""
    g1, g0, d1, d0 = orc.tj_constants()
    assert abs(2 * g1 + g0 - 1) < 1e-15
    assert abs(2 * g1 ** 3 + g0 ** 3) < 1e-14
    assert abs(2 * d1 + d0 - 1) < 1e-15
    assert abs(2 * d1 ** 5 + d0 ** 5) < 1e-14


def test_y6_weights_give_order_six_on_a_free_lie_algebra(orc):
    """The 7-stage weights, checked without the order conditions they were
    solved from: with generic matrices A, B, C standing in for the terms of
    log S2(t) = t A + t^3 B + t^5 C, the symmetric product of the seven
    exponentials must equal exp((sum w) t A) up to O(t^7), so the remainder
    over t^5 is O(t^2) (sum w is taken exactly, since the double-rounded
    weights sum to 1 only within 1e-16).  The same weights in another order
    keep sum w^3 = sum w^5 = 0 but not the [A,[A,B]] condition, and leave an
    O(1) remainder, as does the 4th-order triple jump."""
    w0, w1, w2, w3 = orc.y6_weights()
    assert abs(w0 + 2 * (w1 + w2 + w3) - 1) < 1e-15
    mpmath.mp.dps = 50
    rng = np.random.default_rng(31)

    def rnd():
        return mpmath.matrix(rng.uniform(-1, 1, (4, 4)).tolist())

    A, B, C = rnd(), rnd(), rnd()

    def remainder(ws, t):
        t = mpmath.mpf(t)
        P = mpmath.eye(4)
        total = mpmath.mpf(0)
        for w in ws:
            wt = mpmath.mpf(float(w)) * t
            total += mpmath.mpf(float(w))
            P = P * mpmath.expm(wt * A + wt ** 3 * B + wt ** 5 * C)
        return mpmath.mnorm(mpmath.logm(P) - total * t * A, 1) / t ** 5

    good = (w3, w2, w1, w0, w1, w2, w3)
    r1, r2 = remainder(good, "2e-3"), remainder(good, "1e-3")
    assert r1 < 1e-3 and 2.5 < r1 / r2 < 6, (r1, r2)          # O(t^2)
    assert remainder((w1, w2, w3, w0, w3, w2, w1), "1e-3") > 1.0
    g1, g0, _, _ = orc.tj_constants()
    assert remainder((g1, g0, g1), "1e-3") > 1.0


# ---------------------------------------------------------------- eq. 2 derivatives
def test_hp_derivatives_against_mpmath(orc):
    rng = np.random.default_rng(11)
    mpmath.mp.dps = 30

    def f(x, y, z):
        return mpmath.cos(x) * mpmath.cos(y) * (1 + mpmath.cos(2 * z))

    for _ in range(8):
        X = rng.uniform(-7, 7, 3)
        hp, g, H6 = orc.hp_derivs(X)
        x, y, z = (mpmath.mpf(float(v)) for v in X)
        assert abs(hp - float(f(x, y, z))) < 1e-15
        for a, order in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            assert abs(g[a] - float(mpmath.diff(f, (x, y, z), order))) < 1e-14
        orders = [(2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
        for a, order in enumerate(orders):
            assert abs(H6[a] - float(mpmath.diff(f, (x, y, z), order))) < 1e-13


def test_hp_third_derivatives_against_mpmath(orc):
    """All 27 third derivatives of eq. 2's Hp (they enter the derivative of the
    tangent kick) against mpmath's numerical differentiation."""
    rng = np.random.default_rng(12)
    mpmath.mp.dps = 30

    def f(x, y, z):
        return mpmath.cos(x) * mpmath.cos(y) * (1 + mpmath.cos(2 * z))

    for _ in range(6):
        X = rng.uniform(-7, 7, 3)
        T3 = orc.hp_third(X)
        x, y, z = (mpmath.mpf(float(v)) for v in X)
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    order = [0, 0, 0]
                    for a in (i, j, k):
                        order[a] += 1
                    ref = float(mpmath.diff(f, (x, y, z), tuple(order)))
                    assert abs(T3[i, j, k] - ref) < 1e-13, ((i, j, k), T3[i, j, k], ref)


def test_hp_fourier_form_and_bound(orc):
    """Product-to-sum form of eq. 2: its Fourier modes are the primary
    resonances (1, +-1, 0) and (1, +-1, +-2); and |Hp| <= 2 (model section)."""
    gold = json.load(open(GOLDEN))
    rng = np.random.default_rng(5)
    for _ in range(20):
        x, y, z = rng.uniform(-10, 10, 3)
        four = 0.5 * (np.cos(x + y) + np.cos(x - y)) + 0.25 * (
            np.cos(x + y + 2 * z) + np.cos(x + y - 2 * z) + np.cos(x - y + 2 * z) + np.cos(x - y - 2 * z))
        s = np.array([x, y, z, 0, 0, 0])
        assert abs(orc.energy(s, 1.0) - four) < 1e-14
        assert abs(orc.energy(s, 1.0)) <= gold["Hp_bound"]["value"]
    assert orc.energy(np.zeros(6), 1.0) == gold["Hp_bound"]["value"]


# ---------------------------------------------------------------- eps = 0
@pytest.mark.parametrize("form", ["stdmap", "s2", "s4", "s6", "y6"])
def test_integrable_limit(orc, form):
    """eps = 0: P constant, X(t) = X(0) + P t, and the tangent grows by the
    linear shear: L_T = 1/2 ln(|dX0 + T h dP0|^2 + |dP0|^2)."""
    rng = np.random.default_rng(1)
    N, T = 16, 300
    ic = rng.uniform(0, 2 * np.pi, (6, N))
    w0 = orc.w0(7, N)
    out, st = orc.ensemble(form, 0.0, H_PAPER, T, ic, w0, want_state=True)
    th = T * H_PAPER
    np.testing.assert_array_equal(st[3:6], ic[3:6])
    np.testing.assert_allclose(st[0:3], ic[0:3] + th * ic[3:6], rtol=1e-12, atol=1e-12)
    L = 0.5 * np.log(np.sum((w0[0:3] + th * w0[3:6]) ** 2, axis=0) + np.sum(w0[3:6] ** 2, axis=0))
    np.testing.assert_allclose(out[0], L, rtol=1e-11)
    # lambda = L / (T h) (the finite-time Lyapunov exponent) and
    # chi = L / ln(1 + T h): the shear alone gives chi <= 1 + ln 2 / (2 ln(1 + T h)).
    np.testing.assert_allclose(out[1], L / th, rtol=1e-11)
    np.testing.assert_allclose(out[2], L / np.log1p(th), rtol=1e-11)
    assert np.all(out[2] <= 1.0 + 0.5 * np.log(2.0) / np.log1p(th))
    np.testing.assert_allclose(out[3:6], ic[3:6], rtol=1e-12, atol=1e-13)
    assert np.all(out[6] == 0) and np.all(out[7] == 0) and np.all(out[8] == 0)


# ---------------------------------------------------------------- the flow of eqs. 1-2
def test_s6_tracks_hamiltonian_flow(orc):
    """S6 at a small step reproduces the DOP853 solution of Hamilton's
    equations of eqs. 1-2 (force from the printed eq. 2, not from the oracle)."""
    rng = np.random.default_rng(2)
    for eps in (1.0, 0.1):
        s0 = np.concatenate([rng.uniform(0, 2 * np.pi, 3), rng.uniform(-1.5, 1.5, 3)])
        h, T = 0.02, 100
        ref = exact_flow(s0, eps, h * T)
        got = orc.map_state("s6", eps, h, T, s0)
        assert np.max(np.abs(got - ref)) < 1e-10


@pytest.mark.parametrize("form,order,h", [("stdmap", 1, 0.02), ("s2", 2, 0.05), ("s4", 4, 0.1), ("s6", 6, 0.2),
                                          ("y6", 6, 0.2)])
def test_convergence_order(orc, form, order, h):
    """Error against the exact flow falls by 2^order per halving of h."""
    s0 = np.array([0.3, 1.1, 0.7, 0.9, -0.4, 0.6])
    t, eps = 2.0, 1.0
    ref = exact_flow(s0, eps, t)
    errs = []
    for hh in (h, h / 2):
        T = int(round(t / hh))
        errs.append(np.max(np.abs(orc.map_state(form, eps, hh, T, s0) - ref)))
    ratio = errs[0] / errs[1]
    assert 0.75 * 2 ** order < ratio < 1.3 * 2 ** order, (errs, ratio)


# ---------------------------------------------------------------- symplecticity, reversibility
@pytest.mark.parametrize("form", ["stdmap", "s6", "y6"])
def test_symplectic_jacobian(orc, form):
    Om = np.block([[np.zeros((3, 3)), np.eye(3)], [-np.eye(3), np.zeros((3, 3))]])
    s0 = np.array([0.4, 2.0, 1.3, 0.7, 0.2, -0.5])
    _, M = orc.jacobian(form, 0.3, H_PAPER, 50, s0)
    assert np.max(np.abs(M.T @ Om @ M - Om)) < 1e-11
    assert abs(np.linalg.det(M) - 1.0) < 1e-10


@pytest.mark.parametrize("form", ["stdmap", "s6"])
def test_jacobian_against_finite_differences(orc, form):
    s0 = np.array([0.4, 2.0, 1.3, 0.7, 0.2, -0.5])
    eps, T, d = 0.05, 20, 1e-6
    _, M = orc.jacobian(form, eps, H_PAPER, T, s0)
    fd = np.empty((6, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = d
        fd[:, j] = (orc.map_state(form, eps, H_PAPER, T, s0 + e) - orc.map_state(form, eps, H_PAPER, T, s0 - e)) / (2 * d)
    assert np.max(np.abs(M - fd)) < 1e-7


@pytest.mark.parametrize("form", ["s2", "s4", "s6", "y6"])
def test_time_reversibility(orc, form):
    """Symmetric compositions: S(-h) S(h) = id and R S R S = id, R(X, P) = (X, -P)."""
    s0 = np.array([0.4, 2.0, 1.3, 0.7, 0.2, -0.5])
    fwd = orc.map_state(form, 0.5, H_PAPER, 40, s0)
    back = orc.map_state(form, 0.5, -H_PAPER, 40, fwd)
    assert np.max(np.abs(back - s0)) < 1e-12
    r = fwd.copy()
    r[3:] *= -1
    rr = orc.map_state(form, 0.5, H_PAPER, 40, r)
    rr[3:] *= -1
    assert np.max(np.abs(rr - s0)) < 1e-12


# ---------------------------------------------------------------- invariant plane
def test_invariant_plane_is_two_chirikov_maps(orc):
    """On z = p_z = 0, eq. 2 reduces to eps (cos u + cos v) with u = x + y,
    v = x - y, and the kick-then-drift map becomes, for each of u and v, the
    Chirikov standard map I' = I + K sin u, u' = u + I', I = 2 h p_u, K = 2 eps h^2."""
    eps, h, T = 0.2, 0.3, 60
    s = np.array([0.9, -0.35, 0.0, 0.4, 1.3, 0.0])
    u, v = s[0] + s[1], s[0] - s[1]
    Iu, Iv = 2 * h * (s[3] + s[4]) / 2, 2 * h * (s[3] - s[4]) / 2
    K = 2 * eps * h * h
    for _ in range(T):
        s = orc.map_state("stdmap", eps, h, 1, s)
        Iu = Iu + K * np.sin(u)
        u = u + Iu
        Iv = Iv + K * np.sin(v)
        v = v + Iv
        assert s[2] == 0.0 and s[5] == 0.0
    assert abs((s[0] + s[1]) - u) < 1e-11 and abs((s[0] - s[1]) - v) < 1e-11
    assert abs(2 * h * (s[3] + s[4]) / 2 - Iu) < 1e-12
    assert abs(2 * h * (s[3] - s[4]) / 2 - Iv) < 1e-12
    # The 6th-order map keeps the plane invariant too (exact zeros).
    s6 = orc.map_state("s6", 0.01, H_PAPER, 500, np.array([0.0, 0.0, 0.0, 2.0, 1.0, 0.0]))
    assert s6[2] == 0.0 and s6[5] == 0.0


def _chirikov_observables(s0, w0, eps, h, T):
    """Per-orbit rows (L, lambda, chi, V, dP2, J, dE) of the kick-then-drift
    map on the invariant plane, accumulated from two textbook Chirikov maps
    in u = x + y, v = x - y (I = 2 h p_u, K = 2 eps h^2) and the linear map of
    the out-of-plane tangent.  On the plane eq. 2 is eps (cos u + cos v), so
    H = p_u^2 + p_v^2 + eps (cos u + cos v) with p_u = (px + py)/2, and
    |P - P0|^2 = 2 (dp_u^2 + dp_v^2).  Off the plane, Hp_zz = -4 cos x cos y =
    -2 (cos u + cos v) at z = 0, so the kick sends dp_z -> dp_z + 2 h eps
    (cos u + cos v) dz; the drift dz -> dz + h dp_z."""
    K = 2.0 * eps * h * h
    u, v = s0[0] + s0[1], s0[0] - s0[1]
    Iu, Iv = h * (s0[3] + s0[4]), h * (s0[3] - s0[4])
    u0, v0, Iu0, Iv0 = u, v, Iu, Iv
    # tangent: (du, dIu), (dv, dIv), (dz, dpz)
    du, dv = w0[0] + w0[1], w0[0] - w0[1]
    dIu, dIv = h * (w0[3] + w0[4]), h * (w0[3] - w0[4])
    dz, dpz = w0[2], w0[5]
    jsum = 0.0
    for _ in range(T):
        cs = np.cos(u) + np.cos(v)
        dIu = dIu + K * np.cos(u) * du
        dIv = dIv + K * np.cos(v) * dv
        dpz = dpz + 2.0 * h * eps * cs * dz
        Iu = Iu + K * np.sin(u)
        Iv = Iv + K * np.sin(v)
        u, v = u + Iu, v + Iv
        du, dv = du + dIu, dv + dIv
        dz = dz + h * dpz
        jsum += 2.0 * ((Iu - Iu0) ** 2 + (Iv - Iv0) ** 2) / (2.0 * h) ** 2
    th = T * h
    w2 = ((du + dv) / 2) ** 2 + ((du - dv) / 2) ** 2 + dz ** 2 + \
         ((dIu + dIv) / (2 * h)) ** 2 + ((dIu - dIv) / (2 * h)) ** 2 + dpz ** 2
    L = 0.5 * np.log(w2 / np.sum(np.asarray(w0) ** 2))
    energy = lambda a, b, Ia, Ib: (Ia ** 2 + Ib ** 2) / (2 * h) ** 2 + eps * (np.cos(a) + np.cos(b))
    return np.array([L, L / th, L / np.log1p(th),
                     ((u + v) - (u0 + v0)) / 2 / th, ((u - v) - (u0 - v0)) / 2 / th, 0.0,
                     2.0 * ((Iu - Iu0) ** 2 + (Iv - Iv0) ** 2) / (2.0 * h) ** 2, jsum / T,
                     energy(u, v, Iu, Iv) - energy(u0, v0, Iu0, Iv0)])


def test_accumulators_on_invariant_plane(orc):
    """Every per-orbit row at eps != 0 against the two Chirikov maps of the
    invariant plane: the step-averaged drift J = (1/T) sum_{k=1..T} |P_k - P_0|^2,
    the final drift dP2, the mean velocity V, the energy change and the
    tangent growth L (with lambda and chi) -- all from independently written
    textbook maps, so that a slip in the oracle's accumulators (a shifted step
    range, a missing factor, a wrong norm) shows at eps != 0, where J and dP2
    are not zero.  Regular and chaotic starts (K = 0.5 over 30 steps, short enough
    that rounding has not yet separated chaotic orbits), T = 30 to 200."""
    rng = np.random.default_rng(12)
    for eps, h, T in ((0.2, 0.3, 80), (1.0, 0.5, 30), (0.05, H_PAPER, 200)):
        N = 8
        ic = np.zeros((6, N))
        ic[0:2] = rng.uniform(0, 2 * np.pi, (2, N))
        ic[3:5] = rng.uniform(-2.0, 2.0, (2, N))
        w0 = orc.w0(5, N)
        out = orc.ensemble("stdmap", eps, h, T, ic, w0)
        for n in range(N):
            ref = _chirikov_observables(ic[:, n], w0[:, n], eps, h, T)
            assert out[5, n] == 0.0
            np.testing.assert_allclose(out[:, n], ref, rtol=1e-9, atol=1e-12 * max(1.0, abs(ref[0])),
                                       err_msg=f"eps={eps} h={h} T={T} orbit {n}")
            assert out[7, n] > 1e-6 and out[6, n] > 0.0
        # summing over k = 0..T-1 instead would move J by dP2 / T, far beyond the tolerance
        assert np.all(out[6] / T > 1e-6 * out[7])


# ---------------------------------------------------------------- energy
def test_energy_bounded_and_in_layer(orc):
    """No secular energy growth under the symplectic map, and P^2 stays in the
    layer 2(E - 2 eps) <= P^2 <= 2(E + 2 eps) implied by |Hp| <= 2."""
    eps = 1.0
    s = np.array([0.3, 1.0, 2.0, 4.0, 3.0, 2.5])
    E0 = orc.energy(s, eps)
    dE = []
    for _ in range(200):
        s = orc.map_state("s6", eps, H_PAPER, 50, s)
        dE.append(abs(orc.energy(s, eps) - E0))
        p2 = np.sum(s[3:] ** 2)
        assert 2 * (E0 - 2 * eps) - 1e-8 <= p2 <= 2 * (E0 + 2 * eps) + 1e-8
    dE = np.array(dE)
    assert dE.max() < 1e-6
    assert dE[100:].max() < 3 * dE[:100].max() + 1e-12


# ---------------------------------------------------------------- Lyapunov indicator
def test_ftle_at_hyperbolic_point(orc):
    """X = 0, P = 0 is the maximum of eq. 2 (Hp = 2 - x^2 - y^2 - 2 z^2 + ...),
    a fixed point whose linearisation has growth rates sqrt(2 eps) (x, y) and
    sqrt(4 eps) (z); the FTLE tends to the largest."""
    eps, T = 0.1, 20000
    out = orc.ensemble("s6", eps, H_PAPER, T, np.zeros((6, 1)), orc.w0(0, 1))
    assert abs(out[1, 0] - np.sqrt(4 * eps)) < 0.01
    assert out[2, 0] > 2.0


def test_ftle_at_elliptic_point(orc):
    """X = (pi, 0, 0), P = 0 is the minimum of eq. 2: the tangent only rotates,
    L stays bounded and the indicator reads regular."""
    ic = np.array([[np.pi], [0], [0], [0], [0], [0]], dtype=float)
    out = orc.ensemble("s6", 0.1, H_PAPER, 20000, ic, orc.w0(0, 1))
    assert abs(out[0, 0]) < 3.0
    assert out[2, 0] < 0.5


def test_regular_orbits_keep_velocity_near_initial_momentum(orc):
    """Regular orbits keep V close to P(0) (section Main results): at small eps
    |V - P0| is O(eps)."""
    ic = orc.ic_grid2((3, 4), (0.5, 0.5), (2 * np.pi, 2 * np.pi), 8, 8, [0, 0, 0, 0, 0, 1.0])
    for eps in (1e-4, 1e-3):
        out = orc.ensemble("s6", eps, H_PAPER, 2000, ic, orc.w0(0, 64))
        reg = out[2] < 1.5
        assert reg.mean() > 0.8
        dv = np.max(np.abs(out[3:6, reg] - ic[3:6, reg]))
        assert dv < 40 * eps


# ---------------------------------------------------------------- J derivatives
def test_J_forward_mode_against_finite_differences(orc):
    s0 = np.array([0.4, 2.0, 0.3, 0.9, 0.5, 0.2])
    eps, T, d = 1e-2, 300, 1e-6
    J, dJ = orc.J_grad("s6", eps, H_PAPER, T, s0)
    assert J > 0
    for c in range(7):
        if c < 6:
            e = np.zeros(6)
            e[c] = d
            Jp, _ = orc.J_grad("s6", eps, H_PAPER, T, s0 + e)
            Jm, _ = orc.J_grad("s6", eps, H_PAPER, T, s0 - e)
        else:
            Jp, _ = orc.J_grad("s6", eps + d, H_PAPER, T, s0)
            Jm, _ = orc.J_grad("s6", eps - d, H_PAPER, T, s0)
        fd = (Jp - Jm) / (2 * d)
        assert abs(dJ[c] - fd) <= 1e-6 * max(abs(fd), 1e-3), (c, dJ[c], fd)
    # J also equals the accumulator of the one-tangent run.
    out = orc.ensemble("s6", eps, H_PAPER, T, s0.reshape(6, 1), orc.w0(0, 1))
    assert abs(out[7, 0] - J) <= 1e-14 * J


def test_J_gradient_symmetry_on_invariant_plane(orc):
    """z -> -z, p_z -> -p_z is a symmetry of eq. 2, so dJ/dz0 = dJ/dpz0 = 0
    exactly on the plane z = p_z = 0."""
    _, dJ = orc.J_grad("s6", 1e-2, H_PAPER, 200, np.array([0.0, 0.0, 0.0, 1.3, 2.1, 0.0]))
    assert dJ[2] == 0.0 and dJ[5] == 0.0


@pytest.mark.parametrize("form,eps,T", [("s6", 5e-2, 60), ("s6", 1.0, 40), ("stdmap", 0.3, 80), ("s2", 0.1, 50),
                                        ("y6", 0.2, 40)])
def test_ftle_gradient_against_finite_differences(orc, form, eps, T):
    """Forward-over-forward dL/d(x0..pz0, eps) against central differences of
    the plain one-tangent oracle's L (a separate code path: no third
    derivatives), at a fixed tangent start."""
    rng = np.random.default_rng(21)
    d = 1e-6
    for _ in range(3):
        s0 = np.concatenate([rng.uniform(-3, 3, 3), rng.uniform(-1.5, 1.5, 3)])
        w = rng.normal(size=6)
        w /= np.linalg.norm(w)
        L, dL, _ = orc.ftle_grad(form, eps, H_PAPER, T, s0, w)

        def plain(s, e):
            return orc.ensemble(form, e, H_PAPER, T, s.reshape(6, 1), w.reshape(6, 1))[0, 0]

        assert abs(L - plain(s0, eps)) <= 1e-13 * max(1.0, abs(L))
        for c in range(7):
            if c < 6:
                e = np.zeros(6)
                e[c] = d
                fd = (plain(s0 + e, eps) - plain(s0 - e, eps)) / (2 * d)
            else:
                fd = (plain(s0, eps + d) - plain(s0, eps - d)) / (2 * d)
            assert abs(dL[c] - fd) <= 2e-7 * max(1.0, abs(fd)), (c, dL[c], fd)


def test_ftle_gradient_in_the_integrable_limit(orc):
    """eps = 0: L = 1/2 ln(|dX0 + T h dP0|^2 + |dP0|^2) does not depend on the
    initial state, so dL/d(x0..pz0) is exactly 0; dL/deps then follows from
    first-order perturbation of the free flight, checked by differences."""
    s0 = np.array([0.3, 1.2, -0.4, 0.8, -0.6, 1.1])
    w = np.array([0.3, -0.2, 0.5, 0.4, 0.1, -0.6])
    w /= np.linalg.norm(w)
    T = 120
    L, dL, _ = orc.ftle_grad("s6", 0.0, H_PAPER, T, s0, w)
    th = T * H_PAPER
    assert abs(L - 0.5 * np.log(np.sum((w[:3] + th * w[3:]) ** 2) + np.sum(w[3:] ** 2))) < 1e-13
    assert np.all(dL[:6] == 0.0)
    d = 1e-7
    Lp = orc.ftle_grad("s6", d, H_PAPER, T, s0, w)[0]
    Lm = orc.ftle_grad("s6", -d, H_PAPER, T, s0, w)[0]
    assert abs(dL[6] - (Lp - Lm) / (2 * d)) <= 1e-6 * max(1.0, abs(dL[6]))


def test_ftle_gradient_ignores_the_tangent_scale(orc):
    """L is a ratio |w_T| / |w_0|, so scaling w0 changes neither L nor dL."""
    s0 = np.array([0.5, -0.7, 0.2, 1.1, 0.3, -0.4])
    w = np.array([0.2, 0.4, -0.1, -0.3, 0.6, 0.5])
    w /= np.linalg.norm(w)
    L1, d1, _ = orc.ftle_grad("s6", 0.2, H_PAPER, 80, s0, w)
    L2, d2, _ = orc.ftle_grad("s6", 0.2, H_PAPER, 80, s0, 8.0 * w)
    assert abs(L1 - L2) < 1e-13
    np.testing.assert_allclose(d2, d1, rtol=1e-12, atol=1e-13)


def test_ftle_gradient_ensemble_matches_single_orbits(orc):
    ic = orc.ic_box([0.0] * 6, [2 * np.pi] * 6, 5, 16)
    w = orc.w0(0, 16)
    L, dL = orc.ftle_grad_ensemble("s6", 0.05, H_PAPER, 30, ic, w, nthreads=4)
    for n in (0, 7, 15):
        L1, d1, _ = orc.ftle_grad("s6", 0.05, H_PAPER, 30, ic[:, n], w[:, n])
        assert L[n] == L1
        np.testing.assert_array_equal(dL[:, n], d1)


# ---------------------------------------------------------------- resume
def test_chunked_run_is_bitwise_equal(orc):
    s0 = np.array([0.1, 0.2, 0.3, 1.0, 2.0, 0.5])
    w = orc.w0(3, 1)[:, 0]
    full = orc.rec_advance("s6", 0.02, H_PAPER, 500, orc.rec_init(s0, w))
    part = orc.rec_init(s0, w)
    for n in (123, 77, 300):
        part = orc.rec_advance("s6", 0.02, H_PAPER, n, part)
    np.testing.assert_array_equal(part, full)
    np.testing.assert_array_equal(orc.rec_finish(part, 0.02, H_PAPER), orc.rec_finish(full, 0.02, H_PAPER))


# ---------------------------------------------------------------- inputs
def test_splitmix64_counter_form_matches_sequential_generator(orc):
    """Output c of the sequential SplitMix64 generator (state += gamma; mix)."""
    M = (1 << 64) - 1

    def seq(seed, n):
        st, out = seed, []
        for _ in range(n):
            st = (st + 0x9E3779B97F4A7C15) & M
            z = st
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            out.append(z ^ (z >> 31))
        return out

    for seed in (0, 1, 2, 12345678901234567):
        ref = seq(seed, 40)
        assert [orc.splitmix64(seed, c) for c in range(40)] == ref
        assert all(orc.u01(seed, c) == (ref[c] >> 11) * 2.0 ** -53 for c in range(40))


def test_uniform_draws_are_uniform(orc):
    from scipy.stats import kstest
    ic = orc.ic_box([0] * 6, [1] * 6, 2, 20000)
    for k in range(6):
        assert kstest(ic[k], "uniform").pvalue > 1e-4
    w = orc.w0(0, 1000)
    np.testing.assert_allclose(np.sqrt(np.sum(w * w, axis=0)), 1.0, atol=2e-16)


def test_grid_left_edges(orc):
    ic = orc.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), 64, 32, [9, 8, 7, 6, 5, 4])
    d0, d1 = 2 * np.pi / 64, 2 * np.pi / 32
    n = np.arange(64 * 32)
    np.testing.assert_array_equal(ic[3], (n % 64) * d0)
    np.testing.assert_array_equal(ic[4], (n // 64) * d1)
    assert ic[3].min() == 0 and ic[3].max() < 2 * np.pi
    np.testing.assert_array_equal(ic[[0, 1, 2, 5]], np.array([[9], [8], [7], [4]]) * np.ones((1, n.size)))
    sub = orc.ic_grid2((3, 4), (0, 0), (2 * np.pi, 2 * np.pi), 64, 32, [9, 8, 7, 6, 5, 4], idx=[5, 700])
    np.testing.assert_array_equal(sub, ic[:, [5, 700]])


# ---------------------------------------------------------------- images
def test_hist2d_matches_numpy(orc):
    rng = np.random.default_rng(9)
    N, W, H = 50000, 37, 23
    a = rng.uniform(-0.5, 7.0, N)
    b = rng.uniform(-0.2, 6.5, N)
    v = rng.normal(size=N)
    counts, sums, dropped = orc.hist2d(a, b, v, (0, 0), (2 * np.pi, 2 * np.pi), W, H)
    ref, _, _ = np.histogram2d(b, a, bins=[H, W], range=[[0, 2 * np.pi], [0, 2 * np.pi]])
    np.testing.assert_array_equal(counts, ref.astype(np.uint32))
    assert counts.sum() + dropped == N
    i = np.floor(a / (2 * np.pi) * W).astype(int)
    j = np.floor(b / (2 * np.pi) * H).astype(int)
    ok = (i >= 0) & (i < W) & (j >= 0) & (j < H)
    ref_s = np.zeros((H, W))
    np.add.at(ref_s, (j[ok], i[ok]), v[ok])
    np.testing.assert_allclose(sums, ref_s, rtol=1e-12, atol=1e-12)


def test_direction_density_is_equal_area(orc):
    """Isotropic directions give a flat density 1/(4 pi) in (phi, mu) bins."""
    rng = np.random.default_rng(4)
    N, W, H = 400000, 16, 8
    V = rng.normal(size=(3, N)) * 3.0
    dens, counts, dropped = orc.hist_vdir(V, W, H)
    assert dropped == 0 and counts.sum() == N
    expect = N / (W * H)
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < W * H + 6 * np.sqrt(2 * W * H)
    np.testing.assert_allclose(dens.mean(), 1 / (4 * np.pi), rtol=1e-12)


# ---------------------------------------------------------------- paper constants
def test_paper_constants(orc):
    g = json.load(open(GOLDEN))
    # eq. 3: eps_eff = max|Hp| / H = 2 / E, with eps = 1.
    assert 2.0 / g["E_weak"]["value"] == pytest.approx(g["eps_eff_weak"]["value"], rel=1e-15)
    a, b = g["eps_eff_moderate"]["value"]
    assert 2.0 / g["E_moderate"]["value"] == pytest.approx(a / b, rel=1e-15)
    # W = (sqrt E, sqrt E, 0) lies on the three resonance planes and on the sphere P^2 = 2E.
    E = g["E_moderate"]["value"]
    W = np.sqrt(E) * np.array(g["W_point_over_sqrtE"]["value"])
    for m in g["W_resonances"]["value"]:
        assert abs(np.dot(m, W)) < 1e-14
    assert abs(W @ W - 2 * E) < 1e-12
    assert H_PAPER == pytest.approx(g["step_over_T"]["value"] * 2 * np.pi)


# ---------------------------------------------------------------- fixed-energy ensembles
def test_sphere_initial_conditions_lie_on_the_energy_shell(orc):
    """Figs. 2-3 start from a fixed total energy (eq. 1): H(P, X) = E exactly
    up to rounding, the direction of P uniform in area on the chosen segment of
    the sphere (uniform in phi and in mu = cos theta), X uniform on the torus."""
    from scipy.stats import kstest
    g = json.load(open(GOLDEN))
    for E, seg in ((g["E_weak"]["value"], (-np.pi, np.pi, -1.0, 1.0)), (g["E_moderate"]["value"], (0.3, 0.9, 0.1, 0.4))):
        N = 20000
        ic = orc.ic_sphere(E, 1.0, seg[:2], seg[2:], [0, 0, 0], [2 * np.pi] * 3, 7, N)
        H = np.array([orc.energy(ic[:, n], 1.0) for n in range(0, N, 97)])
        np.testing.assert_allclose(H, E, rtol=1e-14)
        P = ic[3:]
        r = np.sqrt(np.sum(P * P, axis=0))
        phi, mu = np.arctan2(P[1], P[0]), P[2] / r
        assert phi.min() >= seg[0] - 1e-12 and phi.max() <= seg[1] + 1e-12
        assert mu.min() >= seg[2] - 1e-12 and mu.max() <= seg[3] + 1e-12
        assert kstest((phi - seg[0]) / (seg[1] - seg[0]), "uniform").pvalue > 1e-4
        assert kstest((mu - seg[2]) / (seg[3] - seg[2]), "uniform").pvalue > 1e-4
        assert kstest(ic[0] / (2 * np.pi), "uniform").pvalue > 1e-4


def test_window_test(orc):
    """The stay-in-area test: with the whole sphere as window no orbit leaves;
    at eps = 0 the momentum is constant, so the margin is the initial one; a
    window around an orbit's start that the orbit crosses flags it."""
    N = 64
    ic = orc.ic_sphere(15.0, 1.0, (-np.pi, np.pi), (-1.0, 1.0), [0, 0, 0], [2 * np.pi] * 3, 3, N)
    w0 = orc.w0(0, N)
    _, left, margin = orc.ensemble_window("s6", 1.0, H_PAPER, 300, ic, w0, (-np.pi, np.pi, -1.0, 1.0))
    assert not left.any() and np.all(margin >= 0)
    seg = (0.2, 0.6, -0.3, 0.2)
    ic = orc.ic_sphere(15.0, 1.0, seg[:2], seg[2:], [0, 0, 0], [2 * np.pi] * 3, 5, N)
    _, left0, m0 = orc.ensemble_window("s6", 0.0, H_PAPER, 50, ic, w0, seg)
    P = ic[3:]
    phi, mu = np.arctan2(P[1], P[0]), P[2] / np.sqrt(np.sum(P * P, axis=0))
    init = np.minimum.reduce([phi - seg[0], seg[1] - phi, mu - seg[2], seg[3] - mu])
    np.testing.assert_allclose(m0, init, atol=1e-15)
    assert not left0.any()
    # with the full perturbation most momenta wander out of a narrow window
    _, left1, m1 = orc.ensemble_window("s6", 1.0, H_PAPER, 2000, ic, w0, seg)
    assert left1.mean() > 0.5 and np.all((m1 < 0) == (left1 == 1))


def test_fig4_cloud(orc):
    """Fig. 4's injected cloud: a Gaussian in (vx, vy) around W = (sqrt E, sqrt E)
    with the printed dispersions, X uniform on the torus, vz from H = E."""
    from scipy.stats import kstest
    g = json.load(open(GOLDEN))
    E = g["E_moderate"]["value"]
    W = np.sqrt(E) * np.array(g["W_point_over_sqrtE"]["value"])
    s = g["fig4_sigma_v"]["value"]
    ic = orc.ic_cloud(E, 1.0, [W[0], W[1], s, s], [0, 0, 0], [2 * np.pi] * 3, 11, n_orbits=20000)
    Hs = np.array([orc.energy(ic[:, n], 1.0) for n in range(0, 20000, 37)])
    np.testing.assert_allclose(Hs, E, rtol=1e-14)
    for k in (3, 4):
        assert kstest((ic[k] - W[k - 3]) / s, "norm").pvalue > 1e-4
    assert abs((ic[5] > 0).mean() - 0.5) < 0.02
    # a real vz needs Hp(X) <= -sqrt(E) (dvx + dvy) - (dvx^2 + dvy^2)/2, i.e. Hp <~ 0.1 here
    hp = np.array([orc.energy(np.r_[ic[:3, n], 0, 0, 0], 1.0) for n in range(0, 20000, 37)])
    assert np.all(hp <= 0.2) and np.mean(hp) < -0.3


def test_window_velocities_at_eps0(orc):
    """At eps = 0 every window's mean velocity is the constant momentum."""
    ic = orc.ic_box([0] * 6, [2 * np.pi] * 6, 1, 16)
    V = orc.window_velocities("s6", 0.0, H_PAPER, ic, 4, 25)
    for w in range(4):
        np.testing.assert_allclose(V[w], ic[3:], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- 50-digit re-run
def _hp_mp(x, y, z):
    """Eq. 2 as printed, in mpmath."""
    return mpmath.cos(x) * mpmath.cos(y) * (1 + mpmath.cos(2 * z))


def _stages_mp(form, h):
    """The stage list of a form from its definition (section "Computational
    method" and the triple jump of the appendix): S2(t) = D(t/2) K(t) D(t/2);
    S4(t) = S2(g1 t) S2(g0 t) S2(g1 t) with g1 = 1/(2 - 2^(1/3)), g0 = 1 - 2 g1;
    S6(t) = S4(d1 t) S4(d0 t) S4(d1 t) with d1 = 1/(2 - 2^(1/5)), d0 = 1 - 2 d1;
    the standard map K(h) then D(h).  Adjacent drifts are not merged."""
    if form == "stdmap":
        return [("K", h), ("D", h)]
    s2 = lambda t: [("D", t / 2), ("K", t), ("D", t / 2)]  # noqa: E731
    g1 = 1 / (2 - mpmath.cbrt(2))
    s4 = lambda t: s2(g1 * t) + s2((1 - 2 * g1) * t) + s2(g1 * t)  # noqa: E731
    if form == "s4":
        return s4(h)
    d1 = 1 / (2 - mpmath.root(2, 5))
    return s4(d1 * h) + s4((1 - 2 * d1) * h) + s4(d1 * h)


def _map_mp(form, eps, h, T, s):
    """T steps at 50 digits; the force is mpmath's numerical derivative of the
    printed eq. 2 (no hand-derived gradient)."""
    X, P = [mpmath.mpf(v) for v in s[:3]], [mpmath.mpf(v) for v in s[3:]]
    eps = mpmath.mpf(eps)
    stages = _stages_mp(form, mpmath.mpf(h))
    for _ in range(T):
        for kind, t in stages:
            if kind == "D":
                X = [X[i] + t * P[i] for i in range(3)]
            else:
                x, y, z = X
                g = (mpmath.diff(lambda a: _hp_mp(a, y, z), x), mpmath.diff(lambda a: _hp_mp(x, a, z), y),
                     mpmath.diff(lambda a: _hp_mp(x, y, a), z))
                P = [P[i] - t * eps * g[i] for i in range(3)]
    return X + P


@pytest.mark.parametrize("form,eps", [("s6", 1.0), ("s6", 0.05), ("s4", 0.3), ("stdmap", 0.5)])
def test_map_and_ftle_against_a_50_digit_rerun(orc, form, eps):
    """Twenty steps of two random orbits redone at 50 digits from the
    definitions alone: the oracle's binary64 state within 1e-13, and its
    L = ln(|w_T| / |w_0|) within 1e-13 of the 50-digit value, whose tangent is
    the central difference of the 50-digit map (step 1e-20, error ~1e-40), so
    that neither the oracle's stage weights nor its Hessian are reused."""
    mpmath.mp.dps = 50
    try:
        rng = np.random.default_rng(7 + int(eps * 100))
        T = 20
        for _ in range(2):
            s0 = np.concatenate([rng.uniform(0, 2 * np.pi, 3), rng.uniform(-2, 2, 3)])
            w0 = rng.normal(size=6)
            w0 /= np.linalg.norm(w0)
            ref = _map_mp(form, eps, H_PAPER, T, s0)
            got = orc.map_state(form, eps, H_PAPER, T, s0)
            for i in range(6):
                assert abs(got[i] - float(ref[i])) <= 1e-13 * max(1.0, abs(float(ref[i]))), (form, i)
            d = mpmath.mpf("1e-20")
            sp = _map_mp(form, eps, H_PAPER, T, [mpmath.mpf(s0[i]) + d * mpmath.mpf(w0[i]) for i in range(6)])
            sm = _map_mp(form, eps, H_PAPER, T, [mpmath.mpf(s0[i]) - d * mpmath.mpf(w0[i]) for i in range(6)])
            wT = [(sp[i] - sm[i]) / (2 * d) for i in range(6)]
            L_ref = mpmath.log(mpmath.sqrt(mpmath.fsum(v * v for v in wT)) /
                               mpmath.sqrt(mpmath.fsum(mpmath.mpf(v) ** 2 for v in w0)))
            out = orc.ensemble(form, eps, H_PAPER, T, s0.reshape(6, 1), w0.reshape(6, 1))
            assert abs(out[0, 0] - float(L_ref)) <= 1e-13, (form, out[0, 0], float(L_ref))
    finally:
        mpmath.mp.dps = 15


# ---------------------------------------------------------------- random-input properties
def test_reversibility_and_symplecticity_on_random_inputs(orc):
    """Hypothesis draws the initial state, eps, h and the form: every
    symmetric composition satisfies S(-h) S(h) = id, and the 6x6 Jacobian of
    ten steps of every form is symplectic (M^T Omega M = Omega)."""
    from hypothesis import given, settings, strategies as st
    Om = np.block([[np.zeros((3, 3)), np.eye(3)], [-np.eye(3), np.zeros((3, 3))]])

    @settings(max_examples=60, deadline=None, derandomize=True)
    @given(x=st.lists(st.floats(0.0, 2 * np.pi), min_size=3, max_size=3),
           p=st.lists(st.floats(-3.0, 3.0), min_size=3, max_size=3),
           eps=st.floats(0.0, 1.0), h=st.floats(0.005, 0.1),
           form=st.sampled_from(["stdmap", "s2", "s4", "s6", "y6"]))
    def check(x, p, eps, h, form):
        s0 = np.array(x + p)
        T = 10
        if form != "stdmap":
            back = orc.map_state(form, eps, -h, T, orc.map_state(form, eps, h, T, s0))
            assert np.max(np.abs(back - s0)) <= 1e-12 * max(1.0, np.max(np.abs(s0)))
        _, M = orc.jacobian(form, eps, h, T, s0)
        assert np.max(np.abs(M.T @ Om @ M - Om)) <= 1e-10 * max(1.0, np.max(np.abs(M)) ** 2)

    check()
