"""Synthetic workloads: the ensembles the tests and the benchmark run.

Only parameters and seeded draws live here; nothing of the method's
arithmetic.  All runs use M = 3, FP64, h = 0.01 * 2 pi (section "Computational
method") and the 6th-order map unless stated.

  c1  eps = 1e-2, 64 x 64 slice of (px, py) in [0, 2 pi)^2 (left edges), other
      coordinates 0, T = 1000, tangent start seed 0: the indicator image.
  c2  as c1 with eps = 1e-3, 1024 x 1024, T = 1e5: indicator image and the
      regular/chaotic class map at chi > 2.
  c3  64 ensembles in one persistent launch: eps_k = 10^(-4 + 3k/63), grid
      size per ensemble drawn from {128, 256, 512, 1024}^2 and T from
      {1e4, 3e4, 1e5} with numpy's default_rng(1).
  c4  gradients: eps = 1e-2, 512 x 512 slice, T = 1e4, checkpoint every 100
      steps; 256 orbits drawn with default_rng(3) among the regular ones.
  c5  1e7 orbits uniform on [0, 2 pi)^6 (SplitMix64 seed 2), eps = 5e-3 (the
      paper's weak-regime eps_eff = 2/400), T = 1e6; momentum drift
      |P_T - P_0|^2 averaged on a 512 x 512 image keyed on (px0, py0), and the
      density of the direction of V on the sphere.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from . import Ensemble, ImageSpec, OUT_CHI, OUT_DP2

TWO_PI = 2.0 * math.pi


def slice_ensemble(eps: float, n: int, T: int, map_form: str = "s6", pz0: float = 0.0,
                   tangent: bool = True) -> Ensemble:
    """The (px, py) slice of the configs, x = y = z = 0, pz = pz0."""
    return Ensemble(eps=eps, n_steps=T, map_form=map_form, ic_kind="grid2", axis=(3, 4),
                    lo=(0.0, 0.0), hi=(TWO_PI, TWO_PI), nx=n, ny=n,
                    base=(0.0, 0.0, 0.0, 0.0, 0.0, pz0), seed_tangent=0, chi_threshold=2.0,
                    tangent=tangent)


def c1(map_form: str = "s6") -> Ensemble:
    return slice_ensemble(1e-2, 64, 1000, map_form)


def c2() -> Ensemble:
    return slice_ensemble(1e-3, 1024, 100_000)


def c3_draw():
    """(eps, grid side, T) of the 64 batched ensembles."""
    rng = np.random.default_rng(1)
    G = rng.choice([128, 256, 512, 1024], 64)
    T = rng.choice([10_000, 30_000, 100_000], 64)
    eps = [10.0 ** (-4.0 + 3.0 * k / 63.0) for k in range(64)]
    return [(eps[k], int(G[k]), int(T[k])) for k in range(64)]


def c3(t_scale: float = 1.0) -> List[Ensemble]:
    return [slice_ensemble(e, g, max(1, int(round(t * t_scale)))) for e, g, t in c3_draw()]


def eps_sweep(n: int = 256, T: int = 30_000, n_eps: int = 16, pz0: float = 0.0) -> List[Ensemble]:
    """Chaotic fraction against eps (the model section: the web volume scales
    as sqrt(eps) and thickens as eps grows): eps log-spaced over 1e-4..1e-1 at
    one grid size and horizon, on the literal slice (pz0 = 0) or its pz0 = 1
    companion."""
    return [slice_ensemble(10.0 ** (-4.0 + 3.0 * k / (n_eps - 1)), n, T, pz0=pz0) for k in range(n_eps)]


def c4() -> Ensemble:
    return slice_ensemble(1e-2, 512, 10_000, tangent=False)


C4_CKPT = 100


def c4_pick(chi: np.ndarray, n_pick: int = 256, seed: int = 3) -> np.ndarray:
    """Indices of n_pick orbits drawn without replacement among those with chi < 1.5."""
    reg = np.flatnonzero(chi < 1.5)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(reg, size=min(n_pick, reg.size), replace=False))


def c5(n_orbits: int = 10_000_000, T: int = 1_000_000) -> Ensemble:
    return Ensemble(eps=5e-3, n_steps=T, ic_kind="box", box_lo=(0.0,) * 6, box_hi=(TWO_PI,) * 6,
                    n_orbits=n_orbits, seed_ic=2, seed_tangent=0, chi_threshold=2.0)


def c5_p0_image() -> ImageSpec:
    return ImageSpec(kind="hist_p0", field=OUT_DP2, W=512, H=512, key_axis=(3, 4), lo=(0.0, 0.0),
                     hi=(TWO_PI, TWO_PI))


def c5_vdir_image() -> ImageSpec:
    return ImageSpec(kind="hist_vdir", W=512, H=512)


def chi_image(n: int) -> ImageSpec:
    return ImageSpec(kind="ic_grid", field=OUT_CHI, W=n, H=n)


# ---------------------------------------------------------------------------
# The paper's own geometry (section "Main results", Figs. 2-3): eps = 1, the
# direction of P uniform on the momentum sphere at fixed energy E, X uniform on
# the torus [0, 2 pi)^3, averaging time Delta t = 50 T = 5000 steps.

FIG2_E = 400.0      # eps_eff = 2/E = 0.005, the weak regime (Fig. 2)
FIG3_E = 15.0       # eps_eff = 2/15, moderate perturbation (Fig. 3)
DT50 = 5000         # Delta t = 50 T with T = 2 pi, h = T/100


def sphere_ensemble(E: float, n_orbits: int, T: int = DT50, window=(-math.pi, math.pi, -1.0, 1.0),
                    stay_in_window: bool = False, tangent: bool = False, seed: int = 4) -> Ensemble:
    return Ensemble(eps=1.0, n_steps=T, ic_kind="sphere", n_orbits=n_orbits, energy=E, window=tuple(window),
                    box_lo=(0.0,) * 6, box_hi=(TWO_PI,) * 6, seed_ic=seed, seed_tangent=0,
                    stay_in_window=stay_in_window, tangent=tangent)


def fig2(n_orbits: int = 100_000_000, T: int = DT50) -> Ensemble:
    """Fig. 2: E = 400, the whole sphere, N ~ 1e8, Delta t = 50 T."""
    return sphere_ensemble(FIG2_E, n_orbits, T)


def fig3_zoom(n_orbits: int = 4_000_000, T: int = DT50) -> Ensemble:
    """Fig. 3 (b, c) style zoom: E = 15, a segment of the sphere, keeping only
    the orbits whose momentum stays inside it."""
    return sphere_ensemble(FIG3_E, n_orbits, T, window=(0.55, 1.05, -0.25, 0.25), stay_in_window=True)


def sphere_image(W: int = 1024, H: int = 512, window=None) -> ImageSpec:
    if window is None:
        return ImageSpec(kind="hist_vdir", W=W, H=H)
    return ImageSpec(kind="hist_vdir", W=W, H=H, lo=(window[0], window[2]), hi=(window[1], window[3]))


def fig4_cloud(n_orbits: int = 32_000, T: int = 1_000_000_000) -> Ensemble:
    """Fig. 4: N = 3.2e4 orbits injected at W = (sqrt E, sqrt E, 0), E = 15,
    Gaussian in (vx, vy) with sigma = 0.01, X on the torus, vz from H = E; the
    paper propagates them to t_p = 1e7 T (1e9 steps) and averages F over the
    windows between plots."""
    w = math.sqrt(FIG3_E)
    return Ensemble(eps=1.0, n_steps=T, ic_kind="cloud", n_orbits=n_orbits, energy=FIG3_E,
                    cloud=(w, w, 0.01, 0.01), box_lo=(0.0,) * 6, box_hi=(TWO_PI,) * 6, seed_ic=6, tangent=False)
