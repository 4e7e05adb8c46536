"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``aw_oracle.c``: a plain FP64 implementation of the
ensemble propagation of eqs. 1-2 of arXiv:1107.4107 (symplectic map, tangent
vector, per-orbit observables, histograms, forward-mode derivatives of J and
forward-over-forward derivatives of the tangent growth L).  Only the
tests, the package smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the HIP library.

Array convention: structure of arrays, ``ic[6, N]`` = (x, y, z, px, py, pz).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STDMAP, S2, S4, S6, Y6 = 1, 2, 4, 6, 7
FORMS = {"stdmap": STDMAP, "s2": S2, "s4": S4, "s6": S6, "y6": Y6}
OUT_ROWS = ("L", "lambda", "chi", "Vx", "Vy", "Vz", "dP2", "J", "dE")
REC_LEN = 21

CFLAGS = ["-O3", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-shared", "-fPIC", "-Wall", "-Wextra"]
# Build variants.  "default" is portable (it is built here and may run on
# another host); "native" tunes for the host that builds it (the CPU-baseline
# timing builds it on the machine it times); "sanitize" instruments the oracle
# with AddressSanitizer and UndefinedBehaviorSanitizer for the CPU tests.
# Contraction stays off in every variant, so all of them compute bitwise the
# same results.
VARIANT_FLAGS = {
    "default": [],
    "native": ["-march=native"],
    "sanitize": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"],
}
# Set to the path of another build of the oracle to load that one instead.
LIB_ENV = "AW_ORACLE_LIB"


def build(force: bool = True, variant: str = "default", out: str | None = None) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    out = out or _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.run(["gcc", *CFLAGS, *VARIANT_FLAGS[variant], "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, out)
    return out


_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_up = ctypes.POINTER(ctypes.c_uint32)


def use_build(path: str) -> None:
    """Load the oracle from another build of the same source (a build
    variant) for every later call in this process."""
    global _lib
    _lib = open_library(path)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get(LIB_ENV) or _LIB
    if path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = open_library(path)
    _lib = lib
    return lib


def open_library(path: str):
    """Load one build of the oracle and declare its entry points."""
    lib = ctypes.CDLL(path)
    i, l, d, u64 = ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_uint64
    sig = {
        "oracle_rec_init": (None, [_dp, _dp, _dp]),
        "oracle_rec_advance": (i, [i, d, d, l, _dp]),
        "oracle_rec_finish": (None, [_dp, d, d, _dp]),
        "oracle_ensemble": (i, [i, d, d, l, l, _dp, _dp, _dp, _dp, i]),
        "oracle_map": (i, [i, d, d, l, _dp]),
        "oracle_jacobian": (i, [i, d, d, l, _dp, _dp, _dp]),
        "oracle_J_grad": (i, [i, d, d, l, _dp, _dp, _dp]),
        "oracle_J_grad_ensemble": (i, [i, d, d, l, l, _dp, _dp, _dp, i]),
        "oracle_ftle_grad": (i, [i, d, d, l, _dp, _dp, _dp, _dp, _dp]),
        "oracle_ftle_grad_ensemble": (i, [i, d, d, l, l, _dp, _dp, _dp, _dp, i]),
        "oracle_hp_third": (None, [_dp, _dp]),
        "oracle_splitmix64": (u64, [u64, u64]),
        "oracle_u01": (d, [u64, u64]),
        "oracle_ic_grid2": (i, [i, i, d, d, d, d, l, l, _dp, _lp, l, _dp]),
        "oracle_ic_box": (None, [_dp, _dp, u64, _lp, l, _dp]),
        "oracle_ic_sphere": (None, [d, d, d, d, d, d, _dp, _dp, u64, _lp, l, _dp]),
        "oracle_ic_cloud": (None, [d, d, _dp, _dp, _dp, u64, _lp, l, _dp]),
        "oracle_window_velocities": (i, [i, d, d, l, _dp, l, l, _dp, i]),
        "oracle_ensemble_window": (i, [i, d, d, l, l, _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_uint8), _dp, i]),
        "oracle_w0": (None, [u64, _lp, l, _dp]),
        "oracle_hist2d": (l, [l, _dp, _dp, _dp, d, d, d, d, i, i, i, _up, _dp]),
        "oracle_vdir_keys": (None, [l, _dp, _dp, _dp]),
        "oracle_energy": (d, [_dp, d]),
        "oracle_hp_derivs": (None, [_dp, _dp, _dp, _dp]),
        "oracle_tj_constants": (None, [_dp]),
        "oracle_y6_weights": (None, [_dp]),
        "oracle_max_threads": (i, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _idx(idx):
    if idx is None:
        return None, None
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    return idx, idx.ctypes.data_as(_lp)


def _form(form):
    return FORMS[form] if isinstance(form, str) else int(form)


# ---------------------------------------------------------------- generators
def splitmix64(seed: int, counter: int) -> int:
    return int(_load().oracle_splitmix64(seed, counter))


def u01(seed: int, counter: int) -> float:
    return float(_load().oracle_u01(seed, counter))


def ic_grid2(axes, lo, hi, nx, ny, base, idx=None):
    """GRID2 slice: orbit n = j*nx + i; returns ic[6, M]."""
    idx, ip = _idx(idx)
    M = nx * ny if idx is None else len(idx)
    ic = np.empty((6, M))
    b = _f64(base, (6,))
    rc = _load().oracle_ic_grid2(int(axes[0]), int(axes[1]), lo[0], hi[0], lo[1], hi[1],
                                 nx, ny, _ptr(b), ip, M, _ptr(ic))
    if rc:
        raise ValueError("bad GRID2 description")
    return ic


def ic_box(lo, hi, seed, n_orbits=None, idx=None):
    idx, ip = _idx(idx)
    M = n_orbits if idx is None else len(idx)
    ic = np.empty((6, M))
    lo_, hi_ = _f64(lo, (6,)), _f64(hi, (6,))
    _load().oracle_ic_box(_ptr(lo_), _ptr(hi_), seed, ip, M, _ptr(ic))
    return ic


def ic_sphere(E, eps, phi, mu, xlo, xhi, seed, n_orbits=None, idx=None):
    """Fixed-energy initial conditions: X uniform on [xlo, xhi), direction of P
    uniform on the sphere segment phi x mu, |P| = sqrt(2 (E - eps Hp(X)))."""
    idx, ip = _idx(idx)
    M = n_orbits if idx is None else len(idx)
    ic = np.empty((6, M))
    lo_, hi_ = _f64(xlo, (3,)), _f64(xhi, (3,))
    _load().oracle_ic_sphere(E, eps, phi[0], phi[1], mu[0], mu[1], _ptr(lo_), _ptr(hi_), seed, ip, M, _ptr(ic))
    return ic


def ic_cloud(E, eps, cloud, xlo, xhi, seed, n_orbits=None, idx=None):
    """Fig. 4 cloud: Gaussian (vx, vy), X on the torus by rejection, vz from H = E."""
    idx, ip = _idx(idx)
    M = n_orbits if idx is None else len(idx)
    ic = np.empty((6, M))
    _load().oracle_ic_cloud(E, eps, _ptr(_f64(cloud, (4,))), _ptr(_f64(xlo, (3,))), _ptr(_f64(xhi, (3,))), seed, ip,
                            M, _ptr(ic))
    return ic


def window_velocities(form, eps, h, ic, n_windows, window_steps, nthreads=0):
    """Mean velocity of every orbit over consecutive windows: V[n_windows, 3, N]."""
    ic = _f64(ic)
    N = ic.shape[1]
    V = np.empty((n_windows, 3, N))
    if _load().oracle_window_velocities(_form(form), eps, h, N, _ptr(ic), int(n_windows), int(window_steps), _ptr(V),
                                        int(nthreads)):
        raise ValueError("oracle_window_velocities rejected its arguments")
    return V


def ensemble_window(form, eps, h, T, ic, w0_, window, nthreads=0):
    """oracle ensemble plus the stay-in-window test; returns (out, left, margin)."""
    ic = _f64(ic)
    w = _f64(w0_)
    N = ic.shape[1]
    out = np.empty((9, N))
    left = np.empty(N, dtype=np.uint8)
    margin = np.empty(N)
    win = _f64(window, (4,))
    rc = _load().oracle_ensemble_window(_form(form), eps, h, int(T), N, _ptr(ic), _ptr(w), _ptr(win), _ptr(out),
                                        left.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _ptr(margin),
                                        int(nthreads))
    if rc:
        raise ValueError("oracle_ensemble_window rejected its arguments")
    return out, left, margin


def w0(seed, n_orbits=None, idx=None):
    idx, ip = _idx(idx)
    M = n_orbits if idx is None else len(idx)
    w = np.empty((6, M))
    _load().oracle_w0(seed, ip, M, _ptr(w))
    return w


# ---------------------------------------------------------------- propagation
def ensemble(form, eps, h, T, ic, w0_, want_state=False, nthreads=0):
    """Run every orbit of ic[6, N]; returns out[9, N] (and state[12, N])."""
    ic = _f64(ic)
    w = _f64(w0_)
    N = ic.shape[1]
    out = np.empty((9, N))
    st = np.empty((12, N)) if want_state else None
    rc = _load().oracle_ensemble(_form(form), eps, h, int(T), N, _ptr(ic), _ptr(w), _ptr(out),
                                 _ptr(st) if st is not None else None, int(nthreads))
    if rc:
        raise ValueError("oracle_ensemble rejected its arguments")
    return (out, st) if want_state else out


def map_state(form, eps, h, T, s):
    s = _f64(s, (6,)).copy()
    if _load().oracle_map(_form(form), eps, h, int(T), _ptr(s)):
        raise ValueError("bad map form")
    return s


def jacobian(form, eps, h, T, s0):
    s0 = _f64(s0, (6,))
    sT = np.empty(6)
    M = np.empty(36)
    if _load().oracle_jacobian(_form(form), eps, h, int(T), _ptr(s0), _ptr(sT), _ptr(M)):
        raise ValueError("bad map form")
    return sT, M.reshape(6, 6)


def J_grad(form, eps, h, T, s0):
    """Returns (J, dJ[7]) with dJ = d/d(x,y,z,px,py,pz,eps)."""
    s0 = _f64(s0, (6,))
    J = ctypes.c_double()
    dJ = np.empty(7)
    if _load().oracle_J_grad(_form(form), eps, h, int(T), _ptr(s0), ctypes.byref(J), _ptr(dJ)):
        raise ValueError("bad map form")
    return J.value, dJ


def J_grad_ensemble(form, eps, h, T, ic, nthreads=0):
    """Forward-mode J and dJ[7, N] (d/d x..pz, eps) for every orbit of ic[6, N]."""
    ic = _f64(ic)
    N = ic.shape[1]
    J = np.empty(N)
    dJ = np.empty((7, N))
    if _load().oracle_J_grad_ensemble(_form(form), eps, h, int(T), N, _ptr(ic), _ptr(J), _ptr(dJ), int(nthreads)):
        raise ValueError("bad map form")
    return J, dJ


def ftle_grad(form, eps, h, T, s0, w0_):
    """Returns (L, dL[7], final state and unit tangent [12]) with
    dL = d/d(x, y, z, px, py, pz, eps) of L = ln(|w_T| / |w_0|) at fixed w0."""
    s0 = _f64(s0, (6,))
    w = _f64(w0_, (6,))
    L = ctypes.c_double()
    dL = np.empty(7)
    sT = np.empty(12)
    if _load().oracle_ftle_grad(_form(form), eps, h, int(T), _ptr(s0), _ptr(w), ctypes.byref(L), _ptr(dL), _ptr(sT)):
        raise ValueError("bad map form")
    return L.value, dL, sT


def ftle_grad_ensemble(form, eps, h, T, ic, w0_, nthreads=0):
    """Forward-over-forward L[N] and dL[7, N] for every orbit of ic[6, N] with
    tangent starts w0[6, N]."""
    ic = _f64(ic)
    w = _f64(w0_)
    N = ic.shape[1]
    L = np.empty(N)
    dL = np.empty((7, N))
    if _load().oracle_ftle_grad_ensemble(_form(form), eps, h, int(T), N, _ptr(ic), _ptr(w), _ptr(L), _ptr(dL),
                                         int(nthreads)):
        raise ValueError("bad map form")
    return L, dL


def rec_init(s0, w0_):
    rec = np.empty(REC_LEN)
    _load().oracle_rec_init(_ptr(_f64(s0, (6,))), _ptr(_f64(w0_, (6,))), _ptr(rec))
    return rec


def rec_advance(form, eps, h, nsteps, rec):
    if _load().oracle_rec_advance(_form(form), eps, h, int(nsteps), _ptr(rec)):
        raise ValueError("bad map form")
    return rec


def rec_finish(rec, eps, h):
    out = np.empty(9)
    _load().oracle_rec_finish(_ptr(rec), eps, h, _ptr(out))
    return out


# ---------------------------------------------------------------- images
def hist2d(a, b, v, lo, hi, W, H, closed_upper=False):
    """Serial histogram in orbit order; returns (counts[H, W] u32, sums[H, W], dropped)."""
    a, b, v = _f64(a), _f64(b), _f64(v)
    counts = np.empty((H, W), dtype=np.uint32)
    sums = np.empty((H, W))
    dropped = _load().oracle_hist2d(len(a), _ptr(a), _ptr(b), _ptr(v), lo[0], hi[0], lo[1], hi[1],
                                    W, H, int(bool(closed_upper)),
                                    counts.ctypes.data_as(_up), _ptr(sums))
    return counts, sums, int(dropped)


def vdir_keys(V):
    V = _f64(V)
    N = V.shape[1]
    phi, mu = np.empty(N), np.empty(N)
    _load().oracle_vdir_keys(N, _ptr(V), _ptr(phi), _ptr(mu))
    return phi, mu


def hist_p0(ic, values, key_axes, lo, hi, W, H):
    """Image keyed on two initial coordinates; returns (mean[H, W], counts, dropped)."""
    counts, sums, dropped = hist2d(ic[key_axes[0]], ic[key_axes[1]], values, lo, hi, W, H)
    mean = np.where(counts > 0, sums / np.maximum(counts, 1), 0.0)
    return mean, counts, dropped


def hist_vdir(V, W, H, n_total=None):
    """Equal-area density of the direction of V; returns (density[H, W], counts, dropped)."""
    phi, mu = vdir_keys(V)
    counts, _, dropped = hist2d(phi, mu, np.zeros(len(phi)), (-np.pi, -1.0), (np.pi, 1.0), W, H,
                                closed_upper=True)
    n = V.shape[1] if n_total is None else n_total
    dphi, dmu = 2.0 * np.pi / W, 2.0 / H
    dens = counts / (n * dphi * dmu)
    return dens, counts, dropped


# ---------------------------------------------------------------- accessors
def energy(s, eps):
    return float(_load().oracle_energy(_ptr(_f64(s, (6,))), eps))


def hp_derivs(X):
    X = _f64(X, (3,))
    hp = ctypes.c_double()
    g = np.empty(3)
    H6 = np.empty(6)
    _load().oracle_hp_derivs(_ptr(X), ctypes.byref(hp), _ptr(g), _ptr(H6))
    return hp.value, g, H6


def hp_third(X):
    """Third derivatives of Hp at X as a [3, 3, 3] array."""
    X = _f64(X, (3,))
    t = np.empty(27)
    _load().oracle_hp_third(_ptr(X), _ptr(t))
    return t.reshape(3, 3, 3)


def tj_constants():
    c = np.empty(4)
    _load().oracle_tj_constants(_ptr(c))
    return c


def y6_weights():
    """(w0, w1, w2, w3) of the 7-stage 6th-order composition, solved by the oracle."""
    w = np.empty(4)
    _load().oracle_y6_weights(_ptr(w))
    return w


def max_threads():
    return int(_load().oracle_max_threads())
