"""MI355X ensemble mapper for the Arnold web of arXiv:1107.4107.

Python binding of libaw (include/aw.h): argument marshalling only.  Device
memory and streams come from PyTorch; every step of the computation runs in
the HIP kernels of the library.  There is no CPU fallback: if libaw.so is not
built, or no GPU is present, calls raise.

Model (eqs. 1-2): H = |P|^2/2 + eps cos x cos y (1 + cos 2z), stepped by the
6th-order triple-jump composition (default) or the coupled standard map.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _abi
from ._abi import (AwError, F_TANGENT, F_WINDOW, IC_BOX, IC_EXPLICIT, IC_GRID2, IC_SPHERE, IMG_HIST_P0, IMG_HIST_VDIR,
                   IMG_IC_GRID, MAP_S2, MAP_S4, MAP_S6, MAP_STDMAP, MAP_Y6, NCARRY, NOUT, OUT_CHI, OUT_DE,
                   OUT_DP2, OUT_J, OUT_L, OUT_LAMBDA, OUT_VX, OUT_VY, OUT_VZ)

H_PAPER = 0.01 * 2.0 * math.pi  # h = 10^-2 T, T = 2 pi (section "Computational method")
FORMS = {"stdmap": MAP_STDMAP, "s2": MAP_S2, "s4": MAP_S4, "s6": MAP_S6, "y6": MAP_Y6}
OUT_ROWS = ("L", "lambda", "chi", "Vx", "Vy", "Vz", "dP2", "J", "dE")

__all__ = [
    "Ensemble", "Tuning", "ImageSpec", "map_ensemble", "map_ensembles", "map_ensemble_steps",
    "indicator_image", "indicator_images", "histogram2d", "vdir_keys", "generate_ic", "image_workspace_bytes",
    "reserve",
    "indicator_grad", "IndicatorJ", "ftle_grad_workspace_bytes", "ftle_grad", "IndicatorL", "Graph", "timing_enable", "timing_read", "step_op_counts",
    "AwError", "H_PAPER", "OUT_ROWS",
]


def _lib():
    return _abi.load()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t: torch.Tensor, shape=None, name="tensor") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _p(t: Optional[torch.Tensor]):
    return t.data_ptr() if t is not None else None


@dataclass
class Ensemble:
    """Descriptor of one ensemble (aw_ensemble)."""
    eps: float
    n_steps: int
    h: float = H_PAPER
    map_form: str = "s6"
    ic_kind: str = "grid2"              # "grid2" | "box" | "explicit" | "sphere"
    axis: Sequence[int] = (3, 4)        # GRID2: varied coordinates (px, py by default)
    lo: Sequence[float] = (0.0, 0.0)
    hi: Sequence[float] = (2 * math.pi, 2 * math.pi)
    nx: int = 64
    ny: int = 64
    base: Sequence[float] = (0.0,) * 6
    box_lo: Sequence[float] = (0.0,) * 6
    box_hi: Sequence[float] = (2 * math.pi,) * 6
    n_orbits: int = 0
    seed_ic: int = 0
    seed_tangent: int = 0
    chi_threshold: float = 2.0
    tangent: bool = True
    M: int = 3
    energy: float = 0.0                 # sphere: total energy E (eq. 1)
    window: Sequence[float] = (-math.pi, math.pi, -1.0, 1.0)   # phi_lo, phi_hi, mu_lo, mu_hi
    stay_in_window: bool = False        # the "remained within the area" test
    cloud: Sequence[float] = (0.0, 0.0, 0.0, 0.0)   # cloud: centre (vx, vy), sigma (x, y)

    def to_c(self) -> _abi.AwEnsemble:
        e = _abi.AwEnsemble()
        e.M = self.M
        e.map_form = FORMS[self.map_form] if isinstance(self.map_form, str) else int(self.map_form)
        e.eps = float(self.eps)
        e.h = float(self.h)
        e.n_steps = int(self.n_steps)
        e.ic_kind = {"grid2": IC_GRID2, "box": IC_BOX, "explicit": IC_EXPLICIT, "sphere": IC_SPHERE,
                     "cloud": _abi.IC_CLOUD}[self.ic_kind]
        e.axis[:] = [int(a) for a in self.axis]
        e.lo[:] = [float(v) for v in self.lo]
        e.hi[:] = [float(v) for v in self.hi]
        e.nx, e.ny = int(self.nx), int(self.ny)
        e.base[:] = [float(v) for v in self.base]
        e.box_lo[:] = [float(v) for v in self.box_lo]
        e.box_hi[:] = [float(v) for v in self.box_hi]
        e.n_orbits = int(self.n_orbits)
        e.seed_ic = int(self.seed_ic) & 0xFFFFFFFFFFFFFFFF
        e.seed_tangent = int(self.seed_tangent) & 0xFFFFFFFFFFFFFFFF
        e.chi_threshold = float(self.chi_threshold)
        e.flags = (F_TANGENT if self.tangent else 0) | (F_WINDOW if self.stay_in_window else 0)
        e.energy = float(self.energy)
        e.window[:] = [float(v) for v in self.window]
        e.cloud[:] = [float(v) for v in self.cloud]
        return e

    @property
    def size(self) -> int:
        n = int(_lib().aw_ensemble_size(ctypes.byref(self.to_c())))
        if n < 0:
            raise ValueError("invalid ensemble size")
        return n


@dataclass
class Tuning:
    """Launch shape (aw_tuning); zeros mean library defaults (block 0: chosen
    from the ensemble size, 512 for large ensembles)."""
    block: int = 0
    orbits_per_lane: int = 1
    unroll: int = 1
    renorm_every: int = 8
    persistent_wgs: int = 0
    lanes_per_orbit: int = 0

    def to_c(self) -> _abi.AwTuning:
        return _abi.AwTuning(self.block, self.orbits_per_lane, self.unroll, self.renorm_every,
                             self.persistent_wgs, self.lanes_per_orbit)


@dataclass
class ImageSpec:
    kind: str = "ic_grid"               # "ic_grid" | "hist_p0" | "hist_vdir"
    field: int = OUT_CHI
    W: int = 64
    H: int = 64
    key_axis: Sequence[int] = (3, 4)
    lo: Optional[Sequence[float]] = None   # hist_p0: key ranges (default [0, 2 pi)^2);
    hi: Optional[Sequence[float]] = None   # hist_vdir: (phi, mu) zoom (default: whole sphere)

    def to_c(self) -> _abi.AwImageSpec:
        s = _abi.AwImageSpec()
        s.kind = {"ic_grid": IMG_IC_GRID, "hist_p0": IMG_HIST_P0, "hist_vdir": IMG_HIST_VDIR}[self.kind]
        s.field = int(self.field)
        s.W, s.H = int(self.W), int(self.H)
        s.key_axis[:] = [int(a) for a in self.key_axis]
        if self.lo is None or self.hi is None:
            lo, hi = ((0.0, 0.0), (2 * math.pi, 2 * math.pi)) if self.kind == "hist_p0" else ((0.0, 0.0), (0.0, 0.0))
        else:
            lo, hi = self.lo, self.hi
        s.lo[:] = [float(v) for v in lo]
        s.hi[:] = [float(v) for v in hi]
        return s


def _tuning_ptr(tuning: Optional[Tuning]):
    return ctypes.byref(tuning.to_c()) if tuning is not None else None


def _device():
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the ensemble mapper runs on the GPU only")
    return torch.device("cuda", torch.cuda.current_device())


@dataclass
class MapResult:
    orbit_out: torch.Tensor                       # [9, N] float64
    state: Optional[torch.Tensor] = None          # [12, N] float64
    cls: Optional[torch.Tensor] = None            # [N] uint8


def map_ensembles(ens: List[Ensemble], ic: Optional[List[Optional[torch.Tensor]]] = None,
                  want_state: bool = False, want_class: bool = True,
                  tuning: Optional[Tuning] = None) -> List[MapResult]:
    """Propagate one or more ensembles (more than one: one persistent launch)."""
    dev = _device()
    n = len(ens)
    c_ens = (_abi.AwEnsemble * n)(*[e.to_c() for e in ens])
    sizes = [e.size for e in ens]
    outs = [torch.empty((NOUT, N), dtype=torch.float64, device=dev) for N in sizes]
    states = [torch.empty((12, N), dtype=torch.float64, device=dev) for N in sizes] if want_state else None
    clss = [torch.empty((N,), dtype=torch.uint8, device=dev) for N in sizes] if want_class else None
    ic_ptrs = None
    if ic is not None:
        for k, t in enumerate(ic):
            if t is not None:
                _dev_f64(t, (6, sizes[k]), "ic")
        ic_ptrs = _abi.ptr_array([_p(t) for t in ic])
    _abi.check(_lib().aw_map_ensemble(
        c_ens, n, ic_ptrs, _abi.ptr_array([_p(t) for t in outs]),
        _abi.ptr_array([_p(t) for t in states]) if states else None,
        _abi.ptr_array([_p(t) for t in clss]) if clss else None,
        _tuning_ptr(tuning), _stream()))
    return [MapResult(outs[k], states[k] if states else None, clss[k] if clss else None) for k in range(n)]


def map_ensemble(ens: Ensemble, ic: Optional[torch.Tensor] = None, want_state: bool = False,
                 want_class: bool = True, tuning: Optional[Tuning] = None) -> MapResult:
    return map_ensembles([ens], [ic] if ic is not None else None, want_state, want_class, tuning)[0]


def map_ensemble_steps(ens: Ensemble, carry: torch.Tensor, k_begin: int, k_end: int,
                       ic: Optional[torch.Tensor] = None, orbit_out: Optional[torch.Tensor] = None,
                       state: Optional[torch.Tensor] = None, cls: Optional[torch.Tensor] = None,
                       tuning: Optional[Tuning] = None) -> None:
    """Run global steps [k_begin, k_end) with the state carried in carry[21, N]."""
    N = ens.size
    _dev_f64(carry, (NCARRY, N), "carry")
    if orbit_out is not None:
        _dev_f64(orbit_out, (NOUT, N), "orbit_out")
    if state is not None:
        _dev_f64(state, (12, N), "state")
    if ic is not None:
        _dev_f64(ic, (6, N), "ic")
    if cls is not None and (cls.dtype != torch.uint8 or cls.numel() != N or cls.device.type != "cuda"):
        raise ValueError("cls must be a uint8 CUDA tensor of N elements")
    _abi.check(_lib().aw_map_ensemble_steps(
        ctypes.byref(ens.to_c()), _p(ic), _p(carry), int(k_begin), int(k_end), _p(orbit_out),
        _p(state), _p(cls), _tuning_ptr(tuning), _stream()))


def indicator_images(ens: List[Ensemble], spec: ImageSpec, want_counts: bool = True,
                     want_class: bool = False, tuning: Optional[Tuning] = None):
    """Propagate and reduce to images.  Returns (images, counts, classes) lists."""
    dev = _device()
    n = len(ens)
    c_ens = (_abi.AwEnsemble * n)(*[e.to_c() for e in ens])
    sizes = [e.size for e in ens]
    if spec.kind == "ic_grid" and spec.W == 0 and spec.H == 0:   # each ensemble's own grid
        imgs = [torch.empty((e.ny, e.nx), dtype=torch.float64, device=dev) for e in ens]
    else:
        imgs = [torch.empty((spec.H, spec.W), dtype=torch.float64, device=dev) for _ in ens]
    if want_counts:
        shape = (1,) if spec.kind == "ic_grid" else (spec.H, spec.W)
        cnts = [torch.empty(shape, dtype=torch.int32, device=dev) for _ in ens]  # uint32 bits
    else:
        cnts = None
    clss = [torch.empty((N,), dtype=torch.uint8, device=dev) for N in sizes] if want_class else None
    _abi.check(_lib().aw_indicator_image(
        c_ens, n, ctypes.byref(spec.to_c()), _abi.ptr_array([_p(t) for t in imgs]),
        _abi.ptr_array([_p(t) for t in cnts]) if cnts else None,
        _abi.ptr_array([_p(t) for t in clss]) if clss else None, _tuning_ptr(tuning), _stream()))
    return imgs, cnts, clss


def indicator_image(ens: Ensemble, spec: ImageSpec, want_counts: bool = True, want_class: bool = False,
                    tuning: Optional[Tuning] = None):
    imgs, cnts, clss = indicator_images([ens], spec, want_counts, want_class, tuning)
    return imgs[0], (cnts[0] if cnts else None), (clss[0] if clss else None)


def window_density(ens: Ensemble, carry: torch.Tensor, k_begin: int, n_windows: int, window_steps: int,
                   spec: ImageSpec, counts: torch.Tensor, ic: Optional[torch.Tensor] = None,
                   tuning: Optional[Tuning] = None) -> None:
    """Add the direction counts of V over n_windows consecutive windows to
    counts[H, W] (int32 holding uint32); the state is carried in carry[22, N]."""
    N = ens.size
    _dev_f64(carry, (NCARRY, N), "carry")
    if counts.dtype != torch.int32 or tuple(counts.shape) != (spec.H, spec.W) or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous int32 [H, W] tensor")
    if ic is not None:
        _dev_f64(ic, (6, N), "ic")
    _abi.check(_lib().aw_window_density(ctypes.byref(ens.to_c()), _p(ic), _p(carry), int(k_begin), int(n_windows),
                                        int(window_steps), ctypes.byref(spec.to_c()), _p(counts),
                                        _tuning_ptr(tuning), _stream()))


def histogram2d(a: torch.Tensor, b: torch.Tensor, v: Optional[torch.Tensor], lo, hi, W: int, H: int,
                closed_upper: bool = False, noalloc: bool = False):
    """Counts[H, W] (int32 holding uint32), sums[H, W] (or None) and the dropped count.
    noalloc=True calls aw_histogram2d_noalloc (scratch in the library's fixed
    device array; the outputs are still allocated here)."""
    N = a.numel()
    _dev_f64(a, (N,), "a")
    _dev_f64(b, (N,), "b")
    if v is not None:
        _dev_f64(v, (N,), "v")
    counts = torch.empty((H, W), dtype=torch.int32, device=a.device)
    sums = torch.empty((H, W), dtype=torch.float64, device=a.device) if v is not None else None
    dropped = torch.empty((1,), dtype=torch.int64, device=a.device)
    fn = _lib().aw_histogram2d_noalloc if noalloc else _lib().aw_histogram2d
    _abi.check(fn(N, _p(a), _p(b), _p(v), float(lo[0]), float(hi[0]), float(lo[1]), float(hi[1]), int(W), int(H),
                  int(bool(closed_upper)), _p(counts), _p(sums), _p(dropped), _stream()))
    return counts, sums, dropped


def vdir_keys(V: torch.Tensor):
    N = V.shape[1]
    _dev_f64(V, (3, N), "V")
    phi = torch.empty((N,), dtype=torch.float64, device=V.device)
    mu = torch.empty((N,), dtype=torch.float64, device=V.device)
    _abi.check(_lib().aw_vdir_keys(N, _p(V), _p(phi), _p(mu), _stream()))
    return phi, mu


def image_workspace_bytes(ens: List[Ensemble], spec: Optional[ImageSpec]) -> int:
    """Library scratch one indicator_images (spec None: map_ensembles) call over
    these ensembles takes on its stream."""
    n = len(ens)
    c_ens = (_abi.AwEnsemble * n)(*[e.to_c() for e in ens])
    nb = ctypes.c_size_t()
    _abi.check(_lib().aw_image_workspace(c_ens, n, ctypes.byref(spec.to_c()) if spec is not None else None,
                                         ctypes.byref(nb)))
    return int(nb.value)


def reserve(nbytes: int) -> None:
    """Grow the current stream's library scratch to at least nbytes now."""
    _abi.check(_lib().aw_reserve(int(nbytes), _stream()))


def generate_ic(ens: Ensemble, ic_in: Optional[torch.Tensor] = None):
    """The exact initial state ic[6, N] and tangent start w0[6, N] of an ensemble."""
    dev = _device()
    N = ens.size
    ic = torch.empty((6, N), dtype=torch.float64, device=dev)
    w0 = torch.empty((6, N), dtype=torch.float64, device=dev)
    _abi.check(_lib().aw_generate_ic(ctypes.byref(ens.to_c()), _p(ic_in), _p(ic), _p(w0), _stream()))
    return ic, w0


def grad_workspace_bytes(ens: Ensemble, ckpt_every: int, reversible: bool = False) -> int:
    nb = ctypes.c_size_t()
    fn = _lib().aw_indicator_grad_reversible_workspace if reversible else _lib().aw_indicator_grad_workspace
    _abi.check(fn(ctypes.byref(ens.to_c()), int(ckpt_every), ctypes.byref(nb)))
    return int(nb.value)


def indicator_grad(ens: Ensemble, ic: torch.Tensor, grad_J: Optional[torch.Tensor] = None,
                   ckpt_every: int = 100, tuning: Optional[Tuning] = None,
                   workspace: Optional[torch.Tensor] = None, reversible: bool = False):
    """Adjoint gradient of J.  Returns (J[N], grad_ic[6, N], grad_eps[N]).
    reversible=True sweeps each segment back by inverting the steps instead
    of recomputing and storing them (aw_indicator_grad_reversible)."""
    if ens.ic_kind != "explicit":
        raise ValueError("indicator_grad needs an explicit ensemble")
    N = ens.size
    _dev_f64(ic, (6, N), "ic")
    if grad_J is not None:
        _dev_f64(grad_J, (N,), "grad_J")
    nb = grad_workspace_bytes(ens, ckpt_every, reversible)
    if workspace is None or workspace.numel() * workspace.element_size() < nb:
        workspace = torch.empty((max(nb, 8),), dtype=torch.uint8, device=ic.device)
    J = torch.empty((N,), dtype=torch.float64, device=ic.device)
    gic = torch.empty((6, N), dtype=torch.float64, device=ic.device)
    geps = torch.empty((N,), dtype=torch.float64, device=ic.device)
    fn = _lib().aw_indicator_grad_reversible if reversible else _lib().aw_indicator_grad
    _abi.check(fn(ctypes.byref(ens.to_c()), _p(ic), _p(grad_J), int(ckpt_every), _p(J), _p(gic), _p(geps),
                  _p(workspace), workspace.numel() * workspace.element_size(), _tuning_ptr(tuning), _stream()))
    return J, gic, geps


class IndicatorJ(torch.autograd.Function):
    """J_n = (1/T) sum_k |P_k - P_0|^2 per orbit, differentiable in the initial
    state ic[N, 6] and in eps (a 0-d float64 tensor); the backward pass runs the
    checkpointed adjoint kernels (reversible=True: the store-free sweep)."""

    @staticmethod
    def forward(ctx, ic, eps, n_steps: int, h: float = H_PAPER, map_form: str = "s6", ckpt_every: int = 100,
                reversible: bool = False):
        if ic.dim() != 2 or ic.shape[1] != 6:
            raise ValueError("ic must be [N, 6]")
        soa = ic.detach().t().contiguous()
        e = Ensemble(eps=float(eps), n_steps=n_steps, h=h, map_form=map_form, ic_kind="explicit",
                     n_orbits=ic.shape[0], tangent=False)
        res = map_ensemble(e, soa, want_class=False)
        ctx.save_for_backward(soa)
        ctx.ens = e
        ctx.ckpt = ckpt_every
        ctx.reversible = reversible
        ctx.eps_shape = eps.shape if isinstance(eps, torch.Tensor) else None
        return res.orbit_out[OUT_J].clone()

    @staticmethod
    def backward(ctx, gJ):
        (soa,) = ctx.saved_tensors
        _, gic, geps = indicator_grad(ctx.ens, soa, gJ.contiguous().to(torch.float64), ctx.ckpt,
                                      reversible=ctx.reversible)
        g_eps = geps.sum()
        if ctx.eps_shape is not None:
            g_eps = g_eps.reshape(ctx.eps_shape)
        return gic.t().contiguous(), g_eps, None, None, None, None, None


def ftle_grad_workspace_bytes(ens: Ensemble, ckpt_every: int, reversible: bool = False) -> int:
    nb = ctypes.c_size_t()
    fn = _lib().aw_ftle_grad_reversible_workspace if reversible else _lib().aw_ftle_grad_workspace
    _abi.check(fn(ctypes.byref(ens.to_c()), int(ckpt_every), ctypes.byref(nb)))
    return int(nb.value)


def ftle_grad(ens: Ensemble, ic: torch.Tensor, w0: Optional[torch.Tensor] = None,
              grad_L: Optional[torch.Tensor] = None, ckpt_every: int = 100, tuning: Optional[Tuning] = None,
              workspace: Optional[torch.Tensor] = None, reversible: bool = False):
    """Second-order adjoint gradient of the tangent growth L = ln(|w_T|/|w_0|).
    w0 defaults to the ensemble's seeded tangent start (the one map_ensemble
    uses).  reversible=True sweeps each segment back by inverting the steps
    (aw_ftle_grad_reversible).  Returns (L[N], grad_ic[6, N], grad_eps[N])."""
    if ens.ic_kind != "explicit":
        raise ValueError("ftle_grad needs an explicit ensemble")
    N = ens.size
    _dev_f64(ic, (6, N), "ic")
    if w0 is None:
        _, w0 = generate_ic(ens, ic)
    _dev_f64(w0, (6, N), "w0")
    if grad_L is not None:
        _dev_f64(grad_L, (N,), "grad_L")
    nb = ftle_grad_workspace_bytes(ens, ckpt_every, reversible)
    if workspace is None or workspace.numel() * workspace.element_size() < nb:
        workspace = torch.empty((max(nb, 8),), dtype=torch.uint8, device=ic.device)
    L = torch.empty((N,), dtype=torch.float64, device=ic.device)
    gic = torch.empty((6, N), dtype=torch.float64, device=ic.device)
    geps = torch.empty((N,), dtype=torch.float64, device=ic.device)
    fn = _lib().aw_ftle_grad_reversible if reversible else _lib().aw_ftle_grad
    _abi.check(fn(ctypes.byref(ens.to_c()), _p(ic), _p(w0), _p(grad_L), int(ckpt_every), _p(L), _p(gic), _p(geps),
                  _p(workspace), workspace.numel() * workspace.element_size(), _tuning_ptr(tuning), _stream()))
    return L, gic, geps


class IndicatorL(torch.autograd.Function):
    """L_n = ln(|w_T| / |w_0|) per orbit (the tangent growth behind the FTLE
    lambda = L/(T h) and chi = L/ln(1 + T h)), from the seeded tangent start,
    differentiable in the initial state ic[N, 6] and in eps (a 0-d float64
    tensor); the backward pass runs the second-order adjoint kernels
    (reversible=True: the store-free sweep)."""

    @staticmethod
    def forward(ctx, ic, eps, n_steps: int, h: float = H_PAPER, map_form: str = "s6", ckpt_every: int = 100,
                seed_tangent: int = 0, reversible: bool = False):
        if ic.dim() != 2 or ic.shape[1] != 6:
            raise ValueError("ic must be [N, 6]")
        soa = ic.detach().t().contiguous()
        e = Ensemble(eps=float(eps), n_steps=n_steps, h=h, map_form=map_form, ic_kind="explicit",
                     n_orbits=ic.shape[0], seed_tangent=seed_tangent, tangent=True)
        res = map_ensemble(e, soa, want_class=False)
        ctx.save_for_backward(soa)
        ctx.ens = e
        ctx.ckpt = ckpt_every
        ctx.reversible = reversible
        ctx.eps_shape = eps.shape if isinstance(eps, torch.Tensor) else None
        return res.orbit_out[OUT_L].clone()

    @staticmethod
    def backward(ctx, gL):
        (soa,) = ctx.saved_tensors
        _, gic, geps = ftle_grad(ctx.ens, soa, grad_L=gL.contiguous().to(torch.float64), ckpt_every=ctx.ckpt,
                                 reversible=ctx.reversible)
        g_eps = geps.sum()
        if ctx.eps_shape is not None:
            g_eps = g_eps.reshape(ctx.eps_shape)
        return gic.t().contiguous(), g_eps, None, None, None, None, None, None


class Graph:
    """A HIP graph of the image path (aw_graph_*): the persistent launch over
    every ensemble and, for histogram images, their reductions."""

    def __init__(self, ens: List[Ensemble], spec: ImageSpec, images: List[torch.Tensor],
                 counts: Optional[List[torch.Tensor]] = None, classes: Optional[List[torch.Tensor]] = None,
                 tuning: Optional[Tuning] = None):
        n = len(ens)
        self._keep = (images, counts, classes)
        c_ens = (_abi.AwEnsemble * n)(*[e.to_c() for e in ens])
        h = ctypes.c_void_p()
        _abi.check(_lib().aw_graph_create(
            c_ens, n, ctypes.byref(spec.to_c()), _abi.ptr_array([_p(t) for t in images]),
            _abi.ptr_array([_p(t) for t in counts]) if counts else None,
            _abi.ptr_array([_p(t) for t in classes]) if classes else None, _tuning_ptr(tuning), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _abi.check(_lib().aw_graph_launch(self._h, _stream()))

    def close(self):
        if self._h:
            _lib().aw_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True) -> None:
    _abi.check(_lib().aw_timing_enable(1 if on else 0))


def timing_read():
    """(summed propagation-kernel milliseconds, launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _abi.check(_lib().aw_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def step_op_counts(map_form: str = "s6", tangent: bool = True):
    """FP64 (fma, mul, add) instructions per map step of the kernel as built."""
    f, m, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _abi.check(_lib().aw_step_op_counts(FORMS[map_form], int(tangent), ctypes.byref(f), ctypes.byref(m),
                                        ctypes.byref(a)))
    return f.value, m.value, a.value


def version() -> str:
    return _lib().aw_version().decode()
