// aw_adj.hip -- reverse-mode (adjoint) gradient of the step-averaged momentum
// drift J = (1/T) sum_{k=1..T} |P_k - P_0|^2 with respect to the initial
// state and eps, for the maps of aw_fwd.hip.
//
// Forward kernel: one lane per orbit runs the map (no tangent), accumulates J
// and stores the state at the start of every segment of `ckpt` steps.
// Backward kernel: one lane per orbit walks the segments from the last one;
// for each it recomputes the segment from its checkpoint, keeping the end
// state of every ADJ_SUB-th step (and of the segment's last step), then sweeps
// the steps backwards.  The stages are undone in reverse order by inverting
// them exactly in exact arithmetic (drift: X -= t P; kick: P += t eps grad
// Hp(X)), starting from the kept state at the end of each group of ADJ_SUB
// steps and carrying the rebuilt state through the group, while the adjoint
// is propagated:
//   drift  D(t):  Pbar += t Xbar
//   kick   K(t):  Xbar -= t eps Hess(X) Pbar,  epsbar -= t grad Hp(X) . Pbar
// and the source of J, (2 gJ / T)(P_k - P_0), enters Pbar at every step
// boundary k >= 1.  The explicit P_0 dependence of J adds
// -(2 gJ / T) sum_k (P_k - P_0) to the initial-momentum gradient.
// All of it runs in the rotated frame of the forward kernels (u = x + y,
// v = x - y, momenta alike), where the kick's Jacobian has 7 non-zero entries;
// the checkpoints and step states hold rotated states, and the gradient is
// taken back to (x, y) at the end.
// Each lane only reads back what it wrote itself, so no synchronisation
// between lanes is needed.
//
// Reversible sweep (k_adj_bwd_rev): the same reverse pass without the
// recompute and without storing step states.  Each segment is swept back from
// the exact state at its end (the next checkpoint; the final state for the
// last segment), undoing the steps one after the other by inverting their
// stages.  The reconstructed states carry the rounding of the inversion,
// which restarts from an exact state at every checkpoint.
#include <hip/hip_runtime.h>

#include "aw_device.hpp"
#include "aw_internal.hpp"
#include "aw_launch.hpp"

namespace aw {

template <int FORM>
__device__ __forceinline__ void adj_step_fwd(Orbit &o, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      drift<false>(o, d.drift[F::drift_idx[i]]);
      kick_rot<false>(o, d.ka2[F::kick_idx[i]], tab);
    }
    drift<false>(o, d.drift[F::drift_idx[NK]]);
  } else {
    kick_rot<false>(o, d.ka2[0], tab);
    drift<false>(o, d.drift[0]);
  }
}

struct Adjoint {
  double xb, yb, zb, pxb, pyb, pzb, eb;
};

// Undo D(t) on the state and apply its transpose to the adjoint.
__device__ __forceinline__ void rev_drift(Orbit &o, Adjoint &a, double t) {
  o.x = __builtin_fma(-t, o.px, o.x);
  o.y = __builtin_fma(-t, o.py, o.y);
  o.z = __builtin_fma(-t, o.pz, o.z);
  a.pxb = __builtin_fma(t, a.xb, a.pxb);
  a.pyb = __builtin_fma(t, a.yb, a.pyb);
  a.pzb = __builtin_fma(t, a.zb, a.pzb);
}

// Undo K(t) on the state and apply its transpose to the adjoint, in the
// rotated frame of the forward kernels (u = x + y, v = x - y; the Adjoint's
// xb, yb, pxb, pyb hold the adjoints of u, v, p_u, p_v).  a2 = 2 t eps,
// w2 = 2 t.  With e1 = a2 cz^2, e2 = a2 cz sz, cs = cos u + cos v the kick is
// F = (e1 sin u, e1 sin v, e2 cs) and its Jacobian
//   [[e1 cos u, 0, -2 e2 sin u], [0, e1 cos v, -2 e2 sin v],
//    [-e2 sin u, -e2 sin v, cs (2 e1 - a2)]],
// whose transpose acts on Pbar; dF/deps = F / eps.  For eps != 0 (EPS0
// false) a.eb collects eps epsbar = F . Pbar and the kernel divides by eps
// once at the end; for eps = 0 (EPS0 true) F / eps is formed from w2 = 2 t.
// Sines and cosines from the same table as the forward kick, so the undone
// kick matches it.
template <bool EPS0>
__device__ __forceinline__ void rev_kick(Orbit &o, Adjoint &a, double a2, double w2,
                                         const double2 *__restrict__ tab) {
  const SinCosT U = sincos_tab(o.x, tab), V = sincos_tab(o.y, tab);
  const ZTerms Z = zterms_tab(o.z, tab);
  const double e1 = a2 * Z.cz2, e2 = a2 * Z.czsz;
  const double cs = U.c + V.c;
  const double pub = a.pxb, pvb = a.pyb, pzb = a.pzb;
  const double q = __builtin_fma(U.s, pub, V.s * pvb);   // sin u pu_bar + sin v pv_bar
  if constexpr (EPS0) {
    a.eb = __builtin_fma(w2 * Z.cz2, q, a.eb);
    a.eb = __builtin_fma((w2 * Z.czsz) * cs, pzb, a.eb);
  } else {
    a.eb = __builtin_fma(e1, q, a.eb);
    a.eb = __builtin_fma(e2 * cs, pzb, a.eb);
  }
  const double e2p = e2 * pzb;
  a.xb = __builtin_fma(e1 * U.c, pub, __builtin_fma(-U.s, e2p, a.xb));
  a.yb = __builtin_fma(e1 * V.c, pvb, __builtin_fma(-V.s, e2p, a.yb));
  const double mz = cs * __builtin_fma(2.0, e1, -a2);
  a.zb = __builtin_fma(mz, pzb, __builtin_fma(-2.0 * e2, q, a.zb));
  // P before the kick.
  o.px = __builtin_fma(-e1, U.s, o.px);
  o.py = __builtin_fma(-e1, V.s, o.py);
  o.pz = __builtin_fma(-e2, cs, o.pz);
}

template <int FORM, bool EPS0>
__device__ __forceinline__ void adj_step_rev(Orbit &o, Adjoint &a, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
    rev_drift(o, a, d.drift[F::drift_idx[NK]]);
#pragma unroll
    for (int i = NK - 1; i >= 0; --i) {
      const int u = F::kick_idx[i];
      rev_kick<EPS0>(o, a, d.ka2[u], d.kw2[u], tab);
      rev_drift(o, a, d.drift[F::drift_idx[i]]);
    }
  } else {
    rev_drift(o, a, d.drift[0]);
    rev_kick<EPS0>(o, a, d.ka2[0], d.kw2[0], tab);
  }
}

__device__ __forceinline__ void load6(const double *p, int64_t N, int64_t n, Orbit &o) {
  o.x = p[0 * N + n]; o.y = p[1 * N + n]; o.z = p[2 * N + n];
  o.px = p[3 * N + n]; o.py = p[4 * N + n]; o.pz = p[5 * N + n];
}

__device__ __forceinline__ void store6(double *p, int64_t N, int64_t n, const Orbit &o) {
  p[0 * N + n] = o.x; p[1 * N + n] = o.y; p[2 * N + n] = o.z;
  p[3 * N + n] = o.px; p[4 * N + n] = o.py; p[5 * N + n] = o.pz;
}

template <int FORM>
__global__ __launch_bounds__(512) void k_adj_fwd(AdjDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  Orbit o;
  load6(d.ic, d.N, n, o);
  o.p0x = o.px; o.p0y = o.py; o.p0z = o.pz;
  o.dx = o.dy = o.dz = o.dpx = o.dpy = o.dpz = 0.0;
  to_rot(o);
  o.jsum = 0.0;
  for (int64_t s = 0; s < d.n_seg; ++s) {
    store6(d.ckpts + s * 6 * d.N, d.N, n, o);
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    for (int64_t g = g0; g < g1; ++g) {
      adj_step_fwd<FORM>(o, d, s_tab);
      accum_j_rot(o);
      if (d.fwd_steps && adj_kept(g, g1)) store6(d.steps + adj_slot(g, 0) * 6 * d.N, d.N, n, o);  // one segment
    }
  }
  store6(d.ckpts + d.n_seg * 6 * d.N, d.N, n, o);   // the final state
  if (d.J) d.J[n] = (0.5 * o.jsum) / (double)d.T;
}

// The initial-state gradient: the explicit P_0 share of J, then back from the
// rotated frame (u = x + y, v = x - y, so d/dx = d/du + d/dv and
// d/dy = d/du - d/dv; momenta alike).
__device__ __forceinline__ void store_grad(const AdjDesc &d, int64_t n, const Adjoint &a, double ch, double c,
                                           double su, double sv, double sz) {
  const int64_t N = d.N;
  const double pub = __builtin_fma(-ch, su, a.pxb), pvb = __builtin_fma(-ch, sv, a.pyb);
  d.gic[0 * N + n] = a.xb + a.yb;
  d.gic[1 * N + n] = a.xb - a.yb;
  d.gic[2 * N + n] = a.zb;
  d.gic[3 * N + n] = pub + pvb;
  d.gic[4 * N + n] = pub - pvb;
  d.gic[5 * N + n] = __builtin_fma(-c, sz, a.pzb);
  d.geps[n] = a.eb;
}

template <int FORM, bool EPS0>
__global__ __launch_bounds__(512) void k_adj_bwd_rev(AdjDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  const int64_t N = d.N;
  // P_0 in the rotated frame, rounded as the forward pass formed it.
  const double p0x = d.ic[3 * N + n] + d.ic[4 * N + n], p0y = d.ic[3 * N + n] - d.ic[4 * N + n];
  const double p0z = d.ic[5 * N + n];
  // J = (1/T) sum ((P_u - P0_u)^2 + (P_v - P0_v)^2) / 2 + (P_z - P0_z)^2: the
  // source is c/2 on p_u and p_v and c on p_z.
  const double c = 2.0 * (d.gJ ? d.gJ[n] : 1.0) / (double)d.T;
  const double ch = 0.5 * c;
  Adjoint a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double sx = 0.0, sy = 0.0, sz = 0.0;  // sum_k (P_k - P_0)
  Orbit o;
  o.p0x = p0x; o.p0y = p0y; o.p0z = p0z;
  o.jsum = 0.0;
  o.kexp = 0;
  o.dx = o.dy = o.dz = o.dpx = o.dpy = o.dpz = 0.0;
  for (int64_t s = d.n_seg - 1; s >= 0; --s) {
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    load6(d.ckpts + (s + 1) * 6 * N, N, n, o);        // exact state after step g1 - 1
    for (int64_t g = g1 - 1; g >= g0; --g) {
      const double ex = o.px - p0x, ey = o.py - p0y, ez = o.pz - p0z;
      a.pxb = __builtin_fma(ch, ex, a.pxb);
      a.pyb = __builtin_fma(ch, ey, a.pyb);
      a.pzb = __builtin_fma(c, ez, a.pzb);
      sx += ex; sy += ey; sz += ez;
      adj_step_rev<FORM, EPS0>(o, a, d, s_tab);              // state now at the start of step g
    }
  }
  if (!EPS0) a.eb /= d.eps;   // the kicks collected eps epsbar
  store_grad(d, n, a, ch, c, sx, sy, sz);
}

template <int FORM, bool EPS0>
__global__ __launch_bounds__(512) void k_adj_bwd(AdjDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  const int64_t N = d.N;
  // P_0 in the rotated frame, rounded as the forward pass formed it.
  const double p0x = d.ic[3 * N + n] + d.ic[4 * N + n], p0y = d.ic[3 * N + n] - d.ic[4 * N + n];
  const double p0z = d.ic[5 * N + n];
  // J = (1/T) sum ((P_u - P0_u)^2 + (P_v - P0_v)^2) / 2 + (P_z - P0_z)^2: the
  // source is c/2 on p_u and p_v and c on p_z.
  const double c = 2.0 * (d.gJ ? d.gJ[n] : 1.0) / (double)d.T;
  const double ch = 0.5 * c;
  Adjoint a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double sx = 0.0, sy = 0.0, sz = 0.0;  // sum_k (P_k - P_0)
  Orbit o;
  o.p0x = p0x; o.p0y = p0y; o.p0z = p0z;
  o.jsum = 0.0;
  o.kexp = 0;
  for (int64_t s = d.n_seg - 1; s >= 0; --s) {
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    if (!d.fwd_steps) {  // else the forward pass has kept the step states already
      load6(d.ckpts + s * 6 * N, N, n, o);
      for (int64_t g = g0; g < g1; ++g) {
        adj_step_fwd<FORM>(o, d, s_tab);
        if (adj_kept(g, g1)) store6(d.steps + adj_slot(g, g0) * 6 * N, N, n, o);
      }
    }
    for (int64_t g = g1 - 1; g >= g0; --g) {
      // state after step g: kept, or rebuilt by the inverse of step g + 1
      if (adj_kept(g, g1)) load6(d.steps + adj_slot(g, g0) * 6 * N, N, n, o);
      const double ex = o.px - p0x, ey = o.py - p0y, ez = o.pz - p0z;
      a.pxb = __builtin_fma(ch, ex, a.pxb);
      a.pyb = __builtin_fma(ch, ey, a.pyb);
      a.pzb = __builtin_fma(c, ez, a.pzb);
      sx += ex; sy += ey; sz += ez;
      adj_step_rev<FORM, EPS0>(o, a, d, s_tab);
    }
  }
  if (!EPS0) a.eb /= d.eps;   // the kicks collected eps epsbar
  store_grad(d, n, a, ch, c, sx, sy, sz);
}

hipError_t launch_adj_forward(const AdjDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1: hipLaunchKernelGGL(k_adj_fwd<1>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 2: hipLaunchKernelGGL(k_adj_fwd<2>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 4: hipLaunchKernelGGL(k_adj_fwd<4>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 6: hipLaunchKernelGGL(k_adj_fwd<6>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 7: hipLaunchKernelGGL(k_adj_fwd<7>, dim3(blocks), dim3(tb), 0, s, d); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adj_backward_reversible(const AdjDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const bool e0 = d.eps == 0.0;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<1, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<1, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 2:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<2, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<2, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 4:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<4, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<4, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 6:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<6, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<6, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 7:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<7, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd_rev<7, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adj_backward(const AdjDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const bool e0 = d.eps == 0.0;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<1, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<1, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 2:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<2, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<2, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 4:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<4, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<4, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 6:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<6, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<6, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 7:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<7, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_bwd<7, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aw
