// aw_ftle_adj.hip -- reverse-mode gradient of the tangent-growth indicator
// L = ln(|w_T| / |w_0|) (the finite-time Lyapunov indicator) with respect to
// the initial state and eps, for the maps of aw_fwd.hip: a second-order
// adjoint, since L is a function of the tangent map itself.
//
// The state of one orbit is s = (X, P) and its tangent w = (dX, dP); the
// adjoint carries (Xbar, Pbar, dXbar, dPbar) and epsbar.  With
// M(X) = -t eps Hess Hp(X) for a kick of weight t, the stages and their
// transposes are
//   drift D(t):  X += t P, dX += t dP
//                Pbar += t Xbar, dPbar += t dXbar
//   kick  K(t):  P += -t eps grad Hp(X), dP += M(X) dX
//                Xbar  += M(X) Pbar - t eps T3(X)[dX, dPbar]
//                dXbar += M(X) dPbar
//                epsbar += -t grad Hp(X) . Pbar - t (Hess Hp(X) dX) . dPbar
// where T3 is the third-derivative tensor of Hp (symmetric), contracted
// with dX and dPbar.  The end condition is dL/dw_T = w_T / |w_T|^2.
//
// The tangent is rescaled by exact powers of two after every 8th step
// (global step count), as in the forward kernel.  A rescale w <- 2^-k w is
// linear, so its transpose rescales the adjoint of w by the same 2^-k; the
// exponent is recomputed in the reverse sweep from the stored pre-rescale
// tangent, so it matches the forward pass exactly.
//
// Forward kernel: one lane per orbit runs the map with its tangent, stores
// (s, w) at the start of every segment of `ckpt` steps and writes L.
// Backward kernel: one lane per orbit walks the segments from the last; for
// each it recomputes the segment from its checkpoint, storing (s, w) at the
// end of every step (before any rescale), then sweeps the steps backwards,
// undoing each stage by its exact inverse (drift: X -= t P, dX -= t dP;
// kick: P -= the kick's increment, dP -= M dX) while the adjoint above is
// propagated.  Each lane only reads back what it wrote itself.
//
// Reversible sweep (k_ftle_bwd_rev): no recompute and no stored step states.
// Each segment is swept back from the exact state at its end (the next
// checkpoint; the final state for the last segment), inverting the stages of
// state and tangent step after step.  The exponent of every rescale cannot be
// recovered from the rescaled tangent, so the forward pass records it (one
// 16-bit integer per orbit per 8 steps) and the sweep applies it to the tangent and,
// inversely, to its adjoint.
#include <hip/hip_runtime.h>

#include "aw_device.hpp"
#include "aw_internal.hpp"
#include "aw_launch.hpp"

namespace aw {

namespace {

constexpr double LN2_D = 0.693147180559945309417232121458176568;
constexpr int64_t RESCALE_MASK = 7;  // rescale after steps k with (k + 1) % 8 == 0

template <int FORM>
__device__ __forceinline__ void tan_step(Orbit &o, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      drift<true>(o, d.drift[F::drift_idx[i]]);
      kick_tab<true>(o, d.ka2[F::kick_idx[i]], d.ka4[F::kick_idx[i]], tab);
    }
    drift<true>(o, d.drift[F::drift_idx[NK]]);
  } else {
    kick_tab<true>(o, d.ka2[0], d.ka4[0], tab);
    drift<true>(o, d.drift[0]);
  }
}

struct Adjoint2 {
  double xb, yb, zb, pxb, pyb, pzb;        // state adjoint
  double dxb, dyb, dzb, dpxb, dpyb, dpzb;  // tangent adjoint
  double eb;                               // eps adjoint
};

// Undo D(t) and apply its transpose.
__device__ __forceinline__ void rev_drift2(Orbit &o, Adjoint2 &a, double t) {
  o.x = __builtin_fma(-t, o.px, o.x);
  o.y = __builtin_fma(-t, o.py, o.y);
  o.z = __builtin_fma(-t, o.pz, o.z);
  o.dx = __builtin_fma(-t, o.dpx, o.dx);
  o.dy = __builtin_fma(-t, o.dpy, o.dy);
  o.dz = __builtin_fma(-t, o.dpz, o.dz);
  a.pxb = __builtin_fma(t, a.xb, a.pxb);
  a.pyb = __builtin_fma(t, a.yb, a.pyb);
  a.pzb = __builtin_fma(t, a.zb, a.pzb);
  a.dpxb = __builtin_fma(t, a.dxb, a.dpxb);
  a.dpyb = __builtin_fma(t, a.dyb, a.dpyb);
  a.dpzb = __builtin_fma(t, a.dzb, a.dpzb);
}

// Undo K(t) and apply its transpose.  a2 = 2 t eps, a4 = 4 t eps, w2 = 2 t,
// w4 = 4 t.  Sines and cosines from the same table as the forward kick.
//   t eps Hp_xxx = t eps Hp_xyy = e1 sx cy     t eps Hp_xxy = t eps Hp_yyy = e1 cx sy
//   t eps Hp_xxz = t eps Hp_yyz = e2 cx cy     t eps Hp_xyz = -e2 sx sy
//   t eps Hp_xzz = e3 sx cy   t eps Hp_yzz = e3 cx sy   t eps Hp_zzz = 4 e2 cx cy
// with e1 = 2 t eps cz^2, e2 = 4 t eps cz sz, e3 = 4 t eps (cz^2 - sz^2).
__device__ __forceinline__ void rev_kick2(Orbit &o, Adjoint2 &a, double a2, double a4, double w2, double w4,
                                          const double2 *__restrict__ tab) {
  const SinCosT X = sincos_tab(o.x, tab), Y = sincos_tab(o.y, tab);
  const ZTerms Z = zterms_tab(o.z, tab);
  const double cx = X.c, sx = X.s;
  const double cy = Y.c, sy = Y.s;
  const double psc = sx * cy, pcs = cx * sy, pcc = cx * cy, pss = sx * sy;
  const double e1 = a2 * Z.cz2, e2 = a4 * Z.czsz, e3 = __builtin_fma(4.0, e1, -a4);
  // M = -t eps Hess: diagonal mxx (= myy), mzz; off-diagonal -nxy, -nxz, -nyz.
  const double mxx = e1 * pcc, nxy = e1 * pss, nxz = e2 * psc, nyz = e2 * pcs, mzz = e3 * pcc;
  // The same matrix per unit eps (for epsbar).
  const double f1 = w2 * Z.cz2, f2 = w4 * Z.czsz, f3 = __builtin_fma(4.0, f1, -w4);
  const double wxx = f1 * pcc, vxy = f1 * pss, vxz = f2 * psc, vyz = f2 * pcs, wzz = f3 * pcc;
  const double dx = o.dx, dy = o.dy, dz = o.dz;
  const double pxb = a.pxb, pyb = a.pyb, pzb = a.pzb;
  const double dpxb = a.dpxb, dpyb = a.dpyb, dpzb = a.dpzb;

  // epsbar: d(P')/d eps = -t grad Hp, d(dP')/d eps = (M / eps) dX.
  double eb = a.eb;
  eb = __builtin_fma(f1, __builtin_fma(psc, pxb, pcs * pyb), eb);
  eb = __builtin_fma(f2 * pcc, pzb, eb);
  const double ux = __builtin_fma(wxx, dx, __builtin_fma(-vxy, dy, -vxz * dz));
  const double uy = __builtin_fma(-vxy, dx, __builtin_fma(wxx, dy, -vyz * dz));
  const double uz = __builtin_fma(-vxz, dx, __builtin_fma(-vyz, dy, wzz * dz));
  eb = __builtin_fma(ux, dpxb, eb);
  eb = __builtin_fma(uy, dpyb, eb);
  eb = __builtin_fma(uz, dpzb, eb);
  a.eb = eb;

  // Xbar += M Pbar.
  double xb = a.xb, yb = a.yb, zb = a.zb;
  xb = __builtin_fma(mxx, pxb, xb);
  xb = __builtin_fma(-nxy, pyb, xb);
  xb = __builtin_fma(-nxz, pzb, xb);
  yb = __builtin_fma(-nxy, pxb, yb);
  yb = __builtin_fma(mxx, pyb, yb);
  yb = __builtin_fma(-nyz, pzb, yb);
  zb = __builtin_fma(-nxz, pxb, zb);
  zb = __builtin_fma(-nyz, pyb, zb);
  zb = __builtin_fma(mzz, pzb, zb);
  // Xbar -= t eps T3[dX, dPbar] from the symmetric products of dX and dPbar.
  const double mdiag = __builtin_fma(dx, dpxb, dy * dpyb);        // dx dpxb + dy dpyb
  const double mz = dz * dpzb;
  const double sxy = __builtin_fma(dx, dpyb, dy * dpxb);
  const double sxz = __builtin_fma(dx, dpzb, dz * dpxb);
  const double syz = __builtin_fma(dy, dpzb, dz * dpyb);
  const double q1 = e1 * psc, q2 = e1 * pcs, q3 = e2 * pcc, q4 = -(e2 * pss), q5 = e3 * psc, q6 = e3 * pcs;
  const double q7 = 4.0 * q3;
  xb = __builtin_fma(-q1, mdiag, xb);
  xb = __builtin_fma(-q2, sxy, xb);
  xb = __builtin_fma(-q3, sxz, xb);
  xb = __builtin_fma(-q4, syz, xb);
  xb = __builtin_fma(-q5, mz, xb);
  yb = __builtin_fma(-q2, mdiag, yb);
  yb = __builtin_fma(-q1, sxy, yb);
  yb = __builtin_fma(-q4, sxz, yb);
  yb = __builtin_fma(-q3, syz, yb);
  yb = __builtin_fma(-q6, mz, yb);
  zb = __builtin_fma(-q3, mdiag, zb);
  zb = __builtin_fma(-q4, sxy, zb);
  zb = __builtin_fma(-q5, sxz, zb);
  zb = __builtin_fma(-q6, syz, zb);
  zb = __builtin_fma(-q7, mz, zb);
  a.xb = xb;
  a.yb = yb;
  a.zb = zb;

  // dXbar += M dPbar.
  a.dxb = __builtin_fma(mxx, dpxb, __builtin_fma(-nxy, dpyb, __builtin_fma(-nxz, dpzb, a.dxb)));
  a.dyb = __builtin_fma(-nxy, dpxb, __builtin_fma(mxx, dpyb, __builtin_fma(-nyz, dpzb, a.dyb)));
  a.dzb = __builtin_fma(-nxz, dpxb, __builtin_fma(-nyz, dpyb, __builtin_fma(mzz, dpzb, a.dzb)));

  // Undo the kick: dP -= M dX, P -= (e1 sx cy, e1 cx sy, e2 cx cy).
  o.dpx = __builtin_fma(-mxx, dx, __builtin_fma(nxy, dy, __builtin_fma(nxz, dz, o.dpx)));
  o.dpy = __builtin_fma(nxy, dx, __builtin_fma(-mxx, dy, __builtin_fma(nyz, dz, o.dpy)));
  o.dpz = __builtin_fma(nxz, dx, __builtin_fma(nyz, dy, __builtin_fma(-mzz, dz, o.dpz)));
  o.px = __builtin_fma(-e1, psc, o.px);
  o.py = __builtin_fma(-e1, pcs, o.py);
  o.pz = __builtin_fma(-e2, pcc, o.pz);
}

template <int FORM>
__device__ __forceinline__ void rev_tan_step(Orbit &o, Adjoint2 &a, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
    rev_drift2(o, a, d.drift[F::drift_idx[NK]]);
#pragma unroll
    for (int i = NK - 1; i >= 0; --i) {
      const int u = F::kick_idx[i];
      rev_kick2(o, a, d.ka2[u], d.ka4[u], d.kw2[u], d.kw4[u], tab);
      rev_drift2(o, a, d.drift[F::drift_idx[i]]);
    }
  } else {
    rev_drift2(o, a, d.drift[0]);
    rev_kick2(o, a, d.ka2[0], d.ka4[0], d.kw2[0], d.kw4[0], tab);
  }
}

__device__ __forceinline__ void load12(const double *p, int64_t N, int64_t n, Orbit &o) {
  o.x = p[0 * N + n]; o.y = p[1 * N + n]; o.z = p[2 * N + n];
  o.px = p[3 * N + n]; o.py = p[4 * N + n]; o.pz = p[5 * N + n];
  o.dx = p[6 * N + n]; o.dy = p[7 * N + n]; o.dz = p[8 * N + n];
  o.dpx = p[9 * N + n]; o.dpy = p[10 * N + n]; o.dpz = p[11 * N + n];
}

__device__ __forceinline__ void store12(double *p, int64_t N, int64_t n, const Orbit &o) {
  p[0 * N + n] = o.x; p[1 * N + n] = o.y; p[2 * N + n] = o.z;
  p[3 * N + n] = o.px; p[4 * N + n] = o.py; p[5 * N + n] = o.pz;
  p[6 * N + n] = o.dx; p[7 * N + n] = o.dy; p[8 * N + n] = o.dz;
  p[9 * N + n] = o.dpx; p[10 * N + n] = o.dpy; p[11 * N + n] = o.dpz;
}

__device__ __forceinline__ double tan_norm2(const Orbit &o) {
  double n2 = o.dx * o.dx;
  n2 = __builtin_fma(o.dy, o.dy, n2);
  n2 = __builtin_fma(o.dz, o.dz, n2);
  n2 = __builtin_fma(o.dpx, o.dpx, n2);
  n2 = __builtin_fma(o.dpy, o.dpy, n2);
  n2 = __builtin_fma(o.dpz, o.dpz, n2);
  return n2;
}

// Power-of-two exponent the forward rescale applies to this tangent.
__device__ __forceinline__ int rescale_exponent(const Orbit &o) {
  Orbit t = o;
  t.kexp = 0;
  renorm(t);
  return t.kexp;
}

template <int FORM>
__global__ __launch_bounds__(512) void k_ftle_fwd(FtleDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  const int64_t N = d.N;
  Orbit o;
  o.x = d.ic[0 * N + n]; o.y = d.ic[1 * N + n]; o.z = d.ic[2 * N + n];
  o.px = d.ic[3 * N + n]; o.py = d.ic[4 * N + n]; o.pz = d.ic[5 * N + n];
  o.dx = d.w0[0 * N + n]; o.dy = d.w0[1 * N + n]; o.dz = d.w0[2 * N + n];
  o.dpx = d.w0[3 * N + n]; o.dpy = d.w0[4 * N + n]; o.dpz = d.w0[5 * N + n];
  o.p0x = o.px; o.p0y = o.py; o.p0z = o.pz;
  o.jsum = 0.0;
  o.kexp = 0;
  const double n0 = tan_norm2(o);
  for (int64_t s = 0; s < d.n_seg; ++s) {
    store12(d.ckpts + s * 12 * N, N, n, o);
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    for (int64_t g = g0; g < g1; ++g) {
      tan_step<FORM>(o, d, s_tab);
      if (d.fwd_steps) store12(d.steps + g * 12 * N, N, n, o);  // one segment: g0 = 0
      if (((g + 1) & RESCALE_MASK) == 0) {
        const int k0 = o.kexp;
        renorm(o);
        d.exps[((g + 1) / (RESCALE_MASK + 1) - 1) * N + n] = (int16_t)(o.kexp - k0);
      }
    }
  }
  store12(d.ckpts + d.n_seg * 12 * N, N, n, o);   // the final state (after any last rescale)
  if (d.L) {
    const double n2 = tan_norm2(o);
    const int e = __builtin_amdgcn_frexp_exp(n2);
    const double mant = __builtin_amdgcn_frexp_mant(n2);
    d.L[n] = 0.5 * ((double)(2 * o.kexp + e) * LN2_D + log(mant)) - 0.5 * log(n0);
  }
}

template <int FORM>
__global__ __launch_bounds__(512) void k_ftle_bwd(FtleDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  const int64_t N = d.N;
  const double gl = d.gL ? d.gL[n] : 1.0;
  Adjoint2 a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  Orbit o;
  o.p0x = o.p0y = o.p0z = 0.0;
  o.jsum = 0.0;
  o.kexp = 0;
  for (int64_t s = d.n_seg - 1; s >= 0; --s) {
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    if (!d.fwd_steps) {  // else the forward pass has stored the steps already
      load12(d.ckpts + s * 12 * N, N, n, o);
      for (int64_t g = g0; g < g1; ++g) {
        tan_step<FORM>(o, d, s_tab);
        store12(d.steps + (g - g0) * 12 * N, N, n, o);
        if (((g + 1) & RESCALE_MASK) == 0) renorm(o);
      }
    }
    for (int64_t g = g1 - 1; g >= g0; --g) {
      load12(d.steps + (g - g0) * 12 * N, N, n, o);   // end of step g, before any rescale
      if (g == d.T - 1) {
        // dL/dw_T = w_T / |w_T|^2 (scaled by the upstream gradient).
        const double c = gl / tan_norm2(o);
        a.dxb = c * o.dx; a.dyb = c * o.dy; a.dzb = c * o.dz;
        a.dpxb = c * o.dpx; a.dpyb = c * o.dpy; a.dpzb = c * o.dpz;
      } else if (((g + 1) & RESCALE_MASK) == 0) {
        const int k = rescale_exponent(o);
        a.dxb = __builtin_amdgcn_ldexp(a.dxb, -k);
        a.dyb = __builtin_amdgcn_ldexp(a.dyb, -k);
        a.dzb = __builtin_amdgcn_ldexp(a.dzb, -k);
        a.dpxb = __builtin_amdgcn_ldexp(a.dpxb, -k);
        a.dpyb = __builtin_amdgcn_ldexp(a.dpyb, -k);
        a.dpzb = __builtin_amdgcn_ldexp(a.dpzb, -k);
      }
      rev_tan_step<FORM>(o, a, d, s_tab);
    }
  }
  d.gic[0 * N + n] = a.xb;
  d.gic[1 * N + n] = a.yb;
  d.gic[2 * N + n] = a.zb;
  d.gic[3 * N + n] = a.pxb;
  d.gic[4 * N + n] = a.pyb;
  d.gic[5 * N + n] = a.pzb;
  d.geps[n] = a.eb;
}

template <int FORM>
__global__ __launch_bounds__(512) void k_ftle_bwd_rev(FtleDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  const int64_t N = d.N;
  const double gl = d.gL ? d.gL[n] : 1.0;
  Adjoint2 a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  Orbit o;
  o.p0x = o.p0y = o.p0z = 0.0;
  o.jsum = 0.0;
  o.kexp = 0;
  for (int64_t s = d.n_seg - 1; s >= 0; --s) {
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    // Exact state at the end of step g1 - 1, after any rescale there.
    load12(d.ckpts + (s + 1) * 12 * N, N, n, o);
    for (int64_t g = g1 - 1; g >= g0; --g) {
      // o: the state at the end of step g, after any rescale that followed it.
      if (g == d.T - 1) {
        const double c = gl / tan_norm2(o);
        a.dxb = c * o.dx; a.dyb = c * o.dy; a.dzb = c * o.dz;
        a.dpxb = c * o.dpx; a.dpyb = c * o.dpy; a.dpzb = c * o.dpz;
      }
      if (((g + 1) & RESCALE_MASK) == 0) {
        // the forward set w_post = 2^-k w_pre: restore w_pre, and wbar_pre = 2^-k wbar_post
        const int k = d.exps[((g + 1) / (RESCALE_MASK + 1) - 1) * N + n];
        o.dx = __builtin_amdgcn_ldexp(o.dx, k);
        o.dy = __builtin_amdgcn_ldexp(o.dy, k);
        o.dz = __builtin_amdgcn_ldexp(o.dz, k);
        o.dpx = __builtin_amdgcn_ldexp(o.dpx, k);
        o.dpy = __builtin_amdgcn_ldexp(o.dpy, k);
        o.dpz = __builtin_amdgcn_ldexp(o.dpz, k);
        a.dxb = __builtin_amdgcn_ldexp(a.dxb, -k);
        a.dyb = __builtin_amdgcn_ldexp(a.dyb, -k);
        a.dzb = __builtin_amdgcn_ldexp(a.dzb, -k);
        a.dpxb = __builtin_amdgcn_ldexp(a.dpxb, -k);
        a.dpyb = __builtin_amdgcn_ldexp(a.dpyb, -k);
        a.dpzb = __builtin_amdgcn_ldexp(a.dpzb, -k);
      }
      rev_tan_step<FORM>(o, a, d, s_tab);   // o: the state at the start of step g
    }
  }
  d.gic[0 * N + n] = a.xb;
  d.gic[1 * N + n] = a.yb;
  d.gic[2 * N + n] = a.zb;
  d.gic[3 * N + n] = a.pxb;
  d.gic[4 * N + n] = a.pyb;
  d.gic[5 * N + n] = a.pzb;
  d.geps[n] = a.eb;
}

}  // namespace

hipError_t launch_ftle_backward_reversible(const FtleDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1: hipLaunchKernelGGL(k_ftle_bwd_rev<1>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 2: hipLaunchKernelGGL(k_ftle_bwd_rev<2>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 4: hipLaunchKernelGGL(k_ftle_bwd_rev<4>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 6: hipLaunchKernelGGL(k_ftle_bwd_rev<6>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 7: hipLaunchKernelGGL(k_ftle_bwd_rev<7>, dim3(blocks), dim3(tb), 0, s, d); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ftle_forward(const FtleDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1: hipLaunchKernelGGL(k_ftle_fwd<1>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 2: hipLaunchKernelGGL(k_ftle_fwd<2>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 4: hipLaunchKernelGGL(k_ftle_fwd<4>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 6: hipLaunchKernelGGL(k_ftle_fwd<6>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 7: hipLaunchKernelGGL(k_ftle_fwd<7>, dim3(blocks), dim3(tb), 0, s, d); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ftle_backward(const FtleDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1: hipLaunchKernelGGL(k_ftle_bwd<1>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 2: hipLaunchKernelGGL(k_ftle_bwd<2>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 4: hipLaunchKernelGGL(k_ftle_bwd<4>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 6: hipLaunchKernelGGL(k_ftle_bwd<6>, dim3(blocks), dim3(tb), 0, s, d); break;
  case 7: hipLaunchKernelGGL(k_ftle_bwd<7>, dim3(blocks), dim3(tb), 0, s, d); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aw
