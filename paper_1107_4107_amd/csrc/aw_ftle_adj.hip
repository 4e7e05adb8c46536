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
// The kernels step in the rotated frame of the forward kernels (u = x + y,
// v = x - y, momenta and tangent alike): there the kick's Jacobian has 7
// non-zero entries and is not symmetric (the frame is not orthonormal), the
// norm of w carries the weights (1/2, 1/2, 1, 1/2, 1/2, 1), and the gradient
// is taken back to (x, y) at the end.
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
// each it recomputes the segment from its checkpoint, keeping (s, w) at the
// end of every ADJ_SUB-th step and of the segment's last step (before any
// rescale), then sweeps the steps backwards, undoing each stage by its exact
// inverse (drift: X -= t P, dX -= t dP; kick: P -= the kick's increment,
// dP -= M dX) from the kept state at the end of each group of steps, while the
// adjoint above is propagated.  Each lane only reads back what it wrote itself.
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
static_assert(((RESCALE_MASK + 1) % ADJ_SUB) == 0, "every rescale step must be a kept step");

template <int FORM>
__device__ __forceinline__ void tan_step(Orbit &o, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      drift<true>(o, d.drift[F::drift_idx[i]]);
      kick_rot<true>(o, d.ka2[F::kick_idx[i]], tab);
    }
    drift<true>(o, d.drift[F::drift_idx[NK]]);
  } else {
    kick_rot<true>(o, d.ka2[0], tab);
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

// Undo K(t) and apply its transpose, in the rotated frame of the steps
// (u = x + y, v = x - y; the Adjoint2's x, y, px, py fields hold u, v, p_u,
// p_v and their tangents).  a2 = 2 t eps, w2 = 2 t.  With e1 = a2 cz^2,
// e2 = a2 cz sz, g = 2 e1 - a2 (= de2/dz; de1/dz = -2 e2) and
// cs = cos u + cos v, the kick is F = (e1 sin u, e1 sin v, e2 cs) with Jacobian
//   M = [[e1 cos u, 0, -2 e2 sin u], [0, e1 cos v, -2 e2 sin v],
//        [-e2 sin u, -e2 sin v, cs g]],
// and the tangent kick dP += M dX.  Its transpose gives
//   Xbar  += M^T Pbar + S,   S_k = sum_ij dPbar_i (dM_ij/dX_k) dX_j,
//   dXbar += M^T dPbar,      epsbar += (F . Pbar + (M dX) . dPbar) / eps,
// where, with Bu = e2 cos u du + g sin u dz, Bv = e2 cos v dv + g sin v dz,
//   S_u = -dPbar_u (e1 sin u du + 2 e2 cos u dz) - dPbar_z Bu,
//   S_v = -dPbar_v (e1 sin v dv + 2 e2 cos v dz) - dPbar_z Bv,
//   S_z = -2 dPbar_u Bu - 2 dPbar_v Bv
//         - dPbar_z (g sin u du + g sin v dv + 4 e2 cs dz).
// F and M carry the factor eps.  For eps != 0 (EPS0 false) a.eb collects
// eps epsbar, F . Pbar + (M dX) . dPbar with the M dX the undo needs anyway,
// and the kernel divides by eps once at the end.  For eps = 0 (EPS0 true)
// F / eps and M / eps are formed from w2 = 2 t directly.
// Sines and cosines from the same table as the forward kick.
template <bool EPS0>
__device__ __forceinline__ void rev_kick2(Orbit &o, Adjoint2 &a, double a2, double w2,
                                          const double2 *__restrict__ tab) {
  const SinCosT U = sincos_tab(o.x, tab), V = sincos_tab(o.y, tab);
  const ZTerms Z = zterms_tab(o.z, tab);
  const double e1 = a2 * Z.cz2, e2 = a2 * Z.czsz, g = __builtin_fma(2.0, e1, -a2);
  const double cs = U.c + V.c;
  // F, the kick's increment of P.
  const double fu = e1 * U.s, fv = e1 * V.s, fz = e2 * cs;
  const double du = o.dx, dv = o.dy, dz = o.dz;
  const double pub = a.pxb, pvb = a.pyb, pzb = a.pzb;
  const double dpub = a.dpxb, dpvb = a.dpyb, dpzb = a.dpzb;
  // M; its (u, z) and (v, z) entries are 2 mzu and 2 mzv, and every product
  // with them is formed as mzu (2 dz) and the like, exact rescalings by 2.
  const double muu = e1 * U.c, mvv = e1 * V.c;
  const double mzu = -e2 * U.s, mzv = -e2 * V.s, mzz = cs * g;
  const double dz2 = dz + dz;
  // M dX: the tangent kick of the forward step.
  const double mdu = __builtin_fma(muu, du, mzu * dz2);
  const double mdv = __builtin_fma(mvv, dv, mzv * dz2);
  const double mdz = __builtin_fma(mzu, du, __builtin_fma(mzv, dv, mzz * dz));

  if constexpr (EPS0) {
    // epsbar from F / eps and M / eps.
    const double f1 = w2 * Z.cz2, f2 = w2 * Z.czsz, gf = __builtin_fma(2.0, f1, -w2);
    const double wuu = f1 * U.c, wvv = f1 * V.c, wuz = -2.0 * f2 * U.s, wvz = -2.0 * f2 * V.s;
    const double wzu = -f2 * U.s, wzv = -f2 * V.s, wzz = cs * gf;
    double eb = a.eb;
    eb = __builtin_fma(f1, __builtin_fma(U.s, pub, V.s * pvb), eb);
    eb = __builtin_fma(f2 * cs, pzb, eb);
    eb = __builtin_fma(__builtin_fma(wuu, du, wuz * dz), dpub, eb);
    eb = __builtin_fma(__builtin_fma(wvv, dv, wvz * dz), dpvb, eb);
    eb = __builtin_fma(__builtin_fma(wzu, du, __builtin_fma(wzv, dv, wzz * dz)), dpzb, eb);
    a.eb = eb;
  } else {
    // eps epsbar: F . Pbar + (M dX) . dPbar.
    double eb = a.eb;
    eb = __builtin_fma(fu, pub, eb);
    eb = __builtin_fma(fv, pvb, eb);
    eb = __builtin_fma(fz, pzb, eb);
    eb = __builtin_fma(mdu, dpub, eb);
    eb = __builtin_fma(mdv, dpvb, eb);
    eb = __builtin_fma(mdz, dpzb, eb);
    a.eb = eb;
  }

  // Xbar += M^T Pbar + S.
  const double e2cu = e2 * U.c, e2cv = e2 * V.c, gsu = g * U.s, gsv = g * V.s;
  const double Au = __builtin_fma(fu, du, e2cu * dz2);
  const double Av = __builtin_fma(fv, dv, e2cv * dz2);
  const double Bu = __builtin_fma(e2cu, du, gsu * dz);
  const double Bv = __builtin_fma(e2cv, dv, gsv * dz);
  const double Cz = __builtin_fma(gsu, du, __builtin_fma(gsv, dv, fz * (dz2 + dz2)));
  double xb = a.xb, yb = a.yb, zb = a.zb;
  xb = __builtin_fma(muu, pub, __builtin_fma(mzu, pzb, xb));
  yb = __builtin_fma(mvv, pvb, __builtin_fma(mzv, pzb, yb));
  xb = __builtin_fma(-dpub, Au, __builtin_fma(-dpzb, Bu, xb));
  yb = __builtin_fma(-dpvb, Av, __builtin_fma(-dpzb, Bv, yb));
  // The z row: the terms with a factor 2 summed first, then doubled.
  const double zh = __builtin_fma(mzu, pub, __builtin_fma(mzv, pvb, __builtin_fma(-dpub, Bu, -(dpvb * Bv))));
  zb = __builtin_fma(2.0, zh, __builtin_fma(mzz, pzb, __builtin_fma(-dpzb, Cz, zb)));
  a.xb = xb;
  a.yb = yb;
  a.zb = zb;

  // dXbar += M^T dPbar.
  a.dxb = __builtin_fma(muu, dpub, __builtin_fma(mzu, dpzb, a.dxb));
  a.dyb = __builtin_fma(mvv, dpvb, __builtin_fma(mzv, dpzb, a.dyb));
  a.dzb = __builtin_fma(2.0, __builtin_fma(mzu, dpub, mzv * dpvb), __builtin_fma(mzz, dpzb, a.dzb));

  // Undo the kick: dP -= M dX, P -= F.
  o.dpx -= mdu;
  o.dpy -= mdv;
  o.dpz -= mdz;
  o.px = __builtin_fma(-e1, U.s, o.px);
  o.py = __builtin_fma(-e1, V.s, o.py);
  o.pz = __builtin_fma(-e2, cs, o.pz);
}

template <int FORM, bool EPS0>
__device__ __forceinline__ void rev_tan_step(Orbit &o, Adjoint2 &a, const AdjDesc &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
    rev_drift2(o, a, d.drift[F::drift_idx[NK]]);
#pragma unroll
    for (int i = NK - 1; i >= 0; --i) {
      const int u = F::kick_idx[i];
      rev_kick2<EPS0>(o, a, d.ka2[u], d.kw2[u], tab);
      rev_drift2(o, a, d.drift[F::drift_idx[i]]);
    }
  } else {
    rev_drift2(o, a, d.drift[0]);
    rev_kick2<EPS0>(o, a, d.ka2[0], d.kw2[0], tab);
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

// The tangent's norm in the rotated frame of the steps:
// |w|^2 = (du^2 + dv^2 + dp_u^2 + dp_v^2)/2 + dz^2 + dp_z^2.
__device__ __forceinline__ double tan_norm2_rot(const Orbit &o) {
  double a = o.dx * o.dx;
  a = __builtin_fma(o.dy, o.dy, a);
  a = __builtin_fma(o.dpx, o.dpx, a);
  a = __builtin_fma(o.dpy, o.dpy, a);
  const double n2 = __builtin_fma(o.dz, o.dz, o.dpz * o.dpz);
  return __builtin_fma(0.5, a, n2);
}

// dL/dw_T = G w_T / |w_T|^2 in the rotated frame, G = diag(1/2, 1/2, 1, 1/2, 1/2, 1),
// scaled by the upstream gradient gl.
__device__ __forceinline__ void end_condition(const Orbit &o, Adjoint2 &a, double gl) {
  const double c = gl / tan_norm2_rot(o);
  const double h = 0.5 * c;
  a.dxb = h * o.dx; a.dyb = h * o.dy; a.dzb = c * o.dz;
  a.dpxb = h * o.dpx; a.dpyb = h * o.dpy; a.dpzb = c * o.dpz;
}

// The initial-state gradient, back from the rotated frame (d/dx = d/du + d/dv,
// d/dy = d/du - d/dv; momenta alike).
__device__ __forceinline__ void store_grad2(const FtleDesc &d, int64_t n, const Adjoint2 &a) {
  const int64_t N = d.N;
  d.gic[0 * N + n] = a.xb + a.yb;
  d.gic[1 * N + n] = a.xb - a.yb;
  d.gic[2 * N + n] = a.zb;
  d.gic[3 * N + n] = a.pxb + a.pyb;
  d.gic[4 * N + n] = a.pxb - a.pyb;
  d.gic[5 * N + n] = a.pzb;
  d.geps[n] = a.eb;
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
  renorm_rot(t);
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
  to_rot(o);
  for (int64_t s = 0; s < d.n_seg; ++s) {
    store12(d.ckpts + s * 12 * N, N, n, o);
    const int64_t g0 = s * d.ckpt;
    const int64_t g1 = g0 + d.ckpt < d.T ? g0 + d.ckpt : d.T;
    for (int64_t g = g0; g < g1; ++g) {
      tan_step<FORM>(o, d, s_tab);
      if (d.fwd_steps && adj_kept(g, g1)) store12(d.steps + adj_slot(g, 0) * 12 * N, N, n, o);  // one segment
      if (((g + 1) & RESCALE_MASK) == 0) {
        const int k0 = o.kexp;
        renorm_rot(o);
        d.exps[((g + 1) / (RESCALE_MASK + 1) - 1) * N + n] = (int16_t)(o.kexp - k0);
      }
    }
  }
  store12(d.ckpts + d.n_seg * 12 * N, N, n, o);   // the final state (after any last rescale)
  if (d.L) {
    const double n2 = tan_norm2_rot(o);
    const int e = __builtin_amdgcn_frexp_exp(n2);
    const double mant = __builtin_amdgcn_frexp_mant(n2);
    d.L[n] = 0.5 * ((double)(2 * o.kexp + e) * LN2_D + log(mant)) - 0.5 * log(n0);
  }
}

template <int FORM, bool EPS0>
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
    if (!d.fwd_steps) {  // else the forward pass has kept the step states already
      load12(d.ckpts + s * 12 * N, N, n, o);
      for (int64_t g = g0; g < g1; ++g) {
        tan_step<FORM>(o, d, s_tab);
        if (adj_kept(g, g1)) store12(d.steps + adj_slot(g, g0) * 12 * N, N, n, o);
        if (((g + 1) & RESCALE_MASK) == 0) renorm_rot(o);
      }
    }
    for (int64_t g = g1 - 1; g >= g0; --g) {
      // end of step g, before any rescale: kept (every rescale step is kept,
      // since ADJ_SUB divides 8), or rebuilt by the inverse of step g + 1
      if (adj_kept(g, g1)) load12(d.steps + adj_slot(g, g0) * 12 * N, N, n, o);
      if (g == d.T - 1) {
        // dL/dw_T = w_T / |w_T|^2 (scaled by the upstream gradient).
        end_condition(o, a, gl);
      } else if (((g + 1) & RESCALE_MASK) == 0) {
        const int k = rescale_exponent(o);
        a.dxb = __builtin_amdgcn_ldexp(a.dxb, -k);
        a.dyb = __builtin_amdgcn_ldexp(a.dyb, -k);
        a.dzb = __builtin_amdgcn_ldexp(a.dzb, -k);
        a.dpxb = __builtin_amdgcn_ldexp(a.dpxb, -k);
        a.dpyb = __builtin_amdgcn_ldexp(a.dpyb, -k);
        a.dpzb = __builtin_amdgcn_ldexp(a.dpzb, -k);
      }
      rev_tan_step<FORM, EPS0>(o, a, d, s_tab);
    }
  }
  if (!EPS0) a.eb /= d.eps;   // the kicks collected eps epsbar
  store_grad2(d, n, a);
}

template <int FORM, bool EPS0>
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
        end_condition(o, a, gl);
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
      rev_tan_step<FORM, EPS0>(o, a, d, s_tab);   // o: the state at the start of step g
    }
  }
  if (!EPS0) a.eb /= d.eps;   // the kicks collected eps epsbar
  store_grad2(d, n, a);
}

}  // namespace

hipError_t launch_ftle_backward_reversible(const FtleDesc &d, int form, const Tuning &t, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const bool e0 = d.eps == 0.0;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<1, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<1, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 2:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<2, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<2, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 4:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<4, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<4, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 6:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<6, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<6, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 7:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<7, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd_rev<7, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
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
  const bool e0 = d.eps == 0.0;
  const int tb = block_for(t, d.N);
  const unsigned blocks = (unsigned)((d.N + tb - 1) / tb);
  switch (form) {
  case 1:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<1, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<1, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 2:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<2, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<2, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 4:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<4, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<4, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 6:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<6, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<6, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  case 7:
    if (e0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<7, true>), dim3(blocks), dim3(tb), 0, s, d);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ftle_bwd<7, false>), dim3(blocks), dim3(tb), 0, s, d);
    break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aw
