// aw_device.hpp -- device-side arithmetic of the ensemble mapper (gfx950, FP64).
//
// Model (arXiv:1107.4107, eqs. 1-2): H = |P|^2/2 + eps Hp(X),
// Hp = cos x cos y (1 + cos 2z) = 2 cx cy cz^2.
//   grad Hp = (-2 sx cy cz^2, -2 cx sy cz^2, -4 cx cy cz sz)
//   Hess Hp: xx = yy = -2 cx cy cz^2, zz = -4 cx cy (cz^2 - sz^2),
//            xy = 2 sx sy cz^2, xz = 4 sx cy cz sz, yz = 4 cx sy cz sz.
// Kick K(t): P -= t eps grad Hp(X), dP -= t eps Hess(X) dX.
// Drift D(t): X += t P, dX += t dP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aw_sincos_coef.h"
#include "aw_sincos_tab.h"

namespace aw {

// ---------------------------------------------------------------------------
// sin and cos of an unwrapped angle.
// x = q pi + r with q = nearest integer to x/pi (by adding 1.5*2^52, whose
// low mantissa word then holds q), r reduced with a two-part pi: the first
// fused step is exact for |x| < 2^20 pi and the neglected tail of pi adds at
// most 1e-27 to r there.  sin x = (-1)^q sin r, cos x = (-1)^q cos r.  The
// sign (-1)^q is NOT applied here: `par` returns q's low bit in bit 0 so that
// callers can fold signs of products together.
// ---------------------------------------------------------------------------
struct SinCos {
  double c, s;     // cos r, sin r
  uint32_t par;    // low word of (q + 1.5*2^52): bit 0 = q mod 2
};

__device__ __forceinline__ SinCos sincos_red(double x) {
  const double t = __builtin_fma(x, AW_INV_PI, AW_ROUND_MAGIC);
  const double q = t - AW_ROUND_MAGIC;
  double r = __builtin_fma(-q, AW_PI_A, x);
  r = __builtin_fma(-q, AW_PI_B, r);
  const double u = r * r;
  double ps = AW_SIN_C[AW_SIN_NC - 1];
#pragma unroll
  for (int i = AW_SIN_NC - 2; i >= 0; --i) ps = __builtin_fma(ps, u, AW_SIN_C[i]);
  double pc = AW_COS_C[AW_COS_NC - 1];
#pragma unroll
  for (int i = AW_COS_NC - 2; i >= 0; --i) pc = __builtin_fma(pc, u, AW_COS_C[i]);
  SinCos o;
  o.s = __builtin_fma(r * u, ps, r);
  o.c = __builtin_fma(u, pc, 1.0);
  o.par = (uint32_t)__double2loint(t);
  return o;
}

// Flip the sign of v when bit 31 of `sgn` is set.
__device__ __forceinline__ double flip(double v, uint32_t sgn) {
  return __hiloint2double(__double2hiint(v) ^ (int)sgn, __double2loint(v));
}

// FP64 operation counts of one sincos_red (for the roofline accounting).
constexpr int SC_FMA = 1 + 2 + (AW_SIN_NC - 1) + 1 + (AW_COS_NC - 1) + 1;
constexpr int SC_MUL = 2;  // r*r, r*u
constexpr int SC_ADD = 1;  // t - magic

// ---------------------------------------------------------------------------
// Table-driven sin and cos of an unwrapped angle (the propagation and adjoint
// kernels).  x = q pi/2048 + r with q = nearest integer to 2048 x/pi
// (magic-number rounding: the low mantissa word of q + 1.5*2^52 holds q in
// two's complement), r by a two-part Cody-Waite step, |r| <= pi/4096.  With
// k = q mod 4096 and (S, C) = (sin, cos)(k pi/2048) from a 4096-entry table in
// LDS (64 KB):
//   sin x = S cos r + C sin r,  cos x = C cos r - S sin r,
// sin r = r + r^3 c (one coefficient) and cos r = 1 + r^2 Q(r^2) (two).  The
// table carries every quadrant's signs, so the results are the true sine and
// cosine.  The table's byte offset 16 k is the low word of t shifted left by
// 4 and cut to 16 bits, which one SDWA shift does (dst_sel WORD_0 with zero
// padding), so the offset is below 64 KB whatever t holds and the read stays
// inside the table.  Declared as a kernel's first LDS object, the table sits
// at address 0 and the offset is the address.  8 FMA, 4 MUL, 1 ADD, one
// integer instruction and one 16-byte LDS read.
// ---------------------------------------------------------------------------
struct SinCosT {
  double s, c;
};

__device__ __forceinline__ uint32_t tab_offset(double t) {
  uint32_t a;
  asm("v_lshlrev_b32_sdwa %0, 4, %1 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
      : "=v"(a)
      : "v"((uint32_t)__double2loint(t)));
  return a;
}

__device__ __forceinline__ SinCosT sincos_tab(double x, const double2 *__restrict__ tab) {
  const double t = __builtin_fma(x, AW_INV_PI2K, AW_ROUND_MAGIC);
  const double q = t - AW_ROUND_MAGIC;
  double r = __builtin_fma(-q, AW_PI2K_A, x);
  r = __builtin_fma(-q, AW_PI2K_B, r);
  const double2 e = *(const double2 *)((const char *)tab + tab_offset(t));
  const double u = r * r;
  const double sr = __builtin_fma(r * u, AW_TSIN_C0, r);
  const double pc = __builtin_fma(AW_TCOS_C[1], u, AW_TCOS_C[0]);
  const double cr = __builtin_fma(u, pc, 1.0);
  SinCosT o;
  o.s = __builtin_fma(e.x, cr, e.y * sr);
  o.c = __builtin_fma(e.y, cr, -(e.x * sr));
  return o;
}

// FP64 operation counts of one sincos_tab.
constexpr int SCT_FMA = 1 + 2 + 1 + 2 + 2;
constexpr int SCT_MUL = 4;  // r*r, r*u, and one product per rotated output
constexpr int SCT_ADD = 1;

// The z factors of eq. 2's force and Hessian, cos^2 z and cos z sin z, from
// the same table at the doubled angle: cos^2 z = (1 + cos 2z)/2 and
// cos z sin z = sin(2z)/2.  The reduction is sincos_tab's, x = q pi/2048 + r;
// then 2z = 2q pi/2048 + 2r, whose node 2q mod 4096 sits at the low word of t
// shifted by 5 (cut to 16 bits), and two short polynomials in u = r^2 give
// sin(2r)/2 and cos(2r)/2.  9 FMA, 3 MUL, 1 ADD: as many as one sincos_tab,
// in place of the sincos of z and its two products, and no reduction
// constants beyond sincos_tab's.
struct ZTerms {
  double cz2, czsz;
};

__device__ __forceinline__ uint32_t tab_offset2(double t) {
  uint32_t a;
  asm("v_lshlrev_b32_sdwa %0, 5, %1 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
      : "=v"(a)
      : "v"((uint32_t)__double2loint(t)));
  return a;
}

__device__ __forceinline__ ZTerms zterms_tab(double z, const double2 *__restrict__ tab) {
  const double t = __builtin_fma(z, AW_INV_PI2K, AW_ROUND_MAGIC);
  const double q = t - AW_ROUND_MAGIC;
  double r = __builtin_fma(-q, AW_PI2K_A, z);
  r = __builtin_fma(-q, AW_PI2K_B, r);
  const double2 e = *(const double2 *)((const char *)tab + tab_offset2(t));
  const double u = r * r;
  const double sh = __builtin_fma(r * u, AW_ZSIN_C0, r);                           // sin(2r)/2
  const double ph = __builtin_fma(AW_ZCOS_C[1], u, AW_ZCOS_C[0]);
  const double ch = __builtin_fma(u, ph, 0.5);                                     // cos(2r)/2
  ZTerms o;
  o.czsz = __builtin_fma(e.x, ch, e.y * sh);
  o.cz2 = __builtin_fma(e.y, ch, __builtin_fma(-e.x, sh, 0.5));
  return o;
}

constexpr int ZT_FMA = 1 + 2 + 1 + 2 + 3;
constexpr int ZT_MUL = 3;  // r*r, r*u, C*sh
constexpr int ZT_ADD = 1;

// Fill a block's LDS copy of the (sin, cos)(k pi/2048) table; every thread of
// the block must call this before any of them returns.
__device__ __forceinline__ void load_sincos_table(double2 *tab) {
  for (int i = threadIdx.x; i < AW_TAB_N; i += blockDim.x) tab[i] = make_double2(AW_TAB_SC[2 * i], AW_TAB_SC[2 * i + 1]);
  __syncthreads();
}

// True signed cos/sin (used outside the hot loop).
__device__ __forceinline__ void sincos_full(double x, double &s, double &c) {
  SinCos a = sincos_red(x);
  uint32_t sg = a.par << 31;
  s = flip(a.s, sg);
  c = flip(a.c, sg);
}

// Hp(X) = 2 cx cy cz^2.
__device__ __forceinline__ double hp_value(double x, double y, double z) {
  SinCos X = sincos_red(x), Y = sincos_red(y), Z = sincos_red(z);
  uint32_t sg = (X.par ^ Y.par) << 31;
  return flip(2.0 * X.c * Y.c * (Z.c * Z.c), sg);
}

// ---------------------------------------------------------------------------
// Per-orbit register state.
// ---------------------------------------------------------------------------
struct Orbit {
  double x, y, z, px, py, pz;          // state (X unwrapped)
  double dx, dy, dz, dpx, dpy, dpz;    // tangent vector, scaled by 2^-kexp
  double p0x, p0y, p0z;                // initial momentum
  double jsum;                         // sum_k |P_k - P_0|^2
  int kexp;                            // tangent scale exponent (|w| true = |w| 2^kexp)
};

// The propagation kernels run in the rotated frame u = x + y, v = x - y, with
// momenta p_u = p_x + p_y, p_v = p_x - p_y and the tangent transformed alike
// (the Orbit fields x, y, px, py, dx, dy, dpx, dpy then hold u, v, p_u, p_v,
// du, dv, dp_u, dp_v).  The drift keeps its form (u advances by t p_u), and
// eq. 2's H_p = 2 cx cy cz^2 equals (cos u + cos v) cz^2, so the force and its
// Jacobian no longer couple u and v.  With e1 = a2 cz^2, e2 = a2 cz sz
// (a2 = 2 t eps), cs = cos u + cos v:
//   p_u += e1 sin u,  p_v += e1 sin v,  p_z += e2 cs,
//   dp_u += e1 cos u du - 2 e2 sin u dz,
//   dp_v += e1 cos v dv - 2 e2 sin v dz,
//   dp_z += -e2 sin u du - e2 sin v dv + cs (2 e1 - a2) dz.
template <bool TAN>
__device__ __forceinline__ void kick_rot(Orbit &o, double a2, const double2 *__restrict__ tab) {
  const SinCosT U = sincos_tab(o.x, tab), V = sincos_tab(o.y, tab);
  const ZTerms Z = zterms_tab(o.z, tab);
  const double e1 = a2 * Z.cz2;
  const double e2 = a2 * Z.czsz;
  const double cs = U.c + V.c;
  if (TAN) {
    const double k1 = e2 * U.s, k2 = e2 * V.s;
    const double mu = e1 * U.c, mv = e1 * V.c;
    const double mz = cs * __builtin_fma(2.0, e1, -a2);
    const double du = o.dx, dv = o.dy, dz = o.dz;
    const double m2dz = -2.0 * dz;
    o.dpx = __builtin_fma(mu, du, __builtin_fma(k1, m2dz, o.dpx));
    o.dpy = __builtin_fma(mv, dv, __builtin_fma(k2, m2dz, o.dpy));
    o.dpz = __builtin_fma(-k1, du, __builtin_fma(-k2, dv, __builtin_fma(mz, dz, o.dpz)));
  }
  o.px = __builtin_fma(e1, U.s, o.px);
  o.py = __builtin_fma(e1, V.s, o.py);
  o.pz = __builtin_fma(e2, cs, o.pz);
}

template <bool TAN> struct KickRotOps {
  static constexpr int fma = 2 * SCT_FMA + ZT_FMA + 3 + (TAN ? 1 + 7 : 0);
  static constexpr int mul = 2 * SCT_MUL + ZT_MUL + 2 + (TAN ? 4 + 1 + 1 : 0);
  static constexpr int add = 2 * SCT_ADD + ZT_ADD + 1;
};

// Into and out of the rotated frame (p0 alike; the tangent only with TAN).
__device__ __forceinline__ void to_rot(Orbit &o) {
  const double x = o.x, y = o.y, px = o.px, py = o.py;
  o.x = x + y; o.y = x - y;
  o.px = px + py; o.py = px - py;
  const double p0x = o.p0x, p0y = o.p0y;
  o.p0x = p0x + p0y; o.p0y = p0x - p0y;
  const double dx = o.dx, dy = o.dy, dpx = o.dpx, dpy = o.dpy;
  o.dx = dx + dy; o.dy = dx - dy;
  o.dpx = dpx + dpy; o.dpy = dpx - dpy;
}

// Back to the original frame, as displacements from the initial state s0
// (x, y, z, px, py, pz), whose rotated form is recomputed here exactly as
// to_rot formed it: what the steps did not change comes back unchanged (at
// eps = 0 the momenta exactly).
__device__ __forceinline__ void from_rot(Orbit &o, const double (&s0)[6]) {
#pragma clang fp contract(off)
  const double du0 = o.x - (s0[0] + s0[1]), dv0 = o.y - (s0[0] - s0[1]);
  const double dpu0 = o.px - (s0[3] + s0[4]), dpv0 = o.py - (s0[3] - s0[4]);
  o.x = s0[0] + 0.5 * (du0 + dv0); o.y = s0[1] + 0.5 * (du0 - dv0);
  o.px = s0[3] + 0.5 * (dpu0 + dpv0); o.py = s0[4] + 0.5 * (dpu0 - dpv0);
  const double du = o.dx, dv = o.dy, dpu = o.dpx, dpv = o.dpy;
  o.dx = 0.5 * (du + dv); o.dy = 0.5 * (du - dv);
  o.dpx = 0.5 * (dpu + dpv); o.dpy = 0.5 * (dpu - dpv);
}

// In the rotated frame |P - P0|^2 = (du_p^2 + dv_p^2)/2 + dz_p^2: jsum collects
// twice the step sum, (P_u - P0_u)^2 + (P_v - P0_v)^2 + 2 (P_z - P0_z)^2.
__device__ __forceinline__ void accum_j_rot(Orbit &o) {
  const double eu = o.px - o.p0x, ev = o.py - o.p0y, ez = o.pz - o.p0z;
  const double ez2 = ez + ez;
  o.jsum = __builtin_fma(eu, eu, o.jsum);
  o.jsum = __builtin_fma(ev, ev, o.jsum);
  o.jsum = __builtin_fma(ez, ez2, o.jsum);
}

template <bool TAN>
__device__ __forceinline__ void drift(Orbit &o, double t) {
  o.x = __builtin_fma(t, o.px, o.x);
  o.y = __builtin_fma(t, o.py, o.y);
  o.z = __builtin_fma(t, o.pz, o.z);
  if (TAN) {
    o.dx = __builtin_fma(t, o.dpx, o.dx);
    o.dy = __builtin_fma(t, o.dpy, o.dy);
    o.dz = __builtin_fma(t, o.dpz, o.dz);
  }
}

// Op counts of kick/drift (roofline accounting).
template <bool TAN> struct DriftOps {
  static constexpr int fma = TAN ? 6 : 3;
};

// Rescale the tangent by an exact power of two so that |w|^2 lies in
// [0.5, 2); the scale is accumulated in kexp.  Exact: it changes no mantissa.
// In the rotated frame the tangent's true norm is
// |w|^2 = (du^2 + dv^2 + dp_u^2 + dp_v^2)/2 + dz^2 + dp_z^2.
__device__ __forceinline__ void renorm_rot(Orbit &o) {
  double a = o.dx * o.dx;
  a = __builtin_fma(o.dy, o.dy, a);
  a = __builtin_fma(o.dpx, o.dpx, a);
  a = __builtin_fma(o.dpy, o.dpy, a);
  double n2 = __builtin_fma(o.dz, o.dz, o.dpz * o.dpz);
  n2 = __builtin_fma(0.5, a, n2);
  const int e = __builtin_amdgcn_frexp_exp(n2);
  const int s = e >> 1;
  o.dx = __builtin_amdgcn_ldexp(o.dx, -s);
  o.dy = __builtin_amdgcn_ldexp(o.dy, -s);
  o.dz = __builtin_amdgcn_ldexp(o.dz, -s);
  o.dpx = __builtin_amdgcn_ldexp(o.dpx, -s);
  o.dpy = __builtin_amdgcn_ldexp(o.dpy, -s);
  o.dpz = __builtin_amdgcn_ldexp(o.dpz, -s);
  o.kexp += s;
}

// ---------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea & Flood 2014): output number c of the
// stream seeded with `seed` is mix(seed + (c + 1) * 0x9E3779B97F4A7C15).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double u01(uint64_t seed, uint64_t c) {
  return (double)(splitmix64(seed, c) >> 11) * 0x1.0p-53;
}

}  // namespace aw
