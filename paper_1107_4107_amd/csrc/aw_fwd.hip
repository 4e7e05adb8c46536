// aw_fwd.hip -- ensemble propagation kernels (gfx950, FP64).
//
// One orbit per lane (or two, interleaved, for instruction-level
// parallelism; or, for small tangent-free ensembles, one orbit on two lanes);
// the state, the tangent vector and the accumulators stay in
// VGPRs for the whole run; initial conditions are generated in registers from
// the ensemble descriptor, so the only HBM traffic is the coalesced
// structure-of-arrays store of the per-orbit results (and of the resumable
// carry when a run is split into several launches).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "aw_device.hpp"
#include "aw_internal.hpp"
#include "aw_launch.hpp"

namespace aw {

// ---------------------------------------------------------------------------
// Initial conditions and tangent start.  GRID2, BOX, EXPLICIT and the tangent
// start use exact or correctly rounded operations only, so the values are
// bitwise those of any IEEE implementation of the same formulas; SPHERE also
// takes a cosine, a sine and Hp(X), so it agrees to a few ulps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gen_ic(const FwdDesc &d, int64_t n, double s[6]) {
#pragma clang fp contract(off)
  if (d.ic_kind == 0) {
    const int64_t i = n % d.nx, j = n / d.nx;
    const double v0 = d.lo0 + (double)i * d.d0;
    const double v1 = d.lo1 + (double)j * d.d1;
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = (k == d.ax0) ? v0 : ((k == d.ax1) ? v1 : d.base[k]);
  } else if (d.ic_kind == 1) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      s[k] = d.box_lo[k] + d.box_span[k] * u01(d.seed_ic, 16ull * (uint64_t)n + (uint64_t)k);
  } else if (d.ic_kind == 3) {
    // Fixed energy: X on the torus, direction uniform in area on the (phi, mu)
    // segment, |P| from H(P, X) = E.
    const uint64_t c = 16ull * (uint64_t)n;
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = d.box_lo[k] + d.box_span[k] * u01(d.seed_ic, c + (uint64_t)k);
    const double mu = d.win[2] + (d.win[3] - d.win[2]) * u01(d.seed_ic, c + 3ull);
    const double phi = d.win[0] + (d.win[1] - d.win[0]) * u01(d.seed_ic, c + 4ull);
    const double st = sqrt(1.0 - mu * mu);
    const double p = sqrt(2.0 * (d.energy - d.eps * hp_value(s[0], s[1], s[2])));
    double sp, cp;
    sincos_full(phi, sp, cp);
    s[3] = p * st * cp;
    s[4] = p * st * sp;
    s[5] = p * mu;
  } else if (d.ic_kind == 4) {
    // Fig. 4 cloud: Gaussian (vx, vy) by Box-Muller, X on the torus by
    // rejection until the energy condition leaves a real vz.
    const uint64_t c = 128ull * (uint64_t)n;
    const double u1 = u01(d.seed_ic, c + 120ull), u2 = u01(d.seed_ic, c + 121ull);
    const double rr = sqrt(-2.0 * log(1.0 - u1));
    double sg, cg;
    sincos_full(2.0 * M_PI * u2, sg, cg);
    const double vx = d.cloud[0] + d.cloud[2] * (rr * cg);
    const double vy = d.cloud[1] + d.cloud[3] * (rr * sg);
    double R = -1.0;
    for (int a = 0; a < 40 && R < 0.0; ++a) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        s[k] = d.box_lo[k] + d.box_span[k] * u01(d.seed_ic, c + 3ull * (uint64_t)a + (uint64_t)k);
      R = 2.0 * (d.energy - d.eps * hp_value(s[0], s[1], s[2])) - vx * vx - vy * vy;
    }
    const double vz = sqrt(R > 0.0 ? R : 0.0);
    s[3] = vx;
    s[4] = vy;
    s[5] = u01(d.seed_ic, c + 122ull) < 0.5 ? -vz : vz;
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = d.ic[k * d.N + n];
  }
}

__device__ __forceinline__ void gen_w0(uint64_t seed, int64_t n, double w[6]) {
#pragma clang fp contract(off)
  double u[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) u[k] = 2.0 * u01(seed, 16ull * (uint64_t)n + (uint64_t)k) - 1.0;
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) n2 = n2 + u[k] * u[k];
  const double nu = sqrt(n2);
#pragma unroll
  for (int k = 0; k < 6; ++k) w[k] = u[k] / nu;
}

// ---------------------------------------------------------------------------
// One map step: NK kicks, each preceded by a drift, and a closing drift
// (symmetric compositions), or kick-then-drift (coupled standard map).  The
// kicks take their sines and cosines from the block's LDS table `tab`.
// ---------------------------------------------------------------------------
// The distinct stage weights of the form, copied from the descriptor before
// the step loop.
// Stage weights of the rotated-frame step: the drift's t and the kick's
// a2 = 2 t eps (the kick needs no other weight there).
struct StepWeights {
  double drift[MAX_UNIQUE];
  double ka2[MAX_UNIQUE];
};

template <int FORM, bool TAN, int OPL>
__device__ __forceinline__ void map_step(Orbit (&o)[OPL], const StepWeights &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
#pragma unroll
      for (int j = 0; j < OPL; ++j) drift<TAN>(o[j], d.drift[F::drift_idx[i]]);
#pragma unroll
      for (int j = 0; j < OPL; ++j) kick_rot<TAN>(o[j], d.ka2[F::kick_idx[i]], tab);
    }
#pragma unroll
    for (int j = 0; j < OPL; ++j) drift<TAN>(o[j], d.drift[F::drift_idx[NK]]);
  } else {
#pragma unroll
    for (int j = 0; j < OPL; ++j) kick_rot<TAN>(o[j], d.ka2[0], tab);
#pragma unroll
    for (int j = 0; j < OPL; ++j) drift<TAN>(o[j], d.drift[0]);
  }
}

// Select row r of the nine per-orbit results by masking bit patterns.  A
// chain of selects over the array's elements is folded by the optimizer into
// one load at a selected offset, which keeps the array in memory (private
// scratch, or LDS sized for the whole block); AND/OR of the bits leaves
// nothing to fold.
__device__ __forceinline__ double pick9(const double (&v)[9], int r) {
  uint64_t o = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) o |= (uint64_t)__double_as_longlong(v[k]) & (0ull - (uint64_t)(r == k));
  return __longlong_as_double((long long)o);
}

__device__ __forceinline__ uint32_t bin_of(double a, double b, double lo0, double hi0, double lo1,
                                           double hi1, int W, int H, bool closed) {
#pragma clang fp contract(off)
  if (!isfinite(a) || !isfinite(b)) return BIN_DROP;
  double fi = floor((a - lo0) / (hi0 - lo0) * (double)W);
  double fj = floor((b - lo1) / (hi1 - lo1) * (double)H);
  if (closed) {
    if (fi == (double)W && a == hi0) fi = (double)(W - 1);
    if (fj == (double)H && b == hi1) fj = (double)(H - 1);
  }
  if (!(fi >= 0.0) || fi >= (double)W || !(fj >= 0.0) || fj >= (double)H) return BIN_DROP;
  return (uint32_t)fj * (uint32_t)W + (uint32_t)fi;
}

__device__ __forceinline__ void vdir_key(double vx, double vy, double vz, double &phi, double &mu) {
#pragma clang fp contract(off)
  const double r = sqrt(vx * vx + vy * vy + vz * vz);
  if (r == 0.0) {
    phi = __builtin_nan("");
    mu = __builtin_nan("");
    return;
  }
  phi = atan2(vy, vx);
  mu = vz / r;
}

constexpr double LN2 = 0x1.62e42fefa39efp-1;

// Is the direction of P inside the closed window phi in [phi_lo, phi_hi],
// mu = pz/|P| in [mu_lo, mu_hi]?  The phi test uses half-plane (cross
// product) tests against the edge directions e0, e1 instead of atan2: for a
// window of width w <= pi, phi is inside iff e0 x d >= 0 and d x e1 >= 0; for
// w > pi, iff d is not strictly inside the complementary sector.
__device__ __forceinline__ bool in_window(double px, double py, double pz, const FwdDesc &d) {
#pragma clang fp contract(off)
  bool ok = true;
  if (d.win_phi != 0) {
    const double c0 = d.e0x * py - d.e0y * px;   // e0 x d
    const double c1 = px * d.e1y - py * d.e1x;   // d x e1
    ok = d.win_phi == 1 ? (c0 >= 0.0 && c1 >= 0.0) : !(c0 < 0.0 && c1 < 0.0);
  }
  if (d.win_mu != 0) {
    const double r = sqrt(px * px + py * py + pz * pz);
    ok = ok && pz >= d.win[2] * r && pz <= d.win[3] * r;
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Run the orbits first + j*blockDim.x + threadIdx.x (j < OPL) over global
// steps [k_begin, k_end).  FILT: test the window after every step.  `tab` is
// the block's LDS copy of the sine/cosine table (filled by the caller).
// ---------------------------------------------------------------------------
template <int FORM, bool TAN, int OPL, int UNR, bool FILT = false, bool WINV = false>
__device__ __forceinline__ void run_orbits(const FwdDesc &d, int64_t first, const double2 *__restrict__ tab) {
  int64_t n[OPL];
  bool act[OPL];
#pragma unroll
  for (int j = 0; j < OPL; ++j) {
    const int64_t m = first + (int64_t)j * blockDim.x + threadIdx.x;
    act[j] = m < d.N;
    n[j] = act[j] ? m : d.N - 1;  // inactive slots repeat a valid orbit, never stored
  }
  if (!act[0]) return;

  Orbit o[OPL];
  bool left[OPL];
#pragma unroll
  for (int j = 0; j < OPL; ++j) {
    left[j] = false;
    if (d.k_begin == 0) {
      double s[6];
      gen_ic(d, n[j], s);
      o[j].x = s[0]; o[j].y = s[1]; o[j].z = s[2];
      o[j].px = s[3]; o[j].py = s[4]; o[j].pz = s[5];
      o[j].p0x = s[3]; o[j].p0y = s[4]; o[j].p0z = s[5];
      o[j].jsum = 0.0;
      o[j].kexp = 0;
      if (TAN) {
        double w[6];
        gen_w0(d.seed_tan, n[j], w);
        o[j].dx = w[0]; o[j].dy = w[1]; o[j].dz = w[2];
        o[j].dpx = w[3]; o[j].dpy = w[4]; o[j].dpz = w[5];
      } else {
        o[j].dx = o[j].dy = o[j].dz = o[j].dpx = o[j].dpy = o[j].dpz = 0.0;
      }
      if (FILT) left[j] = !in_window(s[3], s[4], s[5], d);
      to_rot(o[j]);
    } else {
      // The carry holds the rotated-frame state as the loop left it.
      const double *c = d.carry;
      const int64_t N = d.N, m = n[j];
      o[j].x = c[0 * N + m]; o[j].y = c[1 * N + m]; o[j].z = c[2 * N + m];
      o[j].px = c[3 * N + m]; o[j].py = c[4 * N + m]; o[j].pz = c[5 * N + m];
      o[j].dx = c[6 * N + m]; o[j].dy = c[7 * N + m]; o[j].dz = c[8 * N + m];
      o[j].dpx = c[9 * N + m]; o[j].dpy = c[10 * N + m]; o[j].dpz = c[11 * N + m];
      o[j].p0x = c[15 * N + m]; o[j].p0y = c[16 * N + m]; o[j].p0z = c[17 * N + m];
      o[j].jsum = c[18 * N + m];
      o[j].kexp = (int)c[19 * N + m];
      if (FILT) left[j] = c[21 * N + m] != 0.0;
    }
  }

  // Positions at the start of this launch (time-window velocity; rotated).
  double xs[OPL], ys[OPL], zs[OPL];
  if (WINV) {
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
      xs[j] = o[j].x;
      ys[j] = o[j].y;
      zs[j] = o[j].z;
    }
  }

  // Hot loop.  The trip count and the renormalisation test are uniform.
  // UNR = 2 runs steps in pairs plus a one-step tail, written out: the table
  // offset is inline assembly, which the compiler treats as convergent and
  // will not unroll with a remainder.
  const int64_t k0 = d.k_begin, k1 = d.k_end;
  const int64_t mask = d.renorm_mask;
  // Stage weights.  In the plain tangent kernel the kick weights move into
  // VGPRs (an empty asm the compiler must treat as producing per-lane
  // values): across the loop the descriptor fields of the epilogue hold most
  // SGPRs, and kick weights left there are spilled to VGPR lanes and read back
  // with v_readlane every step, 16 VALU instructions per S6 step and 32 per Y6
  // step.  In VGPRs they cost 8 registers and no instruction.  The
  // unrolled, two-orbit and window variants would lose occupancy and keep
  // them in SGPRs.
  constexpr bool kVregW = TAN && OPL == 1 && UNR == 1 && !FILT && !WINV;
  StepWeights sw;
#pragma unroll
  for (int q = 0; q < MAX_UNIQUE; ++q) {
    sw.drift[q] = d.drift[q];
    sw.ka2[q] = d.ka2[q];
    if (kVregW) {
      asm volatile("" : "+v"(sw.drift[q]));
      asm volatile("" : "+v"(sw.ka2[q]));
    }
  }
  auto one_step = [&](int64_t k) {
    map_step<FORM, TAN, OPL>(o, sw, tab);
#pragma unroll
    for (int j = 0; j < OPL; ++j) accum_j_rot(o[j]);
    if (FILT) {
      // 2 P in the original frame, exactly: the window test depends only on
      // the direction of P.
#pragma unroll
      for (int j = 0; j < OPL; ++j)
        left[j] = left[j] || !in_window(o[j].px + o[j].py, o[j].px - o[j].py, o[j].pz + o[j].pz, d);
    }
    if (TAN && ((k + 1) & mask) == 0) {
#pragma unroll
      for (int j = 0; j < OPL; ++j) renorm_rot(o[j]);
    }
  };
  int64_t k = k0;
  if (UNR == 2) {
#pragma nounroll
    for (; k + 1 < k1; k += 2) {
      one_step(k);
      one_step(k + 1);
    }
  }
#pragma nounroll
  for (; k < k1; ++k) one_step(k);

  if (k1 < d.T || WINV) {
    // Intermediate launch (or a time window): store the resumable carry.
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
      if (!act[j]) continue;
      if (WINV) {
#pragma clang fp contract(off)
        double phi, mu;
        const double du = o[j].x - xs[j], dv = o[j].y - ys[j];
        vdir_key(0.5 * (du + dv) / d.wdt, 0.5 * (du - dv) / d.wdt, (o[j].z - zs[j]) / d.wdt, phi, mu);
        d.bins[n[j]] = left[j] ? BIN_DROP : bin_of(phi, mu, d.klo0, d.khi0, d.klo1, d.khi1, d.W, d.H, true);
      }
      double *c = d.carry;
      const int64_t N = d.N, m = n[j];
      double s0[6];
      gen_ic(d, m, s0);
      c[0 * N + m] = o[j].x; c[1 * N + m] = o[j].y; c[2 * N + m] = o[j].z;
      c[3 * N + m] = o[j].px; c[4 * N + m] = o[j].py; c[5 * N + m] = o[j].pz;
      c[6 * N + m] = o[j].dx; c[7 * N + m] = o[j].dy; c[8 * N + m] = o[j].dz;
      c[9 * N + m] = o[j].dpx; c[10 * N + m] = o[j].dpy; c[11 * N + m] = o[j].dpz;
      c[12 * N + m] = s0[0]; c[13 * N + m] = s0[1]; c[14 * N + m] = s0[2];
      c[15 * N + m] = o[j].p0x; c[16 * N + m] = o[j].p0y; c[17 * N + m] = o[j].p0z;
      c[18 * N + m] = o[j].jsum;
      c[19 * N + m] = (double)o[j].kexp;
      c[20 * N + m] = (double)k1;
      c[21 * N + m] = left[j] ? 1.0 : 0.0;
    }
    return;
  }

  // Final launch: per-orbit observables.  Contraction is off so that every
  // kernel variant rounds the sums of products below (L, dP^2, the energies)
  // the same way: whether the compiler fuses a*b + c depends on the code
  // around it, and the results are to be bitwise independent of the launch
  // shape and of batching.
  uint32_t n_chaotic = 0;
#pragma unroll
  for (int j = 0; j < OPL; ++j) {
#pragma clang fp contract(off)
    const int64_t N = d.N, m = n[j];
    double s0[6];
    gen_ic(d, m, s0);
    from_rot(o[j], s0);
    double res[9];
    double wn = 1.0;
    if (TAN) {
      double n2 = o[j].dx * o[j].dx;
      n2 = __builtin_fma(o[j].dy, o[j].dy, n2);
      n2 = __builtin_fma(o[j].dz, o[j].dz, n2);
      n2 = __builtin_fma(o[j].dpx, o[j].dpx, n2);
      n2 = __builtin_fma(o[j].dpy, o[j].dpy, n2);
      n2 = __builtin_fma(o[j].dpz, o[j].dpz, n2);
      const int e = __builtin_amdgcn_frexp_exp(n2);
      const double mant = __builtin_amdgcn_frexp_mant(n2);
      const double L = 0.5 * ((double)(2 * o[j].kexp + e) * LN2 + log(mant));
      res[0] = L;
      res[1] = L / d.th;
      res[2] = L / d.lth;
      wn = sqrt(n2);
    } else {
      res[0] = res[1] = res[2] = __builtin_nan("");
    }
    res[3] = (o[j].x - s0[0]) / d.th;
    res[4] = (o[j].y - s0[1]) / d.th;
    res[5] = (o[j].z - s0[2]) / d.th;
    const double ex = o[j].px - s0[3], ey = o[j].py - s0[4], ez = o[j].pz - s0[5];
    res[6] = ex * ex + ey * ey + ez * ez;
    res[7] = (0.5 * o[j].jsum) / (double)d.T;
    const double E1 = 0.5 * (o[j].px * o[j].px + o[j].py * o[j].py + o[j].pz * o[j].pz) +
                      d.eps * hp_value(o[j].x, o[j].y, o[j].z);
    const double E0 = 0.5 * (s0[3] * s0[3] + s0[4] * s0[4] + s0[5] * s0[5]) +
                      d.eps * hp_value(s0[0], s0[1], s0[2]);
    res[8] = E1 - E0;
    const bool chaotic = TAN && (res[2] > d.chi_thr);
    n_chaotic += (uint32_t)__popcll(__ballot(act[j] && chaotic));
    if (!act[j]) continue;
    if (d.out) {
      double *out = d.out;
      out[0 * N + m] = res[0]; out[1 * N + m] = res[1]; out[2 * N + m] = res[2];
      out[3 * N + m] = res[3]; out[4 * N + m] = res[4]; out[5 * N + m] = res[5];
      out[6 * N + m] = res[6]; out[7 * N + m] = res[7]; out[8 * N + m] = res[8];
    }
    if (d.state) {
      double *st = d.state;
      st[0 * N + m] = o[j].x; st[1 * N + m] = o[j].y; st[2 * N + m] = o[j].z;
      st[3 * N + m] = o[j].px; st[4 * N + m] = o[j].py; st[5 * N + m] = o[j].pz;
      st[6 * N + m] = o[j].dx / wn; st[7 * N + m] = o[j].dy / wn; st[8 * N + m] = o[j].dz / wn;
      st[9 * N + m] = o[j].dpx / wn; st[10 * N + m] = o[j].dpy / wn; st[11 * N + m] = o[j].dpz / wn;
    }
    if (d.cls) d.cls[m] = (uint8_t)((chaotic ? 1 : 0) | (left[j] ? 2 : 0));
    if (d.epi == EPI_IC_GRID) {
      d.img[m] = pick9(res, d.field);
    } else if (d.epi == EPI_HIST_P0) {
      double a = s0[0], b = s0[0];
#pragma unroll
      for (int k = 1; k < 6; ++k) {
        a = (d.key0 == k) ? s0[k] : a;
        b = (d.key1 == k) ? s0[k] : b;
      }
      d.bins[m] = left[j] ? BIN_DROP : bin_of(a, b, d.klo0, d.khi0, d.klo1, d.khi1, d.W, d.H, false);
      d.vals[m] = pick9(res, d.field);
    } else if (d.epi == EPI_HIST_VDIR) {
      double phi, mu;
      vdir_key(res[3], res[4], res[5], phi, mu);
      d.bins[m] = left[j] ? BIN_DROP : bin_of(phi, mu, d.klo0, d.khi0, d.klo1, d.khi1, d.W, d.H, true);
    }
  }
  // Class count of the IC-grid image: one ballot and popcount per wave and
  // slot (above), one atomic per wave from its lowest active lane.
  if (d.epi == EPI_IC_GRID && d.n_class != nullptr && TAN) {
    const uint64_t active = __ballot(1);
    if ((int)__lane_id() == __ffsll((unsigned long long)active) - 1 && n_chaotic != 0)
      atomicAdd(d.n_class, n_chaotic);
  }
}

// Blocks of up to 512 lanes: with the 64 KB table two blocks share a CU, and
// at four waves per SIMD it takes blocks of 512 to fill it.  The one-orbit
// tangent kernels of the sixth-order maps take 129 VGPRs, one block per CU:
// two waves per SIMD already saturate the VALU issue, and holding them to 128
// would cost the single-wave schedule its parallelism (a sixth longer on
// small ensembles).  The window-test and time-window variants hold about twice the
// registers and keep 256.
template <int FORM, bool TAN, int OPL, int UNR, bool FILT = false, bool WINV = false>
__global__ __launch_bounds__((FILT || WINV) ? 256 : 512) void k_fwd(FwdDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * OPL;
  run_orbits<FORM, TAN, OPL, UNR, FILT, WINV>(d, first, s_tab);
}

// ---------------------------------------------------------------------------
// Two lanes per orbit, for tangent-free ensembles too small to give every
// SIMD a wave at one lane per orbit (Fig. 4's 3.2e4 orbits make 500 waves for
// 1024 SIMDs).  In the rotated frame the force does not couple u and v, so
// lane 2m of a pair holds u and p_u and lane 2m + 1 holds v and p_v, and both
// hold z and p_z.  A kick takes one table sine and cosine of the lane's own
// coordinate and the z factors, swaps the cosine with the partner lane
// (cs = cos u + cos v is the same sum in both lanes: IEEE addition commutes),
// and advances the lane's own momentum and p_z; a drift advances the lane's
// coordinate and z.  Every value is formed and rounded as in run_orbits, so
// the states, carries and window bins are bitwise those of one lane per
// orbit.  Intermediate and time-window launches only: the final epilogue and
// the window test run one lane per orbit.
// ---------------------------------------------------------------------------
// Lanes 2m and 2m + 1 exchange v (DPP quad_perm [1, 0, 3, 2] on both halves).
// Every lane of the wave takes part: lanes past the ensemble's end repeat a
// valid orbit.
__device__ __forceinline__ double swap_pair(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

struct HalfOrbit {
  double w, pw;    // own rotated coordinate (u or v) and its momentum
  double z, pz;
  double p0w, p0z;
  double jsum;     // meaningful in the pair's even lane
};

__device__ __forceinline__ void pair_kick(HalfOrbit &h, double a2, const double2 *__restrict__ tab) {
  const SinCosT W = sincos_tab(h.w, tab);
  const ZTerms Z = zterms_tab(h.z, tab);
  const double e1 = a2 * Z.cz2;
  const double e2 = a2 * Z.czsz;
  const double cs = W.c + swap_pair(W.c);
  h.pw = __builtin_fma(e1, W.s, h.pw);
  h.pz = __builtin_fma(e2, cs, h.pz);
}

__device__ __forceinline__ void pair_drift(HalfOrbit &h, double t) {
  h.w = __builtin_fma(t, h.pw, h.w);
  h.z = __builtin_fma(t, h.pz, h.z);
}

template <int FORM>
__device__ __forceinline__ void pair_step(HalfOrbit &h, const StepWeights &d, const double2 *__restrict__ tab) {
  using F = FormPattern<FORM>;
  constexpr int NK = F::NK;
  if constexpr (F::LEAD) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      pair_drift(h, d.drift[F::drift_idx[i]]);
      pair_kick(h, d.ka2[F::kick_idx[i]], tab);
    }
    pair_drift(h, d.drift[F::drift_idx[NK]]);
  } else {
    pair_kick(h, d.ka2[0], tab);
    pair_drift(h, d.drift[0]);
  }
}

template <int FORM, bool WINV>
__global__ __launch_bounds__(256) void k_fwd_pair(FwdDesc d) {
  __shared__ double2 s_tab[AW_TAB_N];
  load_sincos_table(s_tab);
  const int64_t m0 = (int64_t)blockIdx.x * (blockDim.x >> 1) + (threadIdx.x >> 1);
  const bool act = m0 < d.N;
  const int64_t m = act ? m0 : d.N - 1;   // past the end: repeat a valid orbit, never stored
  const bool odd = (threadIdx.x & 1u) != 0;
  const int64_t N = d.N;
  HalfOrbit h;
  if (d.k_begin == 0) {
#pragma clang fp contract(off)
    double s[6];
    gen_ic(d, m, s);
    h.w = odd ? s[0] - s[1] : s[0] + s[1];
    h.pw = odd ? s[3] - s[4] : s[3] + s[4];
    h.z = s[2];
    h.pz = s[5];
    h.p0w = h.pw;
    h.p0z = s[5];
    h.jsum = 0.0;
  } else {
    const double *c = d.carry;
    const int64_t r = odd ? 1 : 0;
    h.w = c[(0 + r) * N + m];
    h.pw = c[(3 + r) * N + m];
    h.z = c[2 * N + m];
    h.pz = c[5 * N + m];
    h.p0w = c[(15 + r) * N + m];
    h.p0z = c[17 * N + m];
    h.jsum = c[18 * N + m];
  }
  const double ws = h.w, zs = h.z;
  StepWeights sw;
#pragma unroll
  for (int q = 0; q < MAX_UNIQUE; ++q) {
    sw.drift[q] = d.drift[q];
    sw.ka2[q] = d.ka2[q];
  }
#pragma nounroll
  for (int64_t k = d.k_begin; k < d.k_end; ++k) {
    pair_step<FORM>(h, sw, s_tab);
    // J as run_orbits accumulates it, in the even lane: (p_u - p0_u)^2, then
    // (p_v - p0_v)^2, then twice (p_z - p0_z)^2.
    const double e = h.pw - h.p0w;
    const double ep = swap_pair(e);
    const double ez = h.pz - h.p0z;
    const double ez2 = ez + ez;
    h.jsum = __builtin_fma(e, e, h.jsum);
    h.jsum = __builtin_fma(ep, ep, h.jsum);
    h.jsum = __builtin_fma(ez, ez2, h.jsum);
  }
  const double dw = h.w - ws;
  const double dwp = swap_pair(dw);   // the partner's displacement
  if (!act) return;
  double *c = d.carry;
  if (odd) {
    c[1 * N + m] = h.w;
    c[4 * N + m] = h.pw;
    c[16 * N + m] = h.p0w;
    return;
  }
  if (WINV) {
#pragma clang fp contract(off)
    double phi, mu;
    const double du = dw, dv = dwp;
    vdir_key(0.5 * (du + dv) / d.wdt, 0.5 * (du - dv) / d.wdt, (h.z - zs) / d.wdt, phi, mu);
    d.bins[m] = bin_of(phi, mu, d.klo0, d.khi0, d.klo1, d.khi1, d.W, d.H, true);
  }
  c[0 * N + m] = h.w;
  c[2 * N + m] = h.z;
  c[3 * N + m] = h.pw;
  c[5 * N + m] = h.pz;
  c[15 * N + m] = h.p0w;
  c[17 * N + m] = h.p0z;
  c[18 * N + m] = h.jsum;
  c[20 * N + m] = (double)d.k_end;
  if (d.k_begin == 0) {
    // what a first launch of run_orbits writes for a tangent-free orbit
    double s0[6];
    gen_ic(d, m, s0);
#pragma unroll
    for (int r = 6; r < 12; ++r) c[r * N + m] = 0.0;
    c[12 * N + m] = s0[0]; c[13 * N + m] = s0[1]; c[14 * N + m] = s0[2];
    c[19 * N + m] = 0.0;
  }
  c[21 * N + m] = 0.0;   // no window test here
}

// Persistent batched propagation: each workgroup takes (ensemble, tile)
// items from a device counter until the list, sorted longest-first, is empty.
// Two orbits per lane take about 266 VGPRs in the rotated frame; held to 256
// (two waves per SIMD instead of one, the spills outside the step loop) the
// batch runs a fifth faster.
template <int FORM, bool TAN, int OPL>
__global__ __launch_bounds__(256, OPL > 1 ? 2 : 1) void k_fwd_persist(const FwdDesc *__restrict__ descs,
                                                     const WorkItem *__restrict__ items,
                                                     int32_t n_items, uint32_t *head) {
  __shared__ double2 s_tab[AW_TAB_N];
  __shared__ int32_t s_item;
  load_sincos_table(s_tab);
  for (;;) {
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(head, 1u);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const int32_t e = __builtin_amdgcn_readfirstlane(items[it].ens);
    const int64_t first = items[it].first;
    run_orbits<FORM, TAN, OPL, 1>(descs[e], first, s_tab);
  }
}

__global__ void k_zero_u32(uint32_t *p, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_gen_ic(FwdDesc d, double *ic, double *w0) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= d.N) return;
  double s[6];
  if (ic) {
    gen_ic(d, n, s);
#pragma unroll
    for (int k = 0; k < 6; ++k) ic[k * d.N + n] = s[k];
  }
  if (w0) {
    gen_w0(d.seed_tan, n, s);
#pragma unroll
    for (int k = 0; k < 6; ++k) w0[k * d.N + n] = s[k];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
int block_for(const Tuning &t, int64_t n) {
  if (t.block) return t.block;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    ncu = 256;
  int b = 512;
  while (b > 64 && (int64_t)b * ncu > n) b >>= 1;
  return b;
}

// Two lanes per orbit: tangent-free intermediate or time-window launches
// without the window test, when asked for (lanes_per_orbit 2) or, by
// default, when one lane per orbit would leave SIMDs without a wave.
static bool use_pair(const FwdDesc &d, const Tuning &t, bool tan) {
  if (tan || d.filter || !(d.window_v || d.k_end < d.T) || d.N <= 0) return false;
  if (t.lpo) return t.lpo == 2;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    ncu = 256;
  return d.N < (int64_t)ncu * 4 * 64;
}

template <int FORM, bool TAN>
static hipError_t fwd_dispatch_opl(const FwdDesc &d, const Tuning &t, hipStream_t s) {
  if (use_pair(d, t, TAN)) {
    // 128 orbits (four waves) per block: with the 64 KB table two blocks share
    // a CU, so a block must bring a wave for each of the CU's four SIMDs.
    const dim3 grid((unsigned)((d.N + 127) / 128));
    if (d.window_v) hipLaunchKernelGGL((k_fwd_pair<FORM, true>), grid, dim3(256), 0, s, d);
    else hipLaunchKernelGGL((k_fwd_pair<FORM, false>), grid, dim3(256), 0, s, d);
    return hipGetLastError();
  }
  const int lanes = block_for(t, (d.N + t.opl - 1) / t.opl);
  const int64_t per_block = (int64_t)lanes * t.opl;
  const int64_t blocks = (d.N + per_block - 1) / per_block;
  if (blocks <= 0) return hipSuccess;
  dim3 grid((unsigned)blocks), block((unsigned)lanes);
  if (d.filter || d.window_v) {
    // The window test and the time-window velocity run with one orbit per
    // lane, no unrolling and at most 256 lanes per block.
    const int wb = std::min(block_for(t, d.N), 256);
    const dim3 wgrid((unsigned)((d.N + wb - 1) / wb));
    block = dim3((unsigned)wb);
    if (d.filter && d.window_v) hipLaunchKernelGGL((k_fwd<FORM, TAN, 1, 1, true, true>), wgrid, block, 0, s, d);
    else if (d.filter) hipLaunchKernelGGL((k_fwd<FORM, TAN, 1, 1, true, false>), wgrid, block, 0, s, d);
    else hipLaunchKernelGGL((k_fwd<FORM, TAN, 1, 1, false, true>), wgrid, block, 0, s, d);
  } else if (t.opl == 1 && t.unroll == 1) hipLaunchKernelGGL((k_fwd<FORM, TAN, 1, 1>), grid, block, 0, s, d);
  else if (t.opl == 1) hipLaunchKernelGGL((k_fwd<FORM, TAN, 1, 2>), grid, block, 0, s, d);
  else if (t.unroll == 1) hipLaunchKernelGGL((k_fwd<FORM, TAN, 2, 1>), grid, block, 0, s, d);
  else hipLaunchKernelGGL((k_fwd<FORM, TAN, 2, 2>), grid, block, 0, s, d);
  return hipGetLastError();
}

hipError_t launch_fwd(const FwdDesc &d, const Tuning &t, int form, bool tan, hipStream_t s) {
  switch (form) {
  case 1: return tan ? fwd_dispatch_opl<1, true>(d, t, s) : fwd_dispatch_opl<1, false>(d, t, s);
  case 2: return tan ? fwd_dispatch_opl<2, true>(d, t, s) : fwd_dispatch_opl<2, false>(d, t, s);
  case 4: return tan ? fwd_dispatch_opl<4, true>(d, t, s) : fwd_dispatch_opl<4, false>(d, t, s);
  case 6: return tan ? fwd_dispatch_opl<6, true>(d, t, s) : fwd_dispatch_opl<6, false>(d, t, s);
  case 7: return tan ? fwd_dispatch_opl<7, true>(d, t, s) : fwd_dispatch_opl<7, false>(d, t, s);
  default: return hipErrorInvalidValue;
  }
}

template <int FORM, bool TAN>
static hipError_t persist_dispatch(const FwdDesc *descs, const WorkItem *items, int32_t n_items,
                                   uint32_t *head, const Tuning &t, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, head, 1);
  dim3 grid((unsigned)n_wg), block((unsigned)block_256(t));
  if (t.opl == 1) hipLaunchKernelGGL((k_fwd_persist<FORM, TAN, 1>), grid, block, 0, s, descs, items, n_items, head);
  else hipLaunchKernelGGL((k_fwd_persist<FORM, TAN, 2>), grid, block, 0, s, descs, items, n_items, head);
  return hipGetLastError();
}

hipError_t launch_fwd_batched(const FwdDesc *descs_dev, const WorkItem *items_dev, int32_t n_items,
                              uint32_t *head_dev, const Tuning &t, int form, bool tan, int n_wg,
                              hipStream_t s) {
  switch (form) {
  case 1: return tan ? persist_dispatch<1, true>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s)
                     : persist_dispatch<1, false>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s);
  case 2: return tan ? persist_dispatch<2, true>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s)
                     : persist_dispatch<2, false>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s);
  case 4: return tan ? persist_dispatch<4, true>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s)
                     : persist_dispatch<4, false>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s);
  case 6: return tan ? persist_dispatch<6, true>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s)
                     : persist_dispatch<6, false>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s);
  case 7: return tan ? persist_dispatch<7, true>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s)
                     : persist_dispatch<7, false>(descs_dev, items_dev, n_items, head_dev, t, n_wg, s);
  default: return hipErrorInvalidValue;
  }
}

int persistent_blocks_per_cu(int form, bool tan, const Tuning &t) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define AW_OCC(F)                                                                                 \
  if (form == F) {                                                                                \
    if (tan) e = t.opl == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_persist<F, true, 1>, block_256(t), 0) \
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_persist<F, true, 2>, block_256(t), 0); \
    else e = t.opl == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_persist<F, false, 1>, block_256(t), 0) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_persist<F, false, 2>, block_256(t), 0); \
  }
  AW_OCC(1) AW_OCC(2) AW_OCC(4) AW_OCC(6) AW_OCC(7)
#undef AW_OCC
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_gen_ic(const FwdDesc &d, double *ic, double *w0, hipStream_t s) {
  if (d.N <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((d.N + 255) / 256);
  hipLaunchKernelGGL(k_gen_ic, dim3(blocks), dim3(256), 0, s, d, ic, w0);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// FP64 instruction counts per map step as built (sincos, kicks, drifts, J,
// amortised renormalisation excluded).
void step_op_counts(int form, bool tan, int64_t *fma, int64_t *mul, int64_t *add) {
  int nk = 0, nd = 0;
  switch (form) {
  case 1: nk = 1; nd = 1; break;
  case 2: nk = 1; nd = 2; break;
  case 4: nk = 3; nd = 4; break;
  case 6: nk = 9; nd = 10; break;
  case 7: nk = 7; nd = 8; break;
  default: break;
  }
  const int kf = tan ? KickRotOps<true>::fma : KickRotOps<false>::fma;
  const int km = tan ? KickRotOps<true>::mul : KickRotOps<false>::mul;
  const int ka = tan ? KickRotOps<true>::add : KickRotOps<false>::add;
  const int df = tan ? DriftOps<true>::fma : DriftOps<false>::fma;
  *fma = (int64_t)nk * kf + (int64_t)nd * df + 3;  // + 3 fma of the J accumulator
  *mul = (int64_t)nk * km;
  *add = (int64_t)nk * ka + 4;                     // + 3 subtractions and a doubling (J accumulator)
}

}  // namespace aw
