// aw_internal.hpp -- descriptors passed from the host library to the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aw {

constexpr int MAX_KICKS = 9;
constexpr int MAX_DRIFTS = 10;
constexpr int MAX_UNIQUE = 4;  // distinct kick (and drift) weights of any form

// Stage pattern of each map form: stage i of the step uses weight
// kick_idx[i] (drift_idx[i]) of the distinct weights.  The symmetric
// compositions are palindromic and the triple jump repeats its weights, so the
// 9 kicks and 10 drifts of the 6th-order step take only 4 + 4 distinct values;
// passing those keeps every weight in scalar registers.
template <int FORM> struct FormPattern;
template <> struct FormPattern<1> {
  static constexpr int NK = 1, ND = 1;
  static constexpr bool LEAD = false;
  static constexpr int kick_idx[1] = {0};
  static constexpr int drift_idx[1] = {0};
};
template <> struct FormPattern<2> {
  static constexpr int NK = 1, ND = 2;
  static constexpr bool LEAD = true;
  static constexpr int kick_idx[1] = {0};
  static constexpr int drift_idx[2] = {0, 0};
};
template <> struct FormPattern<4> {
  static constexpr int NK = 3, ND = 4;
  static constexpr bool LEAD = true;
  static constexpr int kick_idx[3] = {0, 1, 0};
  static constexpr int drift_idx[4] = {0, 1, 1, 0};
};
template <> struct FormPattern<6> {
  static constexpr int NK = 9, ND = 10;
  static constexpr bool LEAD = true;
  static constexpr int kick_idx[9] = {0, 1, 0, 2, 3, 2, 0, 1, 0};
  static constexpr int drift_idx[10] = {0, 1, 1, 2, 3, 3, 2, 1, 1, 0};
};
// Y6: S2(w3) S2(w2) S2(w1) S2(w0) S2(w1) S2(w2) S2(w3).
template <> struct FormPattern<7> {
  static constexpr int NK = 7, ND = 8;
  static constexpr bool LEAD = true;
  static constexpr int kick_idx[7] = {0, 1, 2, 3, 2, 1, 0};
  static constexpr int drift_idx[8] = {0, 1, 2, 3, 3, 2, 1, 0};
};
constexpr uint32_t BIN_DROP = 0xffffffffu;

// Image epilogue selector of the propagation kernel.
enum EpiKind : int32_t { EPI_NONE = 0, EPI_IC_GRID = 1, EPI_HIST_P0 = 2, EPI_HIST_VDIR = 3 };

// One ensemble as the kernels see it.  Distinct stage weights, pre-multiplied:
// drift[u] = c h, ka2[u] = 2 w h eps, ka4[u] = 4 w h eps.
struct FwdDesc {
  double drift[MAX_UNIQUE];
  double ka2[MAX_UNIQUE];
  double ka4[MAX_UNIQUE];
  double eps;
  double th;         // T h
  double lth;        // ln(1 + T h)
  double chi_thr;
  int64_t T;         // total steps of the run
  int64_t k_begin;   // first global step of this launch
  int64_t k_end;     // one past the last global step of this launch
  int64_t N;         // orbits
  // initial conditions
  int32_t ic_kind;   // 0 GRID2, 1 BOX, 2 EXPLICIT
  int32_t ax0, ax1;
  int32_t renorm_mask;  // renormalise after global step k when (k+1) & mask == 0
  int64_t nx;
  double lo0, d0, lo1, d1;
  double base[6];
  double box_lo[6], box_span[6];
  uint64_t seed_ic, seed_tan;
  // fixed-energy (SPHERE) initial conditions and the stay-in-window test
  double energy;
  double win[4];          // phi_lo, phi_hi, mu_lo, mu_hi
  double e0x, e0y;        // (cos phi_lo, sin phi_lo)
  double e1x, e1y;        // (cos phi_hi, sin phi_hi)
  int32_t win_phi;        // 0: every phi; 1: sector of width <= pi; 2: complement of a sector < pi
  int32_t win_mu;         // 0: every mu; 1: test mu_lo <= pz/|P| <= mu_hi
  int32_t filter;         // test the window after every step
  int32_t window_v;       // bin the mean velocity of this launch's steps (time-window density)
  double cloud[4];        // CLOUD: centre (vx, vy), sigma (x, y)
  double wdt;             // window_v: length of the window in time (steps x h)
  const double *ic;  // EXPLICIT [6][N]
  double *carry;     // [AW_NCARRY][N] or null
  double *out;       // [AW_NOUT][N] or null
  double *state;     // [12][N] or null
  uint8_t *cls;      // [N] or null
  // image epilogue
  int32_t epi;       // EpiKind
  int32_t field;     // orbit_out row imaged / averaged
  int32_t W, H;
  int32_t key0, key1;
  double klo0, khi0, klo1, khi1;   // HIST_P0 key ranges; HIST_VDIR (phi, mu) ranges
  double *img;       // IC_GRID: [H][W]
  uint32_t *n_class; // IC_GRID: one counter of class-1 orbits, or null
  uint32_t *bins;    // HIST: per-orbit bin index j*W + i or BIN_DROP
  double *vals;      // HIST_P0: per-orbit value
};

// Work item of the batched persistent launch: (ensemble, first orbit).
struct WorkItem {
  int32_t ens;
  int32_t pad;
  int64_t first;
};

// The store sweeps of the adjoints keep the state at the end of every
// ADJ_SUB-th step (global count: steps g with (g + 1) % ADJ_SUB == 0) and at
// the end of every segment; the reverse sweep rebuilds the steps in between by
// inverting their stages from the next kept state.  Slot of step g in the
// buffer of a segment that starts at g0: (g >> ADJ_SUB_LOG2) - (g0 >> ADJ_SUB_LOG2).
#ifndef AW_ADJ_SUB_LOG2
#define AW_ADJ_SUB_LOG2 2
#endif
constexpr int ADJ_SUB_LOG2 = AW_ADJ_SUB_LOG2;
constexpr int64_t ADJ_SUB = int64_t(1) << ADJ_SUB_LOG2;

__host__ __device__ inline bool adj_kept(int64_t g, int64_t g1) {
  return ((g + 1) & (ADJ_SUB - 1)) == 0 || g == g1 - 1;
}

__host__ __device__ inline int64_t adj_slot(int64_t g, int64_t g0) {
  return (g >> ADJ_SUB_LOG2) - (g0 >> ADJ_SUB_LOG2);
}

// Slots a segment of ck steps needs at most, wherever it starts.
__host__ __device__ inline int64_t adj_slots_max(int64_t ck) { return (ck + ADJ_SUB - 2) / ADJ_SUB + 1; }

// Adjoint descriptor.
struct AdjDesc {
  double drift[MAX_UNIQUE];
  double ka2[MAX_UNIQUE];
  double ka4[MAX_UNIQUE];
  double kw2[MAX_UNIQUE];  // 2 w h (for d/deps)
  double kw4[MAX_UNIQUE];  // 4 w h
  double eps;
  int64_t T;
  int64_t N;
  int64_t ckpt;           // steps per segment
  int64_t n_seg;          // ceil(T / ckpt)
  const double *ic;       // [6][N]
  const double *gJ;       // [N] or null
  double *J;              // [N] or null
  double *gic;            // [6][N]
  double *geps;           // [N]
  double *ckpts;          // [n_seg + 1][6][N] (the last slot: the final state)
  double *steps;          // [adj_slots_max(ckpt)][6][N] (kept step states of a segment)
  int32_t fwd_steps;      // 1: one segment, and the forward pass stores the step
                          // states itself, so that the store sweep skips its recompute
};

}  // namespace aw
