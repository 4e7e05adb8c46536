// aw_api.hip -- the C ABI of libaw (declared in include/aw.h): argument
// validation, stage-weight set-up, library scratch, batching, HIP graphs and
// kernel timing.  Every numerical step runs in the kernels of aw_fwd.hip,
// aw_hist.hip and aw_adj.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "aw.h"
#include "aw_hist.hpp"
#include "aw_internal.hpp"
#include "aw_y6_coef.h"
#include "aw_launch.hpp"

using namespace aw;

namespace {

thread_local std::string g_err;

aw_status fail(aw_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

aw_status hip_fail(hipError_t e, const char *what) {
  return fail(AW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Scratch layout of one call: one area, carved into 256-byte aligned parts.
// ---------------------------------------------------------------------------
constexpr size_t align_up(size_t n) { return (n + 255) / 256 * 256; }

struct Layout {
  // byte offsets into the area
  size_t bins = 0, vals = 0;                               // per orbit, every ensemble (histograms)
  size_t block_counts = 0, block_dropped = 0, tile_start = 0;
  size_t chunk_first = 0, part_first = 0, chunk_tile = 0;  // accumulation chunks
  size_t part_counts = 0, part_sums = 0;                   // partial tiles
  size_t sorted_local = 0, sorted_val = 0;                 // the largest single reduction
  size_t descs = 0, items = 0, head = 0;                   // tables of a batched launch
  size_t total = 0;
};

// hist: histogram images over n_all orbits in all, of which one reduction
// sorts at most n_max items into n_tiles tiles; vals: the items carry values;
// vals_here: the items' values are kept in the area (written by the
// propagation), not read from the caller; n_descs, n_items: tables of a
// batched launch (0 for none).
constexpr Layout layout_of(bool hist, bool vals, bool vals_here, int64_t n_all, int64_t n_max, int64_t n_tiles,
                           size_t n_descs, size_t n_items) {
  Layout l{};
  size_t o = 0;
  if (hist) {
    const size_t na = (size_t)(n_all > 0 ? n_all : 1), nm = (size_t)(n_max > 0 ? n_max : 1);
    const size_t G = (nm + HIST_ITEMS_PER_BLOCK - 1) / HIST_ITEMS_PER_BLOCK;
    // partial tiles: fewer than 2 ceil(N / chunk) <= 2 acc_bound(n_max, n_tiles) of them
    const size_t parts = 2 * (size_t)acc_bound((int64_t)nm, n_tiles);
    l.bins = o;
    o += align_up(sizeof(uint32_t) * na);
    if (vals && vals_here) {
      l.vals = o;
      o += align_up(sizeof(double) * na);
    }
    l.block_counts = o;
    o += align_up(sizeof(uint32_t) * (size_t)n_tiles * G);
    l.block_dropped = o;
    o += align_up(sizeof(uint32_t) * G);
    l.tile_start = o;
    o += align_up(sizeof(uint32_t) * (2 * (size_t)n_tiles + 1));
    l.chunk_first = o;
    o += align_up(sizeof(uint32_t) * ((size_t)n_tiles + 1));
    l.part_first = o;
    o += align_up(sizeof(uint32_t) * ((size_t)n_tiles + 1));
    l.chunk_tile = o;
    o += align_up(sizeof(uint32_t) * ((size_t)n_tiles + parts / 2));
    l.part_counts = o;
    o += align_up(sizeof(uint32_t) * parts * TILE_BINS);
    if (vals) {
      l.part_sums = o;
      o += align_up(sizeof(double) * parts * TILE_BINS);
    }
    l.sorted_local = o;
    o += align_up(sizeof(uint16_t) * nm);
    if (vals) {
      l.sorted_val = o;
      o += align_up(sizeof(double) * nm);
    }
  }
  if (n_descs > 0) {
    l.descs = o;
    o += align_up(sizeof(FwdDesc) * n_descs);
    l.items = o;
    o += align_up(sizeof(WorkItem) * (n_items ? n_items : 1));
    l.head = o;
    o += align_up(sizeof(uint32_t));
  }
  l.total = o;
  return l;
}

HistScratch hist_scratch_at(char *base, const Layout &l, bool vals, int64_t n_tiles) {
  HistScratch w;
  w.block_counts = (uint32_t *)(base + l.block_counts);
  w.block_dropped = (uint32_t *)(base + l.block_dropped);
  w.tile_start = (uint32_t *)(base + l.tile_start);
  w.tile_total = w.tile_start + n_tiles + 1;
  w.chunk_first = (uint32_t *)(base + l.chunk_first);
  w.part_first = (uint32_t *)(base + l.part_first);
  w.chunk_tile = (uint32_t *)(base + l.chunk_tile);
  w.part_counts = (uint32_t *)(base + l.part_counts);
  w.part_sums = vals ? (double *)(base + l.part_sums) : nullptr;
  w.sorted_local = (uint16_t *)(base + l.sorted_local);
  w.sorted_val = vals ? (double *)(base + l.sorted_val) : nullptr;
  return w;
}

// ---------------------------------------------------------------------------
// Library scratch: one area per (device, stream), so that calls on different
// streams never share it.  It grows by allocating a larger area -- at least
// twice the old one, so that retired areas add up to less than the live one --
// and retiring the old area, which earlier work on the stream may still be
// using.  hipFree waits for the device, so the call path never frees: retired
// areas and staging buffers are freed by aw_release().
// ---------------------------------------------------------------------------
// Pinned host staging of batch tables, reused once its copies are done.
struct Stage {
  void *p = nullptr;
  size_t n = 0;
  hipEvent_t done = nullptr;  // recorded after the copies out of p
};

struct StreamScratch {
  void *area = nullptr;
  size_t n = 0;
  std::vector<Stage> stages;
};

struct Retired {
  std::vector<void *> dev;
};

std::mutex g_mu;
std::map<std::pair<int, uintptr_t>, StreamScratch> g_scratch;
std::map<int, Retired> g_retired;

int cur_device() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return dev;
}

StreamScratch &stream_scratch(hipStream_t s) { return g_scratch[{cur_device(), (uintptr_t)s}]; }

aw_status reserve_area(StreamScratch &sc, size_t need) {
  if (sc.n >= need) return AW_OK;
  const size_t n = std::max(need, 2 * sc.n);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) return fail(AW_ENOMEM, "library scratch of %zu bytes: %s", n, hipGetErrorString(e));
  if (sc.area) g_retired[cur_device()].dev.push_back(sc.area);
  sc.area = p;
  sc.n = n;
  return AW_OK;
}

// ---------------------------------------------------------------------------
// Kernel timing.
// ---------------------------------------------------------------------------
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit TimedLaunch(hipStream_t st) : s(st) {
    if (!g_timing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
  }
  ~TimedLaunch() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    g_events.emplace_back(a, b);
  }
};

// ---------------------------------------------------------------------------
// Stage weights of the map forms (merged adjacent drifts).
// ---------------------------------------------------------------------------
struct Stages {
  int nk = 0, nd = 0;
  double kick[MAX_KICKS];
  double drift[MAX_DRIFTS];
};

Stages stages_of(int form) {
  Stages s;
  auto from_kicks = [&](const double *w, int nk) {
    s.nk = nk;
    s.nd = nk + 1;
    for (int i = 0; i < nk; ++i) s.kick[i] = w[i];
    s.drift[0] = 0.5 * w[0];
    for (int i = 1; i < nk; ++i) s.drift[i] = 0.5 * (w[i - 1] + w[i]);
    s.drift[nk] = 0.5 * w[nk - 1];
  };
  const double g1 = 1.0 / (2.0 - std::cbrt(2.0)), g0 = 1.0 - 2.0 * g1;
  const double d1 = 1.0 / (2.0 - std::pow(2.0, 1.0 / 5.0)), d0 = 1.0 - 2.0 * d1;
  if (form == AW_MAP_STDMAP) {
    s.nk = 1;
    s.nd = 1;
    s.kick[0] = 1.0;
    s.drift[0] = 1.0;
  } else if (form == AW_MAP_S2) {
    const double w[1] = {1.0};
    from_kicks(w, 1);
  } else if (form == AW_MAP_S4) {
    const double w[3] = {g1, g0, g1};
    from_kicks(w, 3);
  } else if (form == AW_MAP_S6) {
    const double w[9] = {g1 * d1, g0 * d1, g1 * d1, g1 * d0, g0 * d0, g1 * d0, g1 * d1, g0 * d1, g1 * d1};
    from_kicks(w, 9);
  } else if (form == AW_MAP_Y6) {
    const double *y = AW_Y6_W;  // w0, w1, w2, w3
    const double w[7] = {y[3], y[2], y[1], y[0], y[1], y[2], y[3]};
    from_kicks(w, 7);
  }
  return s;
}

// Compile-time stage pattern of a form (see FormPattern).
struct Pattern {
  int nk, nd;
  const int *kidx, *didx;
};

Pattern pattern_of(int form) {
  switch (form) {
  case 1: return {FormPattern<1>::NK, FormPattern<1>::ND, FormPattern<1>::kick_idx, FormPattern<1>::drift_idx};
  case 2: return {FormPattern<2>::NK, FormPattern<2>::ND, FormPattern<2>::kick_idx, FormPattern<2>::drift_idx};
  case 4: return {FormPattern<4>::NK, FormPattern<4>::ND, FormPattern<4>::kick_idx, FormPattern<4>::drift_idx};
  case 7: return {FormPattern<7>::NK, FormPattern<7>::ND, FormPattern<7>::kick_idx, FormPattern<7>::drift_idx};
  default: return {FormPattern<6>::NK, FormPattern<6>::ND, FormPattern<6>::kick_idx, FormPattern<6>::drift_idx};
  }
}

// Distinct stage weights (times h) of a form.  Every stage that shares an
// index must carry bitwise the same weight; false otherwise.
bool unique_weights(int form, double h, double kick[MAX_UNIQUE], double drift[MAX_UNIQUE]) {
  const Stages st = stages_of(form);
  const Pattern pt = pattern_of(form);
  if (pt.nk != st.nk || pt.nd != st.nd) return false;
  bool kset[MAX_UNIQUE] = {false, false, false, false}, dset[MAX_UNIQUE] = {false, false, false, false};
  for (int i = 0; i < MAX_UNIQUE; ++i) kick[i] = drift[i] = 0.0;
  for (int i = 0; i < st.nk; ++i) {
    const int u = pt.kidx[i];
    const double v = st.kick[i] * h;
    if (kset[u] && std::memcmp(&kick[u], &v, sizeof v) != 0) return false;
    kick[u] = v;
    kset[u] = true;
  }
  for (int i = 0; i < st.nd; ++i) {
    const int u = pt.didx[i];
    const double v = st.drift[i] * h;
    if (dset[u] && std::memcmp(&drift[u], &v, sizeof v) != 0) return false;
    drift[u] = v;
    dset[u] = true;
  }
  return true;
}

bool is_fin(double v) { return std::isfinite(v); }

aw_status check_tuning(const aw_tuning *t, Tuning &out) {
  out = Tuning{};
  if (!t) return AW_OK;
  out.block = t->block;
  out.opl = t->orbits_per_lane ? t->orbits_per_lane : 1;
  out.unroll = t->unroll ? t->unroll : 1;
  out.renorm = t->renorm_every ? t->renorm_every : 8;
  out.pwgs = t->persistent_wgs;
  out.lpo = t->lanes_per_orbit;
  if (out.block != 0 && out.block != 64 && out.block != 128 && out.block != 256 && out.block != 512)
    return fail(AW_EINVAL, "tuning.block must be 0 (automatic), 64, 128, 256 or 512 (got %d)", out.block);
  if (out.opl != 1 && out.opl != 2) return fail(AW_EINVAL, "tuning.orbits_per_lane must be 1 or 2");
  if (out.unroll != 1 && out.unroll != 2) return fail(AW_EINVAL, "tuning.unroll must be 1 or 2");
  if (out.renorm < 1 || out.renorm > 16 || (out.renorm & (out.renorm - 1)))
    return fail(AW_EINVAL, "tuning.renorm_every must be 1, 2, 4, 8 or 16");
  if (out.pwgs < 0) return fail(AW_EINVAL, "tuning.persistent_wgs must be >= 0");
  if (out.lpo != 0 && out.lpo != 1 && out.lpo != 2) return fail(AW_EINVAL, "tuning.lanes_per_orbit must be 0, 1 or 2");
  return AW_OK;
}

int64_t ens_size(const aw_ensemble &e) {
  if (e.ic_kind == AW_IC_GRID2) {
    if (e.nx < 1 || e.ny < 1 || e.nx > (int64_t(1) << 31) || e.ny > (int64_t(1) << 31)) return -1;
    return e.nx * e.ny;
  }
  return e.n_orbits >= 0 ? e.n_orbits : -1;
}

aw_status check_ensemble(const aw_ensemble *e, const double *ic, int idx) {
  if (!e) return fail(AW_EINVAL, "ensemble %d: null descriptor", idx);
  if (e->M != 3) return fail(AW_EUNSUPPORTED, "ensemble %d: only M = 3 is defined (got %d)", idx, e->M);
  if (e->map_form != AW_MAP_STDMAP && e->map_form != AW_MAP_S2 && e->map_form != AW_MAP_S4 &&
      e->map_form != AW_MAP_S6 && e->map_form != AW_MAP_Y6)
    return fail(AW_EINVAL, "ensemble %d: unknown map_form %d", idx, e->map_form);
  if (!is_fin(e->eps)) return fail(AW_EINVAL, "ensemble %d: eps must be finite", idx);
  if (!is_fin(e->h) || e->h == 0.0) return fail(AW_EINVAL, "ensemble %d: h must be finite and non-zero", idx);
  if (e->n_steps < 1) return fail(AW_EINVAL, "ensemble %d: n_steps must be >= 1", idx);
  if (e->flags & ~(AW_F_TANGENT | AW_F_WINDOW))
    return fail(AW_EINVAL, "ensemble %d: unknown flags 0x%x", idx, e->flags);
  if (e->ic_kind == AW_IC_SPHERE || (e->flags & AW_F_WINDOW)) {
    const double *w = e->window;
    for (int k = 0; k < 4; ++k)
      if (!is_fin(w[k])) return fail(AW_EINVAL, "ensemble %d: window not finite", idx);
    if (!(-M_PI <= w[0] && w[0] < w[1] && w[1] <= M_PI))
      return fail(AW_EINVAL, "ensemble %d: window needs -pi <= phi_lo < phi_hi <= pi", idx);
    if (!(-1.0 <= w[2] && w[2] < w[3] && w[3] <= 1.0))
      return fail(AW_EINVAL, "ensemble %d: window needs -1 <= mu_lo < mu_hi <= 1", idx);
  }
  {
    double k[MAX_UNIQUE], dr[MAX_UNIQUE];
    if (!unique_weights(e->map_form, e->h, k, dr))
      return fail(AW_EUNSUPPORTED, "ensemble %d: stage weights do not follow the form's pattern", idx);
  }
  if (std::isnan(e->chi_threshold)) return fail(AW_EINVAL, "ensemble %d: chi_threshold is NaN", idx);
  const int64_t N = ens_size(*e);
  if (N < 0) return fail(AW_EINVAL, "ensemble %d: bad size (nx, ny or n_orbits)", idx);
  if (N > (int64_t(1) << 31) - 1) return fail(AW_EINVAL, "ensemble %d: more than 2^31-1 orbits", idx);
  switch (e->ic_kind) {
  case AW_IC_GRID2:
    if (e->axis[0] < 0 || e->axis[0] > 5 || e->axis[1] < 0 || e->axis[1] > 5 || e->axis[0] == e->axis[1])
      return fail(AW_EINVAL, "ensemble %d: GRID2 axes must be distinct and in 0..5", idx);
    for (int k = 0; k < 2; ++k)
      if (!is_fin(e->lo[k]) || !is_fin(e->hi[k])) return fail(AW_EINVAL, "ensemble %d: GRID2 range not finite", idx);
    for (int k = 0; k < 6; ++k)
      if (!is_fin(e->base[k])) return fail(AW_EINVAL, "ensemble %d: GRID2 base not finite", idx);
    break;
  case AW_IC_BOX:
    for (int k = 0; k < 6; ++k)
      if (!is_fin(e->box_lo[k]) || !is_fin(e->box_hi[k]) || !is_fin(e->box_hi[k] - e->box_lo[k]))
        return fail(AW_EINVAL, "ensemble %d: BOX range not finite", idx);
    break;
  case AW_IC_EXPLICIT:
    if (N > 0 && !ic) return fail(AW_EINVAL, "ensemble %d: EXPLICIT needs ic_dev", idx);
    break;
  case AW_IC_CLOUD:
    for (int k = 0; k < 3; ++k)
      if (!is_fin(e->box_lo[k]) || !is_fin(e->box_hi[k]) || !is_fin(e->box_hi[k] - e->box_lo[k]))
        return fail(AW_EINVAL, "ensemble %d: CLOUD position range not finite", idx);
    for (int k = 0; k < 4; ++k)
      if (!is_fin(e->cloud[k])) return fail(AW_EINVAL, "ensemble %d: CLOUD values not finite", idx);
    if (!is_fin(e->energy) || !(e->energy > 2.0 * std::fabs(e->eps)))
      return fail(AW_EINVAL, "ensemble %d: CLOUD needs energy > 2|eps| (|Hp| <= 2, eq. 2)", idx);
    break;
  case AW_IC_SPHERE:
    for (int k = 0; k < 3; ++k)
      if (!is_fin(e->box_lo[k]) || !is_fin(e->box_hi[k]) || !is_fin(e->box_hi[k] - e->box_lo[k]))
        return fail(AW_EINVAL, "ensemble %d: SPHERE position range not finite", idx);
    if (!is_fin(e->energy) || !(e->energy > 2.0 * std::fabs(e->eps)))
      return fail(AW_EINVAL, "ensemble %d: SPHERE needs energy > 2|eps| (|Hp| <= 2, eq. 2)", idx);
    break;
  default:
    return fail(AW_EINVAL, "ensemble %d: unknown ic_kind %d", idx, e->ic_kind);
  }
  return AW_OK;
}

FwdDesc make_desc(const aw_ensemble &e, const double *ic, const Tuning &t) {
  FwdDesc d;
  std::memset(&d, 0, sizeof d);
  double tau[MAX_UNIQUE];
  (void)unique_weights(e.map_form, e.h, tau, d.drift);  // checked by check_ensemble
  for (int u = 0; u < MAX_UNIQUE; ++u) {
    d.ka2[u] = 2.0 * tau[u] * e.eps;
    d.ka4[u] = 4.0 * tau[u] * e.eps;
  }
  d.eps = e.eps;
  d.th = (double)e.n_steps * e.h;
  d.lth = std::log(1.0 + d.th);
  d.chi_thr = e.chi_threshold;
  d.T = e.n_steps;
  d.k_begin = 0;
  d.k_end = e.n_steps;
  d.N = ens_size(e);
  d.ic_kind = e.ic_kind;
  d.ax0 = e.axis[0];
  d.ax1 = e.axis[1];
  d.renorm_mask = t.renorm - 1;
  if (e.ic_kind == AW_IC_GRID2) {
    d.nx = e.nx;
    d.lo0 = e.lo[0];
    d.lo1 = e.lo[1];
    d.d0 = (e.hi[0] - e.lo[0]) / (double)e.nx;
    d.d1 = (e.hi[1] - e.lo[1]) / (double)e.ny;
    for (int k = 0; k < 6; ++k) d.base[k] = e.base[k];
  } else {
    d.nx = 1;
  }
  for (int k = 0; k < 6; ++k) {
    d.box_lo[k] = e.box_lo[k];
    d.box_span[k] = e.box_hi[k] - e.box_lo[k];
  }
  d.seed_ic = e.seed_ic;
  d.seed_tan = e.seed_tangent;
  d.ic = ic;
  d.epi = EPI_NONE;
  d.energy = e.energy;
  for (int k = 0; k < 4; ++k) d.win[k] = e.window[k];
  for (int k = 0; k < 4; ++k) d.cloud[k] = e.cloud[k];
  d.filter = (e.flags & AW_F_WINDOW) ? 1 : 0;
  if (d.filter) {
    const double w = e.window[1] - e.window[0];
    d.e0x = std::cos(e.window[0]);
    d.e0y = std::sin(e.window[0]);
    d.e1x = std::cos(e.window[1]);
    d.e1y = std::sin(e.window[1]);
    d.win_phi = (e.window[0] == -M_PI && e.window[1] == M_PI) ? 0 : (w <= M_PI ? 1 : 2);
    d.win_mu = (e.window[2] == -1.0 && e.window[3] == 1.0) ? 0 : 1;
  }
  return d;
}

bool tangent_on(const aw_ensemble &e) { return (e.flags & AW_F_TANGENT) != 0; }

aw_status launch_one(const FwdDesc &d, const Tuning &t, int form, bool tan, hipStream_t s) {
  hipError_t err;
  {
    TimedLaunch tl(s);
    err = launch_fwd(d, t, form, tan, s);
  }
  if (err != hipSuccess) return hip_fail(err, "propagation launch");
  return AW_OK;
}

// Batched persistent launch of descs (host copies) over n ensembles.
struct BatchTables {
  std::vector<WorkItem> items;
  int form = 6;
  bool tan = true;
};

BatchTables make_items(const std::vector<FwdDesc> &descs, const Tuning &t) {
  BatchTables b;
  const int64_t per = (int64_t)block_256(t) * t.opl;
  for (size_t e = 0; e < descs.size(); ++e)
    for (int64_t f = 0; f < descs[e].N; f += per) b.items.push_back(WorkItem{(int32_t)e, 0, f});
  // Longest processing time first: a tile's cost is its step count.
  std::stable_sort(b.items.begin(), b.items.end(), [&](const WorkItem &a, const WorkItem &c) {
    return descs[a.ens].T > descs[c.ens].T;
  });
  return b;
}

int persistent_wgs(int form, bool tan, const Tuning &t) {
  if (t.pwgs > 0) return t.pwgs;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    ncu = 256;
  return ncu * persistent_blocks_per_cu(form, tan, t);
}

// Copy the batch tables into the area (at l.descs and l.items) through one of
// the stream's pinned staging buffers: one whose earlier copies have finished,
// or a new one -- the host never waits for the device here.
aw_status upload_tables(StreamScratch &sc, const Layout &l, const std::vector<FwdDesc> &descs,
                        const std::vector<WorkItem> &items, hipStream_t s) {
  const size_t bd = descs.size() * sizeof(FwdDesc), bi = items.size() * sizeof(WorkItem);
  hipError_t e;
  Stage *st = nullptr;
  for (Stage &c : sc.stages) {
    if (c.n < bd + bi) continue;
    e = hipEventQuery(c.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    st = &c;
    break;
  }
  if (!st) {
    Stage c;
    c.n = align_up(bd + bi);
    if ((e = hipHostMalloc(&c.p, c.n, hipHostMallocDefault)) != hipSuccess)
      return fail(AW_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
    if ((e = hipEventCreateWithFlags(&c.done, hipEventDisableTiming)) != hipSuccess) {
      (void)hipHostFree(c.p);
      return hip_fail(e, "hipEventCreate");
    }
    sc.stages.push_back(c);
    st = &sc.stages.back();
  }
  std::memcpy(st->p, descs.data(), bd);
  std::memcpy((char *)st->p + bd, items.data(), bi);
  char *base = (char *)sc.area;
  if ((e = hipMemcpyAsync(base + l.descs, st->p, bd, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(base + l.items, (char *)st->p + bd, bi, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "batch table upload");
  if ((e = hipEventRecord(st->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return AW_OK;
}

aw_status launch_batched_tables(const FwdDesc *descs_dev, const WorkItem *items_dev, int32_t n_items,
                                uint32_t *head, const Tuning &t, int form, bool tan, hipStream_t s) {
  const int nwg = std::max(1, std::min<int>(persistent_wgs(form, tan, t), n_items));
  hipError_t err;
  {
    TimedLaunch tl(s);
    err = launch_fwd_batched(descs_dev, items_dev, n_items, head, t, form, tan, nwg, s);
  }
  if (err != hipSuccess) return hip_fail(err, "persistent launch");
  return AW_OK;
}

aw_status validate_batch(const aw_ensemble *ens, int32_t n_ens, const double *const *ic_dev) {
  if (!ens || n_ens < 1) return fail(AW_EINVAL, "need n_ens >= 1 descriptors");
  for (int e = 0; e < n_ens; ++e) {
    aw_status st = check_ensemble(&ens[e], ic_dev ? ic_dev[e] : nullptr, e);
    if (st != AW_OK) return st;
    if (ens[e].map_form != ens[0].map_form || ens[e].flags != ens[0].flags)
      return fail(AW_EINVAL, "batched ensembles must share map_form and flags (ensemble %d differs)", e);
    if (n_ens > 1 && (ens[e].flags & AW_F_WINDOW))
      return fail(AW_EUNSUPPORTED, "the window test runs in single-ensemble launches only");
  }
  return AW_OK;
}

// Image spec checks; fills the epilogue fields of d.
aw_status apply_image(const aw_image_spec *sp, const aw_ensemble &e, int idx, FwdDesc &d, double *img,
                      uint32_t *cnt) {
  if (!sp) return fail(AW_EINVAL, "null image spec");
  const bool own_grid = sp->kind == AW_IMG_IC_GRID && sp->W == 0 && sp->H == 0;
  if (!own_grid && (sp->W < 1 || sp->H < 1)) return fail(AW_EINVAL, "image W, H must be >= 1");
  if (!img) return fail(AW_EINVAL, "ensemble %d: null image buffer", idx);
  d.W = own_grid ? (int32_t)e.nx : sp->W;
  d.H = own_grid ? (int32_t)e.ny : sp->H;
  d.field = sp->field;
  switch (sp->kind) {
  case AW_IMG_IC_GRID:
    if (e.ic_kind != AW_IC_GRID2) return fail(AW_EINVAL, "ensemble %d: IC_GRID images need a GRID2 ensemble", idx);
    if (d.W != e.nx || d.H != e.ny) return fail(AW_EINVAL, "ensemble %d: IC_GRID needs W = nx, H = ny", idx);
    if (sp->field < 0 || sp->field >= AW_NOUT) return fail(AW_EINVAL, "image field out of range");
    d.epi = EPI_IC_GRID;
    d.img = img;
    d.n_class = cnt;
    break;
  case AW_IMG_HIST_P0:
    if (sp->field < 0 || sp->field >= AW_NOUT) return fail(AW_EINVAL, "image field out of range");
    if (sp->key_axis[0] < 0 || sp->key_axis[0] > 5 || sp->key_axis[1] < 0 || sp->key_axis[1] > 5)
      return fail(AW_EINVAL, "HIST_P0 key axes must be in 0..5");
    if (!(sp->lo[0] < sp->hi[0]) || !(sp->lo[1] < sp->hi[1]) || !is_fin(sp->hi[0] - sp->lo[0]) ||
        !is_fin(sp->hi[1] - sp->lo[1]))
      return fail(AW_EINVAL, "HIST_P0 ranges must satisfy lo < hi");
    d.epi = EPI_HIST_P0;
    d.key0 = sp->key_axis[0];
    d.key1 = sp->key_axis[1];
    d.klo0 = sp->lo[0];
    d.khi0 = sp->hi[0];
    d.klo1 = sp->lo[1];
    d.khi1 = sp->hi[1];
    break;
  case AW_IMG_HIST_VDIR:
    d.epi = EPI_HIST_VDIR;
    if (sp->lo[0] == 0.0 && sp->hi[0] == 0.0 && sp->lo[1] == 0.0 && sp->hi[1] == 0.0) {
      d.klo0 = -M_PI;
      d.khi0 = M_PI;
      d.klo1 = -1.0;
      d.khi1 = 1.0;
    } else {
      if (!(sp->lo[0] < sp->hi[0]) || !(sp->lo[1] < sp->hi[1]) || !is_fin(sp->hi[0] - sp->lo[0]) ||
          !is_fin(sp->hi[1] - sp->lo[1]))
        return fail(AW_EINVAL, "HIST_VDIR zoom ranges must satisfy lo < hi");
      d.klo0 = sp->lo[0];
      d.khi0 = sp->hi[0];
      d.klo1 = sp->lo[1];
      d.khi1 = sp->hi[1];
    }
    break;
  default:
    return fail(AW_EINVAL, "unknown image kind %d", sp->kind);
  }
  if (sp->kind != AW_IMG_IC_GRID) {
    const HistPlan p = hist_plan(d.N, sp->W, sp->H);
    if (p.n_tiles > MAX_TILES) return fail(AW_EINVAL, "image too large: %d tiles (max %d)", p.n_tiles, MAX_TILES);
    if ((int64_t)p.n_tiles * p.G > (int64_t(1) << 30)) return fail(AW_EINVAL, "image x ensemble too large");
  }
  return AW_OK;
}

// One image call: validated descriptors, work items and scratch layout.
// batched: one persistent launch over every ensemble, their histogram items
// side by side in the area; otherwise the ensembles run one after the other,
// each reusing the same part of the area (stream order keeps them apart).
struct ImageCall {
  std::vector<FwdDesc> descs;
  std::vector<WorkItem> items;
  std::vector<int64_t> off;  // first item of each ensemble in the bins array
  Layout lay;
  bool hist = false, vals = false, batched = false;
  int form = 6;
  bool tan = true;
  int64_t n_tiles = 0;
};

aw_status prepare_image(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec, double *const *image,
                        uint32_t *const *counts, uint8_t *const *cls, const Tuning &t, bool batched,
                        ImageCall &c) {
  c.descs.assign(n_ens, FwdDesc{});
  c.off.assign(n_ens + 1, 0);
  c.batched = batched && n_ens > 1;
  c.hist = spec->kind != AW_IMG_IC_GRID;
  c.vals = spec->kind == AW_IMG_HIST_P0;
  c.form = ens[0].map_form;
  c.tan = tangent_on(ens[0]);
  int64_t n_max = 0;
  for (int e = 0; e < n_ens; ++e) {
    c.descs[e] = make_desc(ens[e], nullptr, t);
    aw_status st = apply_image(spec, ens[e], e, c.descs[e], image[e], counts ? counts[e] : nullptr);
    if (st != AW_OK) return st;
    c.descs[e].cls = cls ? cls[e] : nullptr;
    c.off[e + 1] = c.off[e] + (c.batched ? c.descs[e].N : 0);
    n_max = std::max<int64_t>(n_max, c.descs[e].N);
  }
  if (c.hist) c.n_tiles = hist_plan(n_max, spec->W, spec->H).n_tiles;
  if (c.batched) c.items = make_items(c.descs, t).items;
  const int64_t n_all = c.batched ? c.off[n_ens] : n_max;
  c.lay = layout_of(c.hist, c.vals, true, n_all, n_max, c.n_tiles, c.batched ? c.descs.size() : 0,
                    c.batched ? c.items.size() : 0);
  return AW_OK;
}

// Point the descriptors' histogram items into the area at `base`.
void place_image(ImageCall &c, char *base) {
  if (!c.hist) return;
  for (size_t e = 0; e < c.descs.size(); ++e) {
    c.descs[e].bins = (uint32_t *)(base + c.lay.bins) + c.off[e];
    c.descs[e].vals = c.vals ? (double *)(base + c.lay.vals) + c.off[e] : nullptr;
  }
}

// Histogram reduction of ensemble e's items into its image.
hipError_t reduce_image(const ImageCall &c, char *base, int e, const aw_image_spec *spec, double *const *image,
                        uint32_t *const *counts, hipStream_t s) {
  const FwdDesc &d = c.descs[e];
  const HistPlan p = hist_plan(d.N, spec->W, spec->H);
  const HistScratch w = hist_scratch_at(base, c.lay, c.vals, p.n_tiles);
  const int mode = c.vals ? 1 : 2;
  const double norm = 1.0 / ((double)d.N * ((d.khi0 - d.klo0) / spec->W) * ((d.khi1 - d.klo1) / spec->H));
  return launch_hist_reduce(d.N, d.bins, d.vals, p, w, mode, norm, counts ? counts[e] : nullptr, image[e], nullptr,
                            s);
}

// Enqueue a prepared and placed image call.  A batched call needs its tables
// at lay.descs / lay.items of the area already (or on their way, earlier on
// the stream).  timed: record the propagation launches for aw_timing_read
// (never inside a graph capture).
aw_status enqueue_image(const ImageCall &c, char *base, const aw_image_spec *spec, double *const *image,
                        uint32_t *const *counts, const Tuning &t, hipStream_t s, bool timed) {
  hipError_t herr;
  const int n_ens = (int)c.descs.size();
  auto propagate = [&](const FwdDesc &d) -> aw_status {
    if (timed) return launch_one(d, t, c.form, c.tan, s);
    hipError_t e2 = launch_fwd(d, t, c.form, c.tan, s);
    return e2 == hipSuccess ? AW_OK : hip_fail(e2, "propagation launch");
  };
  auto zero_counter = [&](const FwdDesc &d) -> aw_status {
    if (d.epi != EPI_IC_GRID || !d.n_class) return AW_OK;
    hipError_t e2 = launch_zero_u32(d.n_class, 1, s);
    return e2 == hipSuccess ? AW_OK : hip_fail(e2, "zero counter");
  };
  aw_status st;
  if (!c.batched) {
    for (int e = 0; e < n_ens; ++e) {
      if ((st = zero_counter(c.descs[e])) != AW_OK || (st = propagate(c.descs[e])) != AW_OK) return st;
      if (c.hist && (herr = reduce_image(c, base, e, spec, image, counts, s)) != hipSuccess)
        return hip_fail(herr, "histogram reduction");
    }
    return AW_OK;
  }
  for (int e = 0; e < n_ens; ++e)
    if ((st = zero_counter(c.descs[e])) != AW_OK) return st;
  if (!c.items.empty()) {
    const FwdDesc *dd = (const FwdDesc *)(base + c.lay.descs);
    const WorkItem *di = (const WorkItem *)(base + c.lay.items);
    uint32_t *head = (uint32_t *)(base + c.lay.head);
    if (timed) {
      st = launch_batched_tables(dd, di, (int32_t)c.items.size(), head, t, c.form, c.tan, s);
    } else {
      const int nwg = std::max(1, std::min<int>(persistent_wgs(c.form, c.tan, t), (int)c.items.size()));
      herr = launch_fwd_batched(dd, di, (int32_t)c.items.size(), head, t, c.form, c.tan, nwg, s);
      st = herr == hipSuccess ? AW_OK : hip_fail(herr, "persistent launch");
    }
    if (st != AW_OK) return st;
  }
  if (c.hist)
    for (int e = 0; e < n_ens; ++e)
      if ((herr = reduce_image(c, base, e, spec, image, counts, s)) != hipSuccess)
        return hip_fail(herr, "histogram reduction");
  return AW_OK;
}

// Propagate n ensembles with image epilogues and run the reductions, in the
// stream's library scratch.
aw_status image_run(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec, double *const *image,
                    uint32_t *const *counts, uint8_t *const *cls, const Tuning &t, hipStream_t s) {
  ImageCall c;
  aw_status st = prepare_image(ens, n_ens, spec, image, counts, cls, t, true, c);
  if (st != AW_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  StreamScratch &sc = stream_scratch(s);
  if ((st = reserve_area(sc, c.lay.total)) != AW_OK) return st;
  char *base = (char *)sc.area;
  place_image(c, base);
  if (c.batched && !c.items.empty() && (st = upload_tables(sc, c.lay, c.descs, c.items, s)) != AW_OK) return st;
  return enqueue_image(c, base, spec, image, counts, t, s, true);
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed scratch of aw_histogram2d_noalloc, for callers that cannot allocate.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is looked up once per device (with that
// device current) and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[AW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_fixed_mu;
char *g_fixed_ptr[MAX_DEVICES] = {};

aw_status fixed_scratch(char **out) {
  const int dev = cur_device();
  if (dev < 0 || dev >= MAX_DEVICES) return fail(AW_EUNSUPPORTED, "device %d: more than %d devices", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "device address of the fixed scratch");
    if (!p) return fail(AW_EDEVICE, "device address of the fixed scratch is null");
    g_fixed_ptr[dev] = (char *)p;
  }
  *out = g_fixed_ptr[dev];
  return AW_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *aw_last_error(void) { return g_err.c_str(); }

const char *aw_version(void) { return "libaw 0.1 (gfx950, FP64)"; }

aw_status aw_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int dev = cur_device();
  (void)hipDeviceSynchronize();
  for (auto it = g_scratch.begin(); it != g_scratch.end();) {
    if (it->first.first != dev) {
      ++it;
      continue;
    }
    StreamScratch &sc = it->second;
    if (sc.area) (void)hipFree(sc.area);
    for (Stage &st : sc.stages) {
      (void)hipHostFree(st.p);
      (void)hipEventDestroy(st.done);
    }
    it = g_scratch.erase(it);
  }
  auto r = g_retired.find(dev);
  if (r != g_retired.end()) {
    for (void *p : r->second.dev) (void)hipFree(p);
    g_retired.erase(r);
  }
  return AW_OK;
}

aw_status aw_image_workspace(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec, size_t *bytes) {
  if (!bytes) return fail(AW_EINVAL, "null bytes");
  aw_status st = validate_batch(ens, n_ens, nullptr);
  if (st != AW_OK) return st;
  if (!spec) {
    if (n_ens == 1) {
      *bytes = 0;
      return AW_OK;
    }
    std::vector<FwdDesc> descs(n_ens);
    for (int e = 0; e < n_ens; ++e) descs[e] = make_desc(ens[e], nullptr, Tuning{});
    *bytes = layout_of(false, false, false, 0, 0, 0, descs.size(), make_items(descs, Tuning{}).items.size()).total;
    return AW_OK;
  }
  std::vector<double> dummy(n_ens, 0.0);
  std::vector<double *> img(n_ens);
  for (int e = 0; e < n_ens; ++e) img[e] = &dummy[e];
  ImageCall c;
  if ((st = prepare_image(ens, n_ens, spec, img.data(), nullptr, nullptr, Tuning{}, true, c)) != AW_OK) return st;
  *bytes = c.lay.total;
  return AW_OK;
}

aw_status aw_reserve(size_t bytes, void *stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  return reserve_area(stream_scratch((hipStream_t)stream), bytes);
}

int64_t aw_ensemble_size(const aw_ensemble *ens) {
  if (!ens) return -1;
  return ens_size(*ens);
}

aw_status aw_generate_ic(const aw_ensemble *ens, const double *ic_in_dev, double *ic_dev, double *w0_dev,
                         void *stream) {
  aw_status st = check_ensemble(ens, ic_in_dev, 0);
  if (st != AW_OK) return st;
  const FwdDesc d = make_desc(*ens, ic_in_dev, Tuning{});
  hipError_t e = launch_gen_ic(d, ic_dev, w0_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "initial-condition launch");
  return AW_OK;
}

aw_status aw_map_ensemble(const aw_ensemble *ens, int32_t n_ens, const double *const *ic_dev,
                          double *const *orbit_out_dev, double *const *state_out_dev, uint8_t *const *cls_dev,
                          const aw_tuning *tuning, void *stream) {
  aw_status st = validate_batch(ens, n_ens, ic_dev);
  if (st != AW_OK) return st;
  Tuning t;
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<FwdDesc> descs(n_ens);
  for (int e = 0; e < n_ens; ++e) {
    descs[e] = make_desc(ens[e], ic_dev ? ic_dev[e] : nullptr, t);
    descs[e].out = orbit_out_dev ? orbit_out_dev[e] : nullptr;
    descs[e].state = state_out_dev ? state_out_dev[e] : nullptr;
    descs[e].cls = cls_dev ? cls_dev[e] : nullptr;
  }
  const int form = ens[0].map_form;
  const bool tan = tangent_on(ens[0]);
  if (n_ens == 1) return launch_one(descs[0], t, form, tan, s);
  BatchTables b = make_items(descs, t);
  if (b.items.empty()) return AW_OK;
  const Layout l = layout_of(false, false, false, 0, 0, 0, descs.size(), b.items.size());
  std::lock_guard<std::mutex> lk(g_mu);
  StreamScratch &sc = stream_scratch(s);
  if ((st = reserve_area(sc, l.total)) != AW_OK) return st;
  if ((st = upload_tables(sc, l, descs, b.items, s)) != AW_OK) return st;
  char *base = (char *)sc.area;
  return launch_batched_tables((const FwdDesc *)(base + l.descs), (const WorkItem *)(base + l.items),
                               (int32_t)b.items.size(), (uint32_t *)(base + l.head), t, form, tan, s);
}

aw_status aw_map_ensemble_steps(const aw_ensemble *ens, const double *ic_dev, double *carry_dev, int64_t k_begin,
                                int64_t k_end, double *orbit_out_dev, double *state_out_dev, uint8_t *cls_dev,
                                const aw_tuning *tuning, void *stream) {
  aw_status st = check_ensemble(ens, ic_dev, 0);
  if (st != AW_OK) return st;
  Tuning t;
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  if (k_begin < 0 || k_end <= k_begin || k_end > ens->n_steps)
    return fail(AW_EINVAL, "need 0 <= k_begin < k_end <= n_steps");
  if (!carry_dev && (k_begin > 0 || k_end < ens->n_steps))
    return fail(AW_EINVAL, "a partial range needs carry_dev");
  FwdDesc d = make_desc(*ens, ic_dev, t);
  d.k_begin = k_begin;
  d.k_end = k_end;
  d.carry = carry_dev;
  d.out = orbit_out_dev;
  d.state = state_out_dev;
  d.cls = cls_dev;
  return launch_one(d, t, ens->map_form, tangent_on(*ens), (hipStream_t)stream);
}

aw_status aw_indicator_image(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec,
                             double *const *image_dev, uint32_t *const *counts_dev, uint8_t *const *cls_dev,
                             const aw_tuning *tuning, void *stream) {
  aw_status st = validate_batch(ens, n_ens, nullptr);
  if (st != AW_OK) return st;
  if (!spec) return fail(AW_EINVAL, "null image spec");
  if (!image_dev) return fail(AW_EINVAL, "null image array");
  for (int e = 0; e < n_ens; ++e)
    if (ens[e].ic_kind == AW_IC_EXPLICIT)
      return fail(AW_EINVAL, "aw_indicator_image generates its initial conditions (GRID2 or BOX)");
  Tuning t;
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  return image_run(ens, n_ens, spec, image_dev, counts_dev, cls_dev, t, (hipStream_t)stream);
}

aw_status aw_window_density(const aw_ensemble *ens, const double *ic_dev, double *carry_dev, int64_t k_begin,
                            int64_t n_windows, int64_t window_steps, const aw_image_spec *spec,
                            uint32_t *counts_accum_dev, const aw_tuning *tuning, void *stream) {
  aw_status st = check_ensemble(ens, ic_dev, 0);
  if (st != AW_OK) return st;
  Tuning t;
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  if (!spec || spec->kind != AW_IMG_HIST_VDIR) return fail(AW_EINVAL, "aw_window_density needs a HIST_VDIR spec");
  if (!carry_dev) return fail(AW_EINVAL, "aw_window_density needs carry_dev");
  if (!counts_accum_dev) return fail(AW_EINVAL, "null counts_accum_dev");
  if (k_begin < 0 || n_windows < 1 || window_steps < 1 || n_windows > (ens->n_steps - k_begin) / window_steps)
    return fail(AW_EINVAL, "need k_begin >= 0, n_windows, window_steps >= 1 and "
                           "k_begin + n_windows * window_steps <= n_steps");
  FwdDesc d = make_desc(*ens, ic_dev, t);
  // The density image is bound to the spec; apply_image checks the zoom and the tile count.
  double dummy_img = 0.0;
  if ((st = apply_image(spec, *ens, 0, d, &dummy_img, nullptr)) != AW_OK) return st;
  d.img = nullptr;
  d.epi = EPI_NONE;
  d.window_v = 1;
  d.wdt = (double)window_steps * ens->h;
  d.carry = carry_dev;
  hipStream_t s = (hipStream_t)stream;
  const HistPlan p = hist_plan(d.N, spec->W, spec->H);
  const Layout l = layout_of(true, false, false, d.N, d.N, p.n_tiles, 0, 0);
  std::lock_guard<std::mutex> lk(g_mu);
  StreamScratch &sc = stream_scratch(s);
  if ((st = reserve_area(sc, l.total)) != AW_OK) return st;
  char *base = (char *)sc.area;
  const HistScratch w = hist_scratch_at(base, l, false, p.n_tiles);
  d.bins = (uint32_t *)(base + l.bins);
  hipError_t e;
  for (int64_t k = 0; k < n_windows; ++k) {
    d.k_begin = k_begin + k * window_steps;
    d.k_end = d.k_begin + window_steps;
    if ((st = launch_one(d, t, ens->map_form, tangent_on(*ens), s)) != AW_OK) return st;
    if ((e = launch_hist_reduce(d.N, d.bins, nullptr, p, w, 2, 0.0, counts_accum_dev, nullptr, nullptr, s, 1)) !=
        hipSuccess)
      return hip_fail(e, "window histogram");
  }
  return AW_OK;
}

// One histogram over caller keys: hist2d_check validates the arguments and
// plans the tiles; hist2d_run enqueues the binning and the reduction with
// their scratch laid out (layout_of) in the area at `base`, which the caller
// has sized.
static aw_status hist2d_check(int64_t N, const double *a_dev, const double *b_dev, double lo0, double hi0, double lo1,
                              double hi1, int32_t W, int32_t H, uint32_t *counts_dev, HistPlan &p) {
  if (N < 0 || N > (int64_t(1) << 31) - 1) return fail(AW_EINVAL, "N out of range");
  if (W < 1 || H < 1) return fail(AW_EINVAL, "W, H must be >= 1");
  if (!(lo0 < hi0) || !(lo1 < hi1) || !is_fin(hi0 - lo0) || !is_fin(hi1 - lo1))
    return fail(AW_EINVAL, "ranges must satisfy lo < hi");
  if (N > 0 && (!a_dev || !b_dev)) return fail(AW_EINVAL, "null key arrays");
  if (!counts_dev) return fail(AW_EINVAL, "null counts");
  p = hist_plan(N, W, H);
  if (p.n_tiles > MAX_TILES) return fail(AW_EINVAL, "image too large: %d tiles (max %d)", p.n_tiles, MAX_TILES);
  return AW_OK;
}

static aw_status hist2d_run(char *base, const Layout &l, const HistPlan &p, int64_t N, const double *a_dev,
                            const double *b_dev, const double *v_dev, double lo0, double hi0, double lo1, double hi1,
                            int32_t W, int32_t H, int32_t closed_upper, uint32_t *counts_dev, double *sums_dev,
                            uint64_t *dropped_dev, hipStream_t s) {
  const HistScratch w = hist_scratch_at(base, l, v_dev != nullptr, p.n_tiles);
  uint32_t *bins = (uint32_t *)(base + l.bins);
  hipError_t e;
  if ((e = launch_hist_bins(N, a_dev, b_dev, lo0, hi0, lo1, hi1, W, H, closed_upper, bins, s)) != hipSuccess)
    return hip_fail(e, "histogram bins");
  if ((e = launch_hist_reduce(N, bins, v_dev, p, w, 0, 1.0, counts_dev, sums_dev, dropped_dev, s)) != hipSuccess)
    return hip_fail(e, "histogram reduction");
  return AW_OK;
}

aw_status aw_histogram2d(int64_t N, const double *a_dev, const double *b_dev, const double *v_dev, double lo0,
                         double hi0, double lo1, double hi1, int32_t W, int32_t H, int32_t closed_upper,
                         uint32_t *counts_dev, double *sums_dev, uint64_t *dropped_dev, void *stream) {
  HistPlan p;
  aw_status st = hist2d_check(N, a_dev, b_dev, lo0, hi0, lo1, hi1, W, H, counts_dev, p);
  if (st != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const Layout l = layout_of(true, v_dev != nullptr, false, N, N, p.n_tiles, 0, 0);
  std::lock_guard<std::mutex> lk(g_mu);
  StreamScratch &sc = stream_scratch(s);
  if ((st = reserve_area(sc, l.total)) != AW_OK) return st;
  return hist2d_run((char *)sc.area, l, p, N, a_dev, b_dev, v_dev, lo0, hi0, lo1, hi1, W, H, closed_upper,
                    counts_dev, sums_dev, dropped_dev, s);
}

aw_status aw_histogram2d_noalloc(int64_t N, const double *a_dev, const double *b_dev, const double *v_dev,
                                 double lo0, double hi0, double lo1, double hi1, int32_t W, int32_t H,
                                 int32_t closed_upper, uint32_t *counts_dev, double *sums_dev, uint64_t *dropped_dev,
                                 void *stream) {
  HistPlan p;
  aw_status st = hist2d_check(N, a_dev, b_dev, lo0, hi0, lo1, hi1, W, H, counts_dev, p);
  if (st != AW_OK) return st;
  const Layout l = layout_of(true, v_dev != nullptr, false, N, N, p.n_tiles, 0, 0);
  if (l.total > (size_t)AW_NOALLOC_SCRATCH_BYTES)
    return fail(AW_EWORKSPACE, "aw_histogram2d_noalloc: %lld items into %d x %d bins need %zu bytes of scratch, "
                               "more than its fixed %zu", (long long)N, W, H, l.total,
                (size_t)AW_NOALLOC_SCRATCH_BYTES);
  char *area = nullptr;
  if ((st = fixed_scratch(&area)) != AW_OK) return st;
  return hist2d_run(area, l, p, N, a_dev, b_dev, v_dev, lo0, hi0, lo1, hi1, W, H, closed_upper, counts_dev, sums_dev,
                    dropped_dev, (hipStream_t)stream);
}

aw_status aw_vdir_keys(int64_t N, const double *V_dev, double *phi_dev, double *mu_dev, void *stream) {
  if (N < 0) return fail(AW_EINVAL, "N < 0");
  if (N > 0 && (!V_dev || !phi_dev || !mu_dev)) return fail(AW_EINVAL, "null array");
  hipError_t e = launch_vdir_keys(N, V_dev, phi_dev, mu_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "vdir launch");
  return AW_OK;
}

aw_status aw_indicator_grad_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes) {
  if (!bytes) return fail(AW_EINVAL, "null bytes");
  if (!ens) return fail(AW_EINVAL, "null ensemble");
  if (ckpt_every < 1) return fail(AW_EINVAL, "ckpt_every must be >= 1");
  if (ens->n_steps < 1) return fail(AW_EINVAL, "n_steps must be >= 1");
  const int64_t N = ens_size(*ens);
  if (N < 0) return fail(AW_EINVAL, "bad ensemble size");
  const int64_t ck = std::min(ckpt_every, ens->n_steps);
  const int64_t n_seg = (ens->n_steps + ck - 1) / ck;
  // n_seg checkpoints, the final state, and the kept step states of one segment
  *bytes = sizeof(double) * 6 * (size_t)N * (size_t)(n_seg + 1 + adj_slots_max(ck));
  return AW_OK;
}

aw_status aw_indicator_grad_reversible_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes) {
  size_t full = 0;
  aw_status st = aw_indicator_grad_workspace(ens, ckpt_every, &full);
  if (st != AW_OK) return st;
  const int64_t N = ens_size(*ens);
  const int64_t ck = std::min(ckpt_every, ens->n_steps);
  const int64_t n_seg = (ens->n_steps + ck - 1) / ck;
  // n_seg checkpoints and the final state
  *bytes = sizeof(double) * 6 * (size_t)N * (size_t)(n_seg + 1);
  return AW_OK;
}

// Validation and descriptor of the adjoint of J (both sweeps).
static aw_status adj_setup(const aw_ensemble *ens, const double *ic_dev, const double *grad_J_dev, int64_t ckpt_every,
                    double *J_out_dev, double *grad_ic_dev, double *grad_eps_dev, void *workspace_dev,
                    size_t ws_bytes, const aw_tuning *tuning, const char *who, bool reversible, AdjDesc &d,
                    Tuning &t) {
  aw_status st = check_ensemble(ens, ic_dev, 0);
  if (st != AW_OK) return st;
  if (ens->ic_kind != AW_IC_EXPLICIT) return fail(AW_EINVAL, "%s needs an EXPLICIT ensemble", who);
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  size_t need = 0;
  st = reversible ? aw_indicator_grad_reversible_workspace(ens, ckpt_every, &need)
                  : aw_indicator_grad_workspace(ens, ckpt_every, &need);
  if (st != AW_OK) return st;
  const int64_t N = ens_size(*ens);
  if (N > 0 && (!grad_ic_dev || !grad_eps_dev)) return fail(AW_EINVAL, "null gradient outputs");
  if (ws_bytes < need || (N > 0 && !workspace_dev))
    return fail(AW_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  std::memset(&d, 0, sizeof d);
  double tau[MAX_UNIQUE];
  (void)unique_weights(ens->map_form, ens->h, tau, d.drift);
  for (int u = 0; u < MAX_UNIQUE; ++u) {
    d.ka2[u] = 2.0 * tau[u] * ens->eps;
    d.ka4[u] = 4.0 * tau[u] * ens->eps;
    d.kw2[u] = 2.0 * tau[u];
    d.kw4[u] = 4.0 * tau[u];
  }
  d.eps = ens->eps;
  d.T = ens->n_steps;
  d.N = N;
  d.ckpt = std::min(ckpt_every, ens->n_steps);
  d.n_seg = (d.T + d.ckpt - 1) / d.ckpt;
  d.ic = ic_dev;
  d.gJ = grad_J_dev;
  d.J = J_out_dev;
  d.gic = grad_ic_dev;
  d.geps = grad_eps_dev;
  d.ckpts = (double *)workspace_dev;
  d.steps = reversible ? nullptr : d.ckpts + (size_t)(d.n_seg + 1) * 6 * (size_t)N;
  return AW_OK;
}

aw_status aw_indicator_grad(const aw_ensemble *ens, const double *ic_dev, const double *grad_J_dev,
                            int64_t ckpt_every, double *J_out_dev, double *grad_ic_dev, double *grad_eps_dev,
                            void *workspace_dev, size_t ws_bytes, const aw_tuning *tuning, void *stream) {
  AdjDesc d;
  Tuning t;
  aw_status st = adj_setup(ens, ic_dev, grad_J_dev, ckpt_every, J_out_dev, grad_ic_dev, grad_eps_dev, workspace_dev,
                           ws_bytes, tuning, "aw_indicator_grad", false, d, t);
  if (st != AW_OK) return st;
  d.fwd_steps = d.n_seg == 1 ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_adj_forward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint forward launch");
  e = launch_adj_backward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint backward launch");
  return AW_OK;
}

aw_status aw_indicator_grad_reversible(const aw_ensemble *ens, const double *ic_dev, const double *grad_J_dev,
                                       int64_t ckpt_every, double *J_out_dev, double *grad_ic_dev,
                                       double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                                       const aw_tuning *tuning, void *stream) {
  AdjDesc d;
  Tuning t;
  aw_status st = adj_setup(ens, ic_dev, grad_J_dev, ckpt_every, J_out_dev, grad_ic_dev, grad_eps_dev, workspace_dev,
                           ws_bytes, tuning, "aw_indicator_grad_reversible", true, d, t);
  if (st != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_adj_forward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint forward launch");
  e = launch_adj_backward_reversible(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint reversible backward launch");
  return AW_OK;
}

aw_status aw_ftle_grad_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes) {
  if (!bytes) return fail(AW_EINVAL, "null bytes");
  if (!ens) return fail(AW_EINVAL, "null ensemble");
  if (ckpt_every < 1) return fail(AW_EINVAL, "ckpt_every must be >= 1");
  if (ens->n_steps < 1) return fail(AW_EINVAL, "n_steps must be >= 1");
  const int64_t N = ens_size(*ens);
  if (N < 0) return fail(AW_EINVAL, "bad ensemble size");
  const int64_t ck = std::min(ckpt_every, ens->n_steps);
  const int64_t n_seg = (ens->n_steps + ck - 1) / ck;
  // checkpoints, the final state and one segment's kept step states (12
  // doubles per orbit each), then one 16-bit rescale exponent per orbit per 8 steps
  *bytes = sizeof(double) * 12 * (size_t)N * (size_t)(n_seg + 1 + adj_slots_max(ck)) +
           sizeof(int16_t) * (size_t)N * (size_t)(ens->n_steps / 8);
  return AW_OK;
}

aw_status aw_ftle_grad_reversible_workspace(const aw_ensemble *ens, int64_t ckpt_every, size_t *bytes) {
  size_t full = 0;
  aw_status st = aw_ftle_grad_workspace(ens, ckpt_every, &full);
  if (st != AW_OK) return st;
  const int64_t N = ens_size(*ens);
  const int64_t ck = std::min(ckpt_every, ens->n_steps);
  const int64_t n_seg = (ens->n_steps + ck - 1) / ck;
  // checkpoints and the final state (12 doubles per orbit each), then the
  // rescale exponents
  *bytes = sizeof(double) * 12 * (size_t)N * (size_t)(n_seg + 1) +
           sizeof(int16_t) * (size_t)N * (size_t)(ens->n_steps / 8);
  return AW_OK;
}

// Validation and descriptor of the adjoint of L (both sweeps).
static aw_status ftle_setup(const aw_ensemble *ens, const double *ic_dev, const double *w0_dev,
                            const double *grad_L_dev, int64_t ckpt_every, double *L_out_dev, double *grad_ic_dev,
                            double *grad_eps_dev, void *workspace_dev, size_t ws_bytes, const aw_tuning *tuning,
                            const char *who, bool reversible, FtleDesc &d, Tuning &t) {
  aw_status st = check_ensemble(ens, ic_dev, 0);
  if (st != AW_OK) return st;
  if (ens->ic_kind != AW_IC_EXPLICIT) return fail(AW_EINVAL, "%s needs an EXPLICIT ensemble", who);
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  size_t need = 0;
  st = reversible ? aw_ftle_grad_reversible_workspace(ens, ckpt_every, &need)
                  : aw_ftle_grad_workspace(ens, ckpt_every, &need);
  if (st != AW_OK) return st;
  const int64_t N = ens_size(*ens);
  if (N > 0 && !w0_dev) return fail(AW_EINVAL, "null tangent start");
  if (N > 0 && (!grad_ic_dev || !grad_eps_dev)) return fail(AW_EINVAL, "null gradient outputs");
  if (ws_bytes < need || (N > 0 && !workspace_dev))
    return fail(AW_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  std::memset(&d, 0, sizeof d);
  double tau[MAX_UNIQUE];
  (void)unique_weights(ens->map_form, ens->h, tau, d.drift);
  for (int u = 0; u < MAX_UNIQUE; ++u) {
    d.ka2[u] = 2.0 * tau[u] * ens->eps;
    d.ka4[u] = 4.0 * tau[u] * ens->eps;
    d.kw2[u] = 2.0 * tau[u];
    d.kw4[u] = 4.0 * tau[u];
  }
  d.eps = ens->eps;
  d.T = ens->n_steps;
  d.N = N;
  d.ckpt = std::min(ckpt_every, ens->n_steps);
  d.n_seg = (d.T + d.ckpt - 1) / d.ckpt;
  d.ic = ic_dev;
  d.w0 = w0_dev;
  d.gL = grad_L_dev;
  d.L = L_out_dev;
  d.gic = grad_ic_dev;
  d.geps = grad_eps_dev;
  d.ckpts = (double *)workspace_dev;
  if (reversible) {
    d.steps = nullptr;
    d.exps = (int16_t *)(d.ckpts + (size_t)(d.n_seg + 1) * 12 * (size_t)N);
  } else {
    d.steps = d.ckpts + (size_t)(d.n_seg + 1) * 12 * (size_t)N;
    d.exps = (int16_t *)(d.steps + (size_t)adj_slots_max(d.ckpt) * 12 * (size_t)N);
  }
  return AW_OK;
}

aw_status aw_ftle_grad(const aw_ensemble *ens, const double *ic_dev, const double *w0_dev, const double *grad_L_dev,
                       int64_t ckpt_every, double *L_out_dev, double *grad_ic_dev, double *grad_eps_dev,
                       void *workspace_dev, size_t ws_bytes, const aw_tuning *tuning, void *stream) {
  FtleDesc d;
  Tuning t;
  aw_status st = ftle_setup(ens, ic_dev, w0_dev, grad_L_dev, ckpt_every, L_out_dev, grad_ic_dev, grad_eps_dev,
                            workspace_dev, ws_bytes, tuning, "aw_ftle_grad", false, d, t);
  if (st != AW_OK) return st;
  d.fwd_steps = d.n_seg == 1 ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_ftle_forward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "FTLE-gradient forward launch");
  e = launch_ftle_backward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "FTLE-gradient backward launch");
  return AW_OK;
}

aw_status aw_ftle_grad_reversible(const aw_ensemble *ens, const double *ic_dev, const double *w0_dev,
                                  const double *grad_L_dev, int64_t ckpt_every, double *L_out_dev,
                                  double *grad_ic_dev, double *grad_eps_dev, void *workspace_dev, size_t ws_bytes,
                                  const aw_tuning *tuning, void *stream) {
  FtleDesc d;
  Tuning t;
  aw_status st = ftle_setup(ens, ic_dev, w0_dev, grad_L_dev, ckpt_every, L_out_dev, grad_ic_dev, grad_eps_dev,
                            workspace_dev, ws_bytes, tuning, "aw_ftle_grad_reversible", true, d, t);
  if (st != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_ftle_forward(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "FTLE-gradient forward launch");
  e = launch_ftle_backward_reversible(d, ens->map_form, t, s);
  if (e != hipSuccess) return hip_fail(e, "FTLE-gradient reversible backward launch");
  return AW_OK;
}

// ---------------------------------------------------------------------------
// Graphs of the batched image path.
// ---------------------------------------------------------------------------
struct aw_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void *> dev_allocs;
};

aw_status aw_graph_create(const aw_ensemble *ens, int32_t n_ens, const aw_image_spec *spec, double *const *image_dev,
                          uint32_t *const *counts_dev, uint8_t *const *cls_dev, const aw_tuning *tuning,
                          aw_graph **out) {
  if (!out) return fail(AW_EINVAL, "null graph handle");
  *out = nullptr;
  aw_status st = validate_batch(ens, n_ens, nullptr);
  if (st != AW_OK) return st;
  if (!spec || !image_dev) return fail(AW_EINVAL, "null image spec or array");
  for (int e = 0; e < n_ens; ++e)
    if (ens[e].ic_kind == AW_IC_EXPLICIT) return fail(AW_EINVAL, "graph ensembles generate their initial conditions");
  Tuning t;
  if ((st = check_tuning(tuning, t)) != AW_OK) return st;
  ImageCall c;
  if ((st = prepare_image(ens, n_ens, spec, image_dev, counts_dev, cls_dev, t, true, c)) != AW_OK) return st;
  aw_graph *g = new aw_graph();
  auto cleanup = [&](aw_status s2) {
    aw_graph_destroy(g);
    return s2;
  };
  // The graph owns its scratch area (histogram items and sort buffers, batch tables).
  void *area = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&area, c.lay.total)) != hipSuccess)
    return cleanup(fail(AW_ENOMEM, "graph scratch of %zu bytes: %s", c.lay.total, hipGetErrorString(e)));
  g->dev_allocs.push_back(area);
  char *base = (char *)area;
  place_image(c, base);
  if (c.batched && !c.items.empty()) {
    if ((e = hipMemcpy(base + c.lay.descs, c.descs.data(), c.descs.size() * sizeof(FwdDesc),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(base + c.lay.items, c.items.data(), c.items.size() * sizeof(WorkItem),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "graph table upload"));
  }
  hipStream_t cs;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return cleanup(hip_fail(e, "stream"));
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return cleanup(hip_fail(e, "graph capture"));
  }
  // Every launch status is checked; on a failure the capture is still ended
  // (and its partial graph destroyed) before the error is returned.
  st = enqueue_image(c, base, spec, image_dev, counts_dev, t, cs, false);
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (st != AW_OK) return cleanup(st);
  if (e != hipSuccess) return cleanup(hip_fail(e, "graph capture"));
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return cleanup(hip_fail(e, "graph instantiate"));
  *out = g;
  return AW_OK;
}

aw_status aw_graph_launch(aw_graph *g, void *stream) {
  if (!g || !g->exec) return fail(AW_EINVAL, "null graph");
  hipError_t e;
  {
    TimedLaunch tl((hipStream_t)stream);
    e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return AW_OK;
}

void aw_graph_destroy(aw_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (!g->dev_allocs.empty()) (void)hipDeviceSynchronize();
  for (void *p : g->dev_allocs) (void)hipFree(p);
  delete g;
}

aw_status aw_timing_enable(int32_t on) {
  g_timing = on != 0;
  return AW_OK;
}

aw_status aw_timing_read(double *ms, int64_t *launches) {
  double total = 0.0;
  int64_t n = 0;
  for (auto &ev : g_events) {
    hipError_t e = hipEventSynchronize(ev.second);
    float t = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&t, ev.first, ev.second) == hipSuccess) {
      total += t;
      ++n;
    }
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  g_events.clear();
  if (ms) *ms = total;
  if (launches) *launches = n;
  return AW_OK;
}

aw_status aw_step_op_counts(int32_t map_form, int32_t tangent, int64_t *fma, int64_t *mul, int64_t *add) {
  if (!fma || !mul || !add) return fail(AW_EINVAL, "null output");
  if (map_form != AW_MAP_STDMAP && map_form != AW_MAP_S2 && map_form != AW_MAP_S4 && map_form != AW_MAP_S6 &&
      map_form != AW_MAP_Y6)
    return fail(AW_EINVAL, "unknown map_form");
  step_op_counts(map_form, tangent != 0, fma, mul, add);
  return AW_OK;
}

}  // extern "C"
