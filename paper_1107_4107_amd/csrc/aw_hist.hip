// aw_hist.hip -- image reductions of per-orbit (bin, value) items.
//
// The W x H image (512 x 512 for the large ensemble: 3 MB of counts and
// sums) does not fit in the 160 KB LDS of a CU, so the reduction is:
//   1. count   : each block counts its items per image tile in LDS;
//   2. scan    : one workgroup per tile turns its row of per-block counts into
//                offsets within the tile, and one more scans the tile totals,
//                so every tile's items become one contiguous range;
//   3. scatter : each block moves its items to their tile's range (LDS cursors);
//   4. accumulate: one workgroup per chunk of a tile's range (a tile of few
//                items is one chunk) adds its items into a TILE_W x TILE_H
//                tile of counts (ds_add_u32) and sums (ds_add_f64) held in LDS
//                and writes the finished tile out, or, for a tile of several
//                chunks, its partial tile;
//   5. merge   : one workgroup per tile of several chunks adds their partial
//                tiles in chunk order and writes the tile out -- no global
//                atomics anywhere.
// Counts are exact and independent of scheduling; the order of the float
// additions inside a chunk is not, so sums can differ in the last bits.
#include <hip/hip_runtime.h>
#include <math.h>

#include "aw_hist.hpp"
#include "aw_internal.hpp"
#include "aw_launch.hpp"

namespace aw {

static_assert(ACC_BLOCK == TILE_BINS, "the merge runs one lane per bin, as many as the accumulation's lanes");

__device__ __forceinline__ uint32_t bin_of_h(double a, double b, double lo0, double hi0, double lo1,
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

// The items' values are read where the caller keeps them, by the scatter.
__global__ void k_hist_bins(int64_t N, const double *__restrict__ a, const double *__restrict__ b, double lo0,
                            double hi0, double lo1, double hi1, int W, int H, int closed,
                            uint32_t *__restrict__ bins) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  bins[n] = bin_of_h(a[n], b[n], lo0, hi0, lo1, hi1, W, H, closed != 0);
}

__global__ void k_vdir_keys(int64_t N, const double *__restrict__ V, double *__restrict__ phi,
                            double *__restrict__ mu) {
#pragma clang fp contract(off)
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double vx = V[n], vy = V[N + n], vz = V[2 * N + n];
  const double r = sqrt(vx * vx + vy * vy + vz * vz);
  if (r == 0.0) {
    phi[n] = __builtin_nan("");
    mu[n] = __builtin_nan("");
    return;
  }
  phi[n] = atan2(vy, vx);
  mu[n] = vz / r;
}

struct TileGeom {
  int W, H, tiles_x, n_tiles;
};

__device__ __forceinline__ void tile_of(uint32_t bin, const TileGeom &g, int &tile, int &local) {
  const int i = (int)(bin % (uint32_t)g.W), j = (int)(bin / (uint32_t)g.W);
  tile = (j / TILE_H) * g.tiles_x + i / TILE_W;
  local = (j % TILE_H) * TILE_W + (i % TILE_W);
}

// Both per-block kernels hold one LDS word per tile, sized at launch to the
// image (n_tiles + 1 words), so that a small image leaves room for more
// blocks per CU.
extern __shared__ uint32_t tile_words[];

// 1. Per-block tile counts; dropped items per block.
__global__ __launch_bounds__(HIST_BLOCK) void k_tile_count(int64_t N, const uint32_t *__restrict__ bins,
                                                           TileGeom g, int32_t G,
                                                           uint32_t *__restrict__ block_counts,
                                                           uint32_t *__restrict__ block_dropped) {
  uint32_t *cnt = tile_words;
  uint32_t &drop = tile_words[g.n_tiles];
  for (int t = threadIdx.x; t < g.n_tiles; t += blockDim.x) cnt[t] = 0u;
  if (threadIdx.x == 0) drop = 0u;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * HIST_ITEMS_PER_BLOCK;
  const int64_t end = beg + HIST_ITEMS_PER_BLOCK < N ? beg + HIST_ITEMS_PER_BLOCK : N;
  const int64_t bd = blockDim.x;
  uint32_t my_drop = 0;
  auto count = [&](uint32_t bin) {
    if (bin == BIN_DROP) {
      ++my_drop;
      return;
    }
    int tile, local;
    tile_of(bin, g, tile, local);
    atomicAdd(&cnt[tile], 1u);
  };
  int64_t n = beg + threadIdx.x;
  for (; n + 3 * bd < end; n += 4 * bd) {  // four loads in flight per lane
    uint32_t b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = bins[n + k * bd];
#pragma unroll
    for (int k = 0; k < 4; ++k) count(b[k]);
  }
  for (; n < end; n += bd) count(bins[n]);
  if (my_drop) atomicAdd(&drop, my_drop);
  __syncthreads();
  for (int t = threadIdx.x; t < g.n_tiles; t += blockDim.x)
    block_counts[(int64_t)t * G + blockIdx.x] = cnt[t];
  if (threadIdx.x == 0) block_dropped[blockIdx.x] = drop;
}

// 2a. Exclusive scan of one tile's row of per-block counts, in place (one
//     workgroup per tile; the row is read and written in coalesced chunks of
//     SCAN_BLOCK entries, scanned by wave shuffles); the row total goes to
//     tile_total[t].
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan_rows(uint32_t *__restrict__ counts, int32_t G,
                                                               uint32_t *__restrict__ tile_total) {
  constexpr int NW = SCAN_BLOCK / 64;
  __shared__ uint32_t wsum[NW];
  uint32_t *row = counts + (int64_t)blockIdx.x * G;
  const int lane = (int)__lane_id(), wv = (int)(threadIdx.x >> 6);
  uint32_t carry = 0;
  for (int32_t base = 0; base < G; base += SCAN_BLOCK) {
    const int32_t e = base + (int32_t)threadIdx.x;
    const uint32_t v = e < G ? row[e] : 0u;
    uint32_t x = v;  // inclusive scan within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t before = carry, total = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      before += k < wv ? wsum[k] : 0u;
      total += wsum[k];
    }
    if (e < G) row[e] = before + x - v;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_total[blockIdx.x] = carry;
}

// Accumulation chunks of a tile of c items (at least one, so that every tile
// is written out).
__device__ __forceinline__ uint32_t n_chunks(uint32_t c, uint32_t chunk) {
  return c == 0u ? 1u : (c + chunk - 1u) / chunk;
}

// 2b. Exclusive scans of the tile totals, of the tiles' chunk counts and of
//     the partial-tile slots of tiles of several chunks, and the count of
//     dropped items (one workgroup of 1024 lanes): tile_start[t] = first
//     sorted position of tile t, tile_start[n_tiles] = items kept;
//     chunk_first[t] = first chunk of tile t, chunk_first[n_tiles] = chunks in
//     all; part_first[t] = first partial slot of tile t; chunk_tile[c] = the
//     tile of chunk c.
__global__ __launch_bounds__(1024) void k_tile_scan_tiles(const uint32_t *__restrict__ tile_total, int32_t n_tiles,
                                                          const uint32_t *__restrict__ block_dropped, int32_t G,
                                                          uint32_t chunk, uint32_t *__restrict__ tile_start,
                                                          uint32_t *__restrict__ chunk_first,
                                                          uint32_t *__restrict__ part_first,
                                                          uint32_t *__restrict__ chunk_tile,
                                                          uint64_t *__restrict__ dropped_out) {
  __shared__ uint32_t part[1024], pch[1024], ppt[1024];
  __shared__ uint64_t dsum[1024];
  const int tid = threadIdx.x;
  const int per = (n_tiles + 1023) / 1024;
  const int beg = tid * per;
  const int end = beg + per < n_tiles ? beg + per : n_tiles;
  uint32_t s = 0, sc = 0, sp = 0;
  for (int t = beg; t < end; ++t) {
    const uint32_t c = tile_total[t], k = n_chunks(c, chunk);
    s += c;
    sc += k;
    sp += k > 1u ? k : 0u;
  }
  part[tid] = s;
  pch[tid] = sc;
  ppt[tid] = sp;
  uint64_t d = 0;
  for (int b = tid; b < G; b += 1024) d += block_dropped[b];
  dsum[tid] = d;
  __syncthreads();
  // Hillis-Steele inclusive scans of the 1024 partial sums.
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = tid >= off ? part[tid - off] : 0u;
    const uint32_t vc = tid >= off ? pch[tid - off] : 0u;
    const uint32_t vp = tid >= off ? ppt[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    pch[tid] += vc;
    ppt[tid] += vp;
    __syncthreads();
  }
  uint32_t run = tid > 0 ? part[tid - 1] : 0u;
  uint32_t runc = tid > 0 ? pch[tid - 1] : 0u;
  uint32_t runp = tid > 0 ? ppt[tid - 1] : 0u;
  for (int t = beg; t < end; ++t) {
    const uint32_t c = tile_total[t], k = n_chunks(c, chunk);
    tile_start[t] = run;
    chunk_first[t] = runc;
    part_first[t] = runp;
    for (uint32_t q = 0; q < k; ++q) chunk_tile[runc + q] = (uint32_t)t;
    run += c;
    runc += k;
    runp += k > 1u ? k : 0u;
  }
  if (tid == 1023) {
    tile_start[n_tiles] = part[1023];
    chunk_first[n_tiles] = pch[1023];
    part_first[n_tiles] = ppt[1023];
  }
  // Tree sum of the dropped counts.
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) dsum[tid] += dsum[tid + off];
    __syncthreads();
  }
  if (tid == 0 && dropped_out) *dropped_out = dsum[0];
}

// 3. Move each block's items to their tile ranges.
__global__ __launch_bounds__(HIST_BLOCK) void k_tile_scatter(int64_t N, const uint32_t *__restrict__ bins,
                                                             const double *__restrict__ vals, TileGeom g,
                                                             int32_t G, const uint32_t *__restrict__ offsets,
                                                             const uint32_t *__restrict__ tile_start,
                                                             uint16_t *__restrict__ sorted_local,
                                                             double *__restrict__ sorted_val) {
  uint32_t *cur = tile_words;
  for (int t = threadIdx.x; t < g.n_tiles; t += blockDim.x)
    cur[t] = tile_start[t] + offsets[(int64_t)t * G + blockIdx.x];
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * HIST_ITEMS_PER_BLOCK;
  const int64_t end = beg + HIST_ITEMS_PER_BLOCK < N ? beg + HIST_ITEMS_PER_BLOCK : N;
  const int64_t bd = blockDim.x;
  auto place = [&](int64_t n, uint32_t bin) {
    if (bin == BIN_DROP) return;
    int tile, local;
    tile_of(bin, g, tile, local);
    const uint32_t pos = atomicAdd(&cur[tile], 1u);
    sorted_local[pos] = (uint16_t)local;
    if (vals) sorted_val[pos] = vals[n];
  };
  int64_t n = beg + threadIdx.x;
  for (; n + 3 * bd < end; n += 4 * bd) {  // four loads in flight per lane
    uint32_t b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = bins[n + k * bd];
#pragma unroll
    for (int k = 0; k < 4; ++k) place(n + k * bd, b[k]);
  }
  for (; n < end; n += bd) place(n, bins[n]);
}

// 3'. The same through LDS, for items with values and images of at most
//     STAGE_MAX_TILES tiles (2-byte keys alone coalesce well enough): each
//     round of STAGE_ITEMS items is grouped by tile in LDS first, then every
//     tile's run is written to consecutive positions, so that the stores fill
//     whole lines instead of landing one item per line (written back as
//     partial lines from several XCDs' L2s otherwise).  A lane loads its
//     round's keys and values once, into registers, and the count's LDS
//     atomic gives each item its rank within its tile for the round.
__global__ __launch_bounds__(STAGE_BLOCK) void k_tile_scatter_staged(int64_t N, const uint32_t *__restrict__ bins,
                                                                   const double *__restrict__ vals, TileGeom g,
                                                                   int32_t G, const uint32_t *__restrict__ offsets,
                                                                   const uint32_t *__restrict__ tile_start,
                                                                   uint16_t *__restrict__ sorted_local,
                                                                   double *__restrict__ sorted_val) {
  constexpr int NW = STAGE_BLOCK / 64;
  constexpr int IPL = STAGE_ITEMS / STAGE_BLOCK;  // items per lane and round
  static_assert(IPL * STAGE_BLOCK == STAGE_ITEMS, "a round is a whole number of items per lane");
  __shared__ double st_val[STAGE_ITEMS];
  __shared__ uint32_t base[STAGE_MAX_TILES], lcnt[STAGE_MAX_TILES], lstart[STAGE_MAX_TILES];
  __shared__ uint16_t st_local[STAGE_ITEMS], st_tile[STAGE_ITEMS];
  __shared__ uint32_t wsum[NW];
  const int nt = g.n_tiles;
  const int tid = threadIdx.x, lane = (int)__lane_id(), wv = tid >> 6;
  for (int t = tid; t < nt; t += blockDim.x) base[t] = tile_start[t] + offsets[(int64_t)t * G + blockIdx.x];
  const int64_t beg = (int64_t)blockIdx.x * HIST_ITEMS_PER_BLOCK;
  const int64_t end = beg + HIST_ITEMS_PER_BLOCK < N ? beg + HIST_ITEMS_PER_BLOCK : N;
  for (int64_t r0 = beg; r0 < end; r0 += STAGE_ITEMS) {
    uint32_t bin[IPL];
    double val[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int64_t n = r0 + tid + (int64_t)k * STAGE_BLOCK;
      bin[k] = n < end ? bins[n] : BIN_DROP;
      val[k] = n < end && vals ? vals[n] : 0.0;
    }
    for (int t = tid; t < nt; t += blockDim.x) lcnt[t] = 0u;
    __syncthreads();
    int tile[IPL];
    uint32_t rank[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      tile[k] = -1;
      if (bin[k] == BIN_DROP) continue;
      int local;
      tile_of(bin[k], g, tile[k], local);
      bin[k] = (uint32_t)local;
      rank[k] = atomicAdd(&lcnt[tile[k]], 1u);
    }
    __syncthreads();
    // Exclusive scan of the round's tile counts (nt <= STAGE_MAX_TILES = blockDim.x).
    const uint32_t v = tid < nt ? lcnt[tid] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t before = 0, kept = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      before += k < wv ? wsum[k] : 0u;
      kept += wsum[k];
    }
    if (tid < nt) lstart[tid] = before + x - v;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      if (tile[k] < 0) continue;
      const uint32_t slot = lstart[tile[k]] + rank[k];
      st_local[slot] = (uint16_t)bin[k];
      st_tile[slot] = (uint16_t)tile[k];
      st_val[slot] = val[k];
    }
    __syncthreads();
    for (uint32_t i = tid; i < kept; i += blockDim.x) {
      const int t = st_tile[i];
      const uint32_t pos = base[t] + (i - lstart[t]);
      sorted_local[pos] = st_local[i];
      if (vals) sorted_val[pos] = st_val[i];
    }
    __syncthreads();
    for (int t = tid; t < nt; t += blockDim.x) base[t] += lcnt[t];
    __syncthreads();
  }
}

// Bin k of tile t, from its count and sum.  mode 0: counts + sums;
// 1: counts + mean; 2: counts + density (count * norm).  accumulate: counts
// are added to what counts_out holds.
__device__ __forceinline__ void write_bin(const TileGeom &g, int t, int k, uint32_t cc, double sk, int32_t mode,
                                          double norm, int32_t accumulate, uint32_t *__restrict__ counts_out,
                                          double *__restrict__ f_out) {
  const int tx = t % g.tiles_x, ty = t / g.tiles_x;
  const int i = tx * TILE_W + (k % TILE_W), j = ty * TILE_H + (k / TILE_W);
  if (i >= g.W || j >= g.H) return;
  const int64_t o = (int64_t)j * g.W + i;
  if (counts_out) counts_out[o] = accumulate ? counts_out[o] + cc : cc;
  if (f_out) {
    double f;
    if (mode == 0) f = sk;
    else if (mode == 1) f = cc ? sk / (double)cc : 0.0;
    else f = (double)cc * norm;
    f_out[o] = f;
  }
}

// 4. One workgroup per chunk: LDS accumulation of the chunk's items, then the
//    tile is written out (a tile of one chunk) or left as the chunk's partial
//    tile (a tile of several).  Each lane takes four items per pass so that
//    four loads are in flight.
__global__ __launch_bounds__(ACC_BLOCK) void k_tile_accum(const uint32_t *__restrict__ tile_start,
                                                           const uint32_t *__restrict__ chunk_first,
                                                           const uint32_t *__restrict__ part_first,
                                                           const uint32_t *__restrict__ chunk_tile, uint32_t chunk,
                                                           const uint16_t *__restrict__ sorted_local,
                                                           const double *__restrict__ sorted_val,
                                                           TileGeom g, int32_t mode, double norm, int32_t accumulate,
                                                           uint32_t *__restrict__ counts_out,
                                                           double *__restrict__ f_out,
                                                           uint32_t *__restrict__ part_counts,
                                                           double *__restrict__ part_sums) {
  __shared__ uint32_t c[TILE_BINS];
  __shared__ double s[TILE_BINS];
  const uint32_t w = blockIdx.x;
  if (w >= chunk_first[g.n_tiles]) return;  // the grid bounds the chunk count from above
  const int t = (int)chunk_tile[w];
  const uint32_t c0 = chunk_first[t], nch = chunk_first[t + 1] - c0;
  const uint32_t te = tile_start[t + 1];
  const uint32_t beg = tile_start[t] + (w - c0) * chunk;
  const uint32_t end = te - beg > chunk ? beg + chunk : te;
  for (int k = threadIdx.x; k < TILE_BINS; k += blockDim.x) {
    c[k] = 0u;
    s[k] = 0.0;
  }
  __syncthreads();
  const bool have_vals = sorted_val != nullptr;
  const uint32_t bd = blockDim.x;
  uint32_t p = beg + threadIdx.x;
  for (; p + 3 * bd < end; p += 4 * bd) {
    int loc[4];
    double val[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) loc[k] = sorted_local[p + k * bd];
    if (have_vals) {
#pragma unroll
      for (int k = 0; k < 4; ++k) val[k] = sorted_val[p + k * bd];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      atomicAdd(&c[loc[k]], 1u);
      if (have_vals) atomicAdd(&s[loc[k]], val[k]);
    }
  }
  for (; p < end; p += bd) {
    const int loc = sorted_local[p];
    atomicAdd(&c[loc], 1u);
    if (have_vals) atomicAdd(&s[loc], sorted_val[p]);
  }
  __syncthreads();
  if (nch == 1u) {
    for (int k = threadIdx.x; k < TILE_BINS; k += blockDim.x)
      write_bin(g, t, k, c[k], s[k], mode, norm, accumulate, counts_out, f_out);
  } else {
    const int64_t slot = (int64_t)(part_first[t] + (w - c0)) * TILE_BINS;
    for (int k = threadIdx.x; k < TILE_BINS; k += blockDim.x) {
      part_counts[slot + k] = c[k];
      if (have_vals) part_sums[slot + k] = s[k];
    }
  }
}

// 5. One workgroup of TILE_BINS lanes per tile; tiles of several chunks add
//    their partial tiles in chunk order (lane k: bin k) and write the tile out.
__global__ __launch_bounds__(TILE_BINS) void k_tile_merge(const uint32_t *__restrict__ chunk_first,
                                                           const uint32_t *__restrict__ part_first, TileGeom g,
                                                           int32_t mode, double norm, int32_t accumulate,
                                                           const uint32_t *__restrict__ part_counts,
                                                           const double *__restrict__ part_sums,
                                                           uint32_t *__restrict__ counts_out,
                                                           double *__restrict__ f_out) {
  const int t = blockIdx.x, k = threadIdx.x;
  const uint32_t nch = chunk_first[t + 1] - chunk_first[t];
  if (nch < 2u) return;
  const int64_t p0 = part_first[t];
  uint32_t cc = 0;
  double sk = 0.0;
  for (uint32_t q = 0; q < nch; ++q) {
    const int64_t o = (p0 + q) * TILE_BINS + k;
    cc += part_counts[o];
    if (part_sums) sk += part_sums[o];
  }
  write_bin(g, t, k, cc, sk, mode, norm, accumulate, counts_out, f_out);
}

hipError_t launch_hist_bins(int64_t N, const double *a, const double *b, double lo0, double hi0, double lo1,
                            double hi1, int W, int H, int closed, uint32_t *bins, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist_bins, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, a, b, lo0, hi0, lo1,
                     hi1, W, H, closed, bins);
  return hipGetLastError();
}

hipError_t launch_vdir_keys(int64_t N, const double *V, double *phi, double *mu, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vdir_keys, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, V, phi, mu);
  return hipGetLastError();
}

HistPlan hist_plan(int64_t N, int W, int H) {
  HistPlan p;
  p.W = W;
  p.H = H;
  p.tiles_x = (W + TILE_W - 1) / TILE_W;
  p.n_tiles = p.tiles_x * ((H + TILE_H - 1) / TILE_H);
  p.G = (int32_t)((N + HIST_ITEMS_PER_BLOCK - 1) / HIST_ITEMS_PER_BLOCK);
  if (p.G < 1) p.G = 1;
  const int64_t n = N > 0 ? N : 0;
  p.chunk = acc_chunk(n, p.n_tiles);
  p.max_chunks = p.n_tiles + (n + p.chunk - 1) / p.chunk;
  return p;
}

hipError_t launch_hist_reduce(int64_t N, const uint32_t *bins, const double *vals, const HistPlan &p,
                              const HistScratch &w, int mode, double norm, uint32_t *counts_out,
                              double *f_out, uint64_t *dropped_out, hipStream_t s, int accumulate) {
  TileGeom g{p.W, p.H, p.tiles_x, p.n_tiles};
  const unsigned tile_lds = (unsigned)(sizeof(uint32_t) * ((size_t)p.n_tiles + 1));  // <= 32 KB + 4 B
  if (N > 0) {
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)p.G), dim3(HIST_BLOCK), tile_lds, s, N, bins, g, p.G,
                       w.block_counts, w.block_dropped);
  } else {
    hipError_t e = launch_zero_u32(w.block_counts, p.n_tiles * p.G, s);
    if (e != hipSuccess) return e;
    e = launch_zero_u32(w.block_dropped, p.G, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tile_scan_rows, dim3((unsigned)p.n_tiles), dim3(SCAN_BLOCK), 0, s, w.block_counts, p.G,
                     w.tile_total);
  hipLaunchKernelGGL(k_tile_scan_tiles, dim3(1), dim3(1024), 0, s, w.tile_total, p.n_tiles, w.block_dropped, p.G,
                     (uint32_t)p.chunk, w.tile_start, w.chunk_first, w.part_first, w.chunk_tile, dropped_out);
  if (N > 0 && vals && p.n_tiles <= STAGE_MAX_TILES)
    hipLaunchKernelGGL(k_tile_scatter_staged, dim3((unsigned)p.G), dim3(STAGE_BLOCK), 0, s, N, bins, vals, g, p.G,
                       w.block_counts, w.tile_start, w.sorted_local, vals ? w.sorted_val : nullptr);
  else if (N > 0)
    hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)p.G), dim3(HIST_BLOCK), tile_lds, s, N, bins, vals, g, p.G,
                       w.block_counts, w.tile_start, w.sorted_local, vals ? w.sorted_val : nullptr);
  double *psums = vals ? w.part_sums : nullptr;
  hipLaunchKernelGGL(k_tile_accum, dim3((unsigned)p.max_chunks), dim3(ACC_BLOCK), 0, s, w.tile_start,
                     w.chunk_first, w.part_first, w.chunk_tile, (uint32_t)p.chunk, w.sorted_local,
                     vals ? w.sorted_val : nullptr, g, mode, norm, accumulate, counts_out, f_out, w.part_counts,
                     psums);
  if (N > p.chunk)  // else no tile has several chunks
    hipLaunchKernelGGL(k_tile_merge, dim3((unsigned)p.n_tiles), dim3(TILE_BINS), 0, s, w.chunk_first, w.part_first,
                       g, mode, norm, accumulate, w.part_counts, psums, counts_out, f_out);
  return hipGetLastError();
}

}  // namespace aw
