// aw_launch.hpp -- host-side launchers of the kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "aw_internal.hpp"

namespace aw {

struct Tuning {
  int block = 0;  // 0: automatic (block_for)
  int opl = 1;
  int unroll = 1;
  int renorm = 8;
  int pwgs = 0;
  int lpo = 0;    // lanes per orbit of tangent-free intermediate launches: 0 auto, 1 or 2
};

// Lanes per block for a launch over n orbits (or lanes).  A block set in the
// tuning is used as is.  Automatic: 512 when every CU gets at least one block
// of 512 (a block holds the 64 KB sine/cosine table, so two blocks share a CU,
// and it takes two of 512 lanes to fill it at four waves per SIMD; a kernel
// above 128 VGPRs fits one, whose two waves per SIMD still saturate the
// issue); below
// that the largest of 256 and 128 that still gives every CU a block, else 64,
// so that small ensembles spread over as much of the chip as they can.  No
// result depends on the block.
int block_for(const Tuning &t, int64_t n);

// Kernels bounded at 256 lanes per block (the window-test and time-window
// propagation and the batched persistent kernel, whose register counts leave
// room for no more) run a larger or automatic block as 256.
inline int block_256(const Tuning &t) { return (t.block == 0 || t.block > 256) ? 256 : t.block; }

// Propagation.
hipError_t launch_fwd(const FwdDesc &d, const Tuning &t, int form, bool tan, hipStream_t s);
hipError_t launch_fwd_batched(const FwdDesc *descs_dev, const WorkItem *items_dev, int32_t n_items,
                              uint32_t *head_dev, const Tuning &t, int form, bool tan, int n_wg,
                              hipStream_t s);
int persistent_blocks_per_cu(int form, bool tan, const Tuning &t);
hipError_t launch_gen_ic(const FwdDesc &d, double *ic, double *w0, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int32_t n, hipStream_t s);
void step_op_counts(int form, bool tan, int64_t *fma, int64_t *mul, int64_t *add);

// Histogram reduction.
struct HistPlan {
  int W = 0, H = 0, tiles_x = 0, n_tiles = 0;
  int32_t G = 0;
  int64_t chunk = 0;       // items per accumulation chunk
  int64_t max_chunks = 0;  // accumulation workgroups launched: n_tiles + ceil(N / chunk)
};
struct HistScratch {
  uint32_t *block_counts = nullptr;
  uint32_t *block_dropped = nullptr;
  uint32_t *tile_start = nullptr;   // n_tiles + 1 entries
  uint32_t *tile_total = nullptr;   // n_tiles entries (in the same buffer, after tile_start)
  uint32_t *chunk_first = nullptr;  // n_tiles + 1: first chunk of each tile; [n_tiles] = chunks in all
  uint32_t *part_first = nullptr;   // n_tiles + 1: first partial-tile slot of each tile of several chunks
  uint32_t *chunk_tile = nullptr;   // the tile of each chunk
  uint32_t *part_counts = nullptr;  // [slots][TILE_BINS] partial counts
  double *part_sums = nullptr;      // [slots][TILE_BINS] partial sums (with values only)
  uint16_t *sorted_local = nullptr;
  double *sorted_val = nullptr;
};
HistPlan hist_plan(int64_t N, int W, int H);
hipError_t launch_hist_bins(int64_t N, const double *a, const double *b, double lo0, double hi0, double lo1,
                            double hi1, int W, int H, int closed, uint32_t *bins, hipStream_t s);
hipError_t launch_vdir_keys(int64_t N, const double *V, double *phi, double *mu, hipStream_t s);
// accumulate != 0: counts are added to counts_out instead of written.
hipError_t launch_hist_reduce(int64_t N, const uint32_t *bins, const double *vals, const HistPlan &p,
                              const HistScratch &w, int mode, double norm, uint32_t *counts_out,
                              double *f_out, uint64_t *dropped_out, hipStream_t s, int accumulate = 0);

// Adjoint.
hipError_t launch_adj_forward(const AdjDesc &d, int form, const Tuning &t, hipStream_t s);
hipError_t launch_adj_backward(const AdjDesc &d, int form, const Tuning &t, hipStream_t s);
hipError_t launch_adj_backward_reversible(const AdjDesc &d, int form, const Tuning &t, hipStream_t s);

// Gradient of the tangent-growth indicator L: the adjoint descriptor, whose
// checkpoint and step buffers then hold 12 rows (state and tangent) per
// orbit, plus the tangent start, the upstream gradient and L.
struct FtleDesc : AdjDesc {
  const double *w0;  // [6][N]
  const double *gL;  // [N] or null (ones)
  double *L;         // [N] or null
  int16_t *exps;     // [floor(T/8)][N]: exponent of each tangent rescale
};
hipError_t launch_ftle_forward(const FtleDesc &d, int form, const Tuning &t, hipStream_t s);
hipError_t launch_ftle_backward(const FtleDesc &d, int form, const Tuning &t, hipStream_t s);
hipError_t launch_ftle_backward_reversible(const FtleDesc &d, int form, const Tuning &t, hipStream_t s);

}  // namespace aw
