// aw_hist.hpp -- geometry of the image reduction (internal).
#pragma once

#include "aw_internal.hpp"

namespace aw {

// Histogram reduction geometry: the W x H image is cut into tiles of
// TILE_W x TILE_H bins; a tile's counts and sums fit in LDS.
constexpr int TILE_W = 32;
constexpr int TILE_H = 32;
constexpr int TILE_BINS = TILE_W * TILE_H;
constexpr int HIST_BLOCK = 256;
constexpr int HIST_ITEMS_PER_BLOCK = 8192;  // items per block in count/scatter
constexpr int ACC_BLOCK = 1024;             // lanes per tile in the accumulation
constexpr int SCAN_BLOCK = 256;             // lanes per tile row in the scan
constexpr int MAX_TILES = 8192;
constexpr int STAGE_MAX_TILES = 1024;       // images up to this many tiles scatter through LDS
constexpr int STAGE_ITEMS = 4096;           // items per LDS staging round
constexpr int STAGE_BLOCK = 1024;

// The accumulation splits every tile's sorted range into chunks of at most
// acc_chunk(N, T) items, one workgroup each; a tile of several chunks leaves a
// partial tile per chunk, which a second kernel adds up in chunk order.  The
// chunk is at least ACC_CHUNK_MIN items, and otherwise twice a tile's share of
// a uniform image (uniform tiles stay whole) but no more than N / 256 (at
// least one chunk per CU), rounded up to a multiple of 4096.  Since
// chunk >= max(ACC_CHUNK_MIN, min(2 N / T, N / 256)), N / chunk is at most
// acc_bound(N, T), which grows with N: the scratch sized for the largest N of
// a call serves every smaller one.  A call has at most T + ceil(N / chunk)
// chunks, and fewer than 2 ceil(N / chunk) of them belong to tiles of several.
constexpr int64_t ACC_CHUNK_MIN = 16384;
constexpr int64_t ACC_ROUND = 4096;
constexpr int64_t acc_chunk(int64_t N, int64_t T) {
  const int64_t share = 2 * ((N + T - 1) / T), per_cu = (N + 255) / 256;
  const int64_t c = ((share < per_cu ? share : per_cu) + ACC_ROUND - 1) / ACC_ROUND * ACC_ROUND;
  return c > ACC_CHUNK_MIN ? c : ACC_CHUNK_MIN;
}
constexpr int64_t acc_bound(int64_t N, int64_t T) {
  const int64_t a = (N + ACC_CHUNK_MIN - 1) / ACC_CHUNK_MIN, h = (T + 1) / 2, b = h > 256 ? h : 256;
  return a < b ? a : b;
}

}  // namespace aw
