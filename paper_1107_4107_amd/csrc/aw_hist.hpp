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

}  // namespace aw
