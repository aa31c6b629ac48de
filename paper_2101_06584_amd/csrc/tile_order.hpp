// tile_order.hpp -- L2-aware mapping of a 1-D grid onto a tiles_m x tiles_n
// grid of output tiles for gfx950's 8 XCDs (each with its own L2).
//
// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8), so blocks b, b + 8, b + 16, ... share an L2.  They are given
// consecutive logical tile indices, and logical indices walk groups of GM
// tile rows column by column, so the blocks resident on one XCD at a time
// cover a compact GM x (few) block of tiles and share their row panels of
// op(A) and column panels of op(B) in that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

constexpr int kXcds = 8;

// Grid size for `tiles` output tiles (a multiple of the XCD count).
inline int64_t xcd_grid(int64_t tiles) { return (tiles + kXcds - 1) / kXcds * kXcds; }

// Tile (tm, tn) of this block; false for the few padding blocks.
template <int GM>
__device__ __forceinline__ bool xcd_tile_coords(int64_t bid, int64_t tiles_m, int64_t tiles_n,
                                                int64_t& tm, int64_t& tn) {
    const int64_t total = tiles_m * tiles_n;
    const int64_t per_xcd = (total + kXcds - 1) / kXcds;
    const int64_t logical = (bid % kXcds) * per_xcd + bid / kXcds;
    if (logical >= total) return false;
    const int64_t group = logical / (GM * tiles_n);
    const int64_t first_m = group * GM;
    const int64_t gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
    const int64_t in_group = logical - group * GM * tiles_n;
    tm = first_m + in_group % gsize;
    tn = in_group / gsize;
    return true;
}

}  // namespace mpg
