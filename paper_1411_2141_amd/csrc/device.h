// Device-side data layout shared by the kernels and the context code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mr {

constexpr int kBlockMax = 128;     // largest dense diagonal block of the solve
constexpr int kSolveThreads = 256;
constexpr int kTile = 16;          // warp tiles are kTile x kTile pixels
constexpr int kNodeChunk = 256;    // nodes per sample work item

// Non-finite flag bits.
constexpr unsigned kFlagNonFiniteNode = 1u;
constexpr unsigned kFlagNonFinitePixel = 2u;

struct DevPair {
  int32_t height, width;
  int64_t pix_off;        // offset of the pair's images in the packed pixel arrays
  int32_t node_off, n;    // nodes [node_off, node_off + n) of the packed node arrays
  int32_t tri_off, nt;
  int32_t tile_off, n_tiles;   // warp tiles [tile_off, tile_off + n_tiles)
  int32_t tiles_x, pad0;
};

struct DevBlock {
  int32_t r0, r1;         // global rows of the packed permuted system
  int32_t fgroup, bgroup; // lanes per row of the off-block dot products
  int64_t doff;           // offset of the packed dense inverse
};

// Work item of the node-parallel kernels: nodes [begin, end) of pair `pair`.
struct NodeItem {
  int32_t pair, begin, end, pad;
};

// Work item of the pixel-parallel kernels: one kTile x kTile tile.
struct TileItem {
  int32_t pair, y0, x0, pad;
};

}  // namespace mr
