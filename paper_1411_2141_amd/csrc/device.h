// Device-side data layout shared by the kernels and the context code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mr {

constexpr int kBlockMax = 96;      // largest dense diagonal block of the solve
constexpr int kSolveLdsBudget = 64 * 1024 - 512;  // dynamic LDS per solve workgroup (static use < 512 B)
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
  int32_t tiles_x;
  int32_t item_off, n_items;   // node work items [item_off, item_off + n_items)
  int32_t pad0;
};

struct DevBlock {
  int32_t r0, r1;         // global rows of the packed permuted system
  int32_t m, fgroup;      // rows below the block; lanes per row of the forward gathers
  int64_t doff;           // offset of the packed dense inverse
  int64_t poff;           // offset of the dense row-major panel (m x b)
  int64_t boff;           // offset of the below-rows list == update-buffer offset
  int32_t nslice, rslice; // forward: nslice workgroups of rslice panel rows each
  int32_t bslice;         // backward: workgroups per block (each walks its rows in
                          // LDS chunks of rslice)
  int32_t part_off;       // backward partial sums: [bslice][b] double2 from here
  int32_t cnt_idx;        // backward arrival counter of the block
  int32_t pad;
};

// LDS bytes a forward work item of block size b with kn panel rows needs,
// and a backward work item with panel chunks of rs rows, for workgroups of
// nt threads; the launch of a level uses the maximum over its items.
inline int64_t solve_fwd_lds_bytes(int b, int kn, int nt) {
  const int64_t nd = (int64_t)b * (b + 1) / 2;
  return 8 * ((nd + (int64_t)kn * b + 1) / 2 * 2) + 16 * (2 * (int64_t)b + nt);
}
inline int64_t solve_bwd_lds_bytes(int b, int rs, int nt) {
  const int64_t nd = (int64_t)b * (b + 1) / 2;
  return 8 * (((int64_t)rs * b + 1) / 2 * 2) + 16 * ((int64_t)rs + nt + b) + 8 * nd;
}

// Apex (dense top of the block tree) of one pair.
struct ApexDesc {
  int32_t n;              // apex rows
  int32_t pad;
  int64_t rows_off;       // offset into the apex row list, contribution CSR and t/y buffers
  int64_t inv_off;        // offset of the packed inverse triangles
};

constexpr int kApexRowsPerGroup = 4;   // one wavefront per apex row / column

// Work item of the node-parallel kernels: nodes [begin, end) of pair `pair`.
struct NodeItem {
  int32_t pair, begin, end, pad;
};

// Work item of the pixel-parallel kernels: one kTile x kTile tile.
struct TileItem {
  int32_t pair, y0, x0, pad;
};

}  // namespace mr
