// Device-side data layout shared by the kernels and the context code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mr {

constexpr int kBlockMax = 96;      // largest dense diagonal block of the solve
constexpr int kSolveLdsBudget = 64 * 1024 - 512;  // dynamic LDS per solve workgroup (static use < 512 B)
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
  int32_t active;              // 0: the pair is retired (its work items return at once)
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
  int32_t active;         // the block's pair is active (else its items return at once)
};

// LDS bytes a forward work item of block size b with kn panel rows needs,
// and a backward work item with chunks of rs panel rows, for workgroups of nt
// threads (the factor entries are read from global memory, only vectors and
// partial sums are held); the launch of a level uses the maximum over its
// items.
inline int64_t solve_fwd_lds_bytes(int b, int kn, int nt) {
  (void)kn;
  return 16 * (2 * (int64_t)b + nt);
}
inline int64_t solve_bwd_lds_bytes(int b, int rs, int nt) {
  return 16 * ((int64_t)rs + nt + b);
}

// Apex of the block tree (all pairs share one numbering of apex positions).
// Forward work item: rows [a0, a1) of one apex block (consecutive, so their
// rows of X follow each other from xoff0 on, row r holding columns c0 .. r)
// against the columns [k0, k1) of one segment of the block's column range;
// the partial sums of row r go to slot part + (r - a0).
struct ApexFwdItem {
  int32_t a0, a1, k0, k1, c0, part;
  int32_t pair, active;         // the item's pair and whether it is active
  int64_t xoff0;
};
// Backward work item: rows [a0, a1) of one apex block ending at e; the path
// list is rows [a0, e) followed by the ancestor ranges rng[rng_off ..
// rng_off + n_rng), len entries in all; row r's column of X covers list
// positions r - a0 .. len - 1 and the columns follow each other from xoff0 on.
struct ApexBwdItem {
  int32_t a0, a1, e, rng_off, n_rng, len;
  int32_t pair, active;         // the item's pair and whether it is active
  int64_t xoff0;
};
// Per apex position: its forward partial slots part + q * stride, q < nseg.
struct ApexRow {
  int32_t part, stride, nseg, row;
};

constexpr int kApexSeg = 1024;        // columns per forward segment (16 KB of LDS)
constexpr int kApexPath = 2048;       // longest backward path (32 KB of LDS)
constexpr int kApexRowsPerItem = 8;   // rows per apex work item (two per wavefront)
constexpr int kApexMaxRanges = 256;   // ancestor ranges of one apex block (at most one per level)

// Right-hand side assembly folded into the first forward level: b for the
// rows of the level's (leaf) blocks is formed by their own workgroups, the
// workgroups after the block items form b for the other solve rows (`rows`,
// NT per workgroup), and, when finish_msd is set, the workgroups after those
// finish the MSD of `partials`.  Node data in solve order: u and h are
// indexed by solve row, the operator's columns too.
struct AssembleArgs {
  const int32_t *mptr;
  const uint32_t *ment;
  const float *minv;
  const float2 *h;
  const double2 *u;
  const int32_t *rows;          // solve rows outside the first level
  int32_t n_rows;
  int32_t n_pairs;
  double tau;
  const DevPair *pairs;
  const double *partials;
  double *finish_msd;
  const int32_t *active;        // per-pair activity, [n_pairs] = any pair retired (or null)
};

// Per-node record of the explicit variant, written by its smoothing launch
// and gathered (one 32-byte load per triangle corner) by its update launch:
// the deformed position V + u, the template sample t and r = t - rho.
struct __align__(32) NodeRec {
  double px, py, t, r;
};

// Work item of the node-parallel kernels: nodes [begin, end) of pair `pair`
// (active: the pair is not retired).
struct NodeItem {
  int32_t pair, begin, end, active;
};

// Work item of the batched prefilter: 64 consecutive rows (row pass) or
// columns (column pass) of pair `pair`, from `first` on; tab_w / tab_h are the
// offsets of the Thomas tables of the pair's width and height.
struct PrefItem {
  int32_t pair, first, tab_w, tab_h;
};

// Work item of the pixel-parallel kernels: one kTile x kTile tile of pair
// `pair` (whose image size and pixel offset it repeats).  The
// tile's distinct triangles (those of T6 over its pixels inside the image,
// ascending, pair-local ids) are tile_tri[ent_off .. ent_off + n_ent), and
// tile_loc[tile * kTile^2 + pixel] is each pixel's position in that list
// (pixels row by row; 0 outside the image).
struct TileItem {
  int32_t pair, y0, x0, active;
  int32_t ent_off, n_ent;
  int32_t height, width;  // the pair's image
  int64_t pix_off;
};

}  // namespace mr
