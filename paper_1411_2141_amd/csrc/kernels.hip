// HIP kernels of the registration hot path for gfx950 (CDNA4, wave64).
//
// Per iteration (Algorithm 1, semi-implicit form):
//   k_sample    node-parallel: template B-spline value and gradient at the
//               displaced node (eq. 3), residual against the reference sample
//               (eq. 4), force density h = r g (eq. 6)
//   k_assemble  node-parallel gather over the mass-matrix row: the
//               area-weighted triangle-to-node average of eq. 10 applied to the
//               P1 load, then b = u - tau f (eq. 5), written in solve order
//   k_solve_fwd / k_solve_bwd
//               block-level-scheduled FP64 triangular solves with the Cholesky
//               factor of I + tau alpha K (eq. 7-8 made implicit, solved directly)
//   warp tiles  pixel-tile-parallel: the affine displacement map of each
//               triangle of a tile (once per triangle, into LDS), the template
//               sample at each displaced pixel centre, squared error,
//               deterministic FP64 reduction to the MSD; run in the next
//               iteration's sample launch (both read the same u), the final sum
//               in its assemble launch
// All node-, tile- and block-parallel launches cover every pair of a batch
// through work lists, so one launch per kernel family advances all pairs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>

#include "device.h"
#include "kernels.h"
#include "launch.h"
#include "spline.h"

namespace mr {

// ---------------------------------------------------------------------------
// Pre-computation kernels (run once per pair, and for the template adjoint)
// ---------------------------------------------------------------------------

// Solve B c = s along each row (thread per row) with the Thomas algorithm;
// tab[k] = (cp_k, 1 / pivot_k) depends only on the row length.  Loads are
// issued U steps ahead of the recurrence.
template <typename Tin>
__global__ void k_prefilter_rows(const Tin *__restrict__ src, double *__restrict__ dst, int H,
                                 int W, const double2 *__restrict__ tab) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= H) return;
  const Tin *s = src + (size_t)r * W;
  double *d = dst + (size_t)r * W;
  if (W == 1) {
    d[0] = (double)s[0];
    return;
  }
  const double off = 1.0 / 6.0;
  constexpr int U = 8;
  double prev = 0.0;
  for (int k0 = 0; k0 < W; k0 += U) {
    double sv[U], mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      sv[u] = k < W ? (double)s[k] : 0.0;
      mv[u] = k < W ? tab[k].y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < W) {
        prev = (sv[u] - off * prev) * mv[u];
        d[k0 + u] = prev;
      }
  }
  for (int k1 = W - 2; k1 >= 0; k1 -= U) {
    double yv[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k1 - u;
      yv[u] = k >= 0 ? d[k] : 0.0;
      cv[u] = k >= 0 ? tab[k].x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k1 - u >= 0) {
        prev = yv[u] - cv[u] * prev;
        d[k1 - u] = prev;
      }
  }
}

// Column pass (thread per column, coalesced across threads), in place on
// `tmp`, writing the FP32 coefficients.
__global__ void k_prefilter_cols(double *__restrict__ tmp, float *__restrict__ out, int H, int W,
                                 const double2 *__restrict__ tab) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= W) return;
  double *d = tmp + col;
  if (H == 1) {
    out[col] = (float)d[0];
    return;
  }
  const double off = 1.0 / 6.0;
  constexpr int U = 8;
  double prev = 0.0;
  for (int k0 = 0; k0 < H; k0 += U) {
    double sv[U], mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      sv[u] = k < H ? d[(size_t)k * W] : 0.0;
      mv[u] = k < H ? tab[k].y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < H) {
        prev = (sv[u] - off * prev) * mv[u];
        d[(size_t)(k0 + u) * W] = prev;
      }
  }
  out[(size_t)(H - 1) * W + col] = (float)prev;
  for (int k1 = H - 2; k1 >= 0; k1 -= U) {
    double yv[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k1 - u;
      yv[u] = k >= 0 ? d[(size_t)k * W] : 0.0;
      cv[u] = k >= 0 ? tab[k].x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k1 - u >= 0) {
        prev = yv[u] - cv[u] * prev;
        out[(size_t)(k1 - u) * W + col] = (float)prev;
      }
  }
}

// The two passes for every pair of a context at once (work items of 64 rows
// or columns of one pair); FP64 in, the row pass may run in place
// (src == tmp: each batch of loads is issued before its writes, later
// batches read only positions not yet written), FP32 coefficients out.
__global__ __launch_bounds__(64) void k_prefilter_rows_all(const PrefItem *__restrict__ items,
                                                           const DevPair *__restrict__ pairs,
                                                           const double *src, double *tmp,
                                                           const double2 *__restrict__ tab) {
  const PrefItem it = items[blockIdx.x];
  const DevPair P = pairs[it.pair];
  const int r = it.first + (int)threadIdx.x;
  if (r >= P.height) return;
  const int W = P.width;
  const double *s = src + P.pix_off + (size_t)r * W;
  double *d = tmp + P.pix_off + (size_t)r * W;
  const double2 *tw = tab + it.tab_w;
  if (W == 1) {
    d[0] = s[0];
    return;
  }
  const double off = 1.0 / 6.0;
  constexpr int U = 8;
  double prev = 0.0;
  for (int k0 = 0; k0 < W; k0 += U) {
    double sv[U], mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      sv[u] = k < W ? s[k] : 0.0;
      mv[u] = k < W ? tw[k].y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < W) {
        prev = (sv[u] - off * prev) * mv[u];
        d[k0 + u] = prev;
      }
  }
  for (int k1 = W - 2; k1 >= 0; k1 -= U) {
    double yv[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k1 - u;
      yv[u] = k >= 0 ? d[k] : 0.0;
      cv[u] = k >= 0 ? tw[k].x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k1 - u >= 0) {
        prev = yv[u] - cv[u] * prev;
        d[k1 - u] = prev;
      }
  }
}

__global__ __launch_bounds__(64) void k_prefilter_cols_all(const PrefItem *__restrict__ items,
                                                           const DevPair *__restrict__ pairs,
                                                           double *tmp, float *__restrict__ out,
                                                           const double2 *__restrict__ tab) {
  const PrefItem it = items[blockIdx.x];
  const DevPair P = pairs[it.pair];
  const int col = it.first + (int)threadIdx.x;
  if (col >= P.width) return;
  const int H = P.height, W = P.width;
  double *d = tmp + P.pix_off + col;
  float *o = out + P.pix_off + col;
  const double2 *th = tab + it.tab_h;
  if (H == 1) {
    o[0] = (float)d[0];
    return;
  }
  const double off = 1.0 / 6.0;
  constexpr int U = 8;
  double prev = 0.0;
  for (int k0 = 0; k0 < H; k0 += U) {
    double sv[U], mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      sv[u] = k < H ? d[(size_t)k * W] : 0.0;
      mv[u] = k < H ? th[k].y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < H) {
        prev = (sv[u] - off * prev) * mv[u];
        d[(size_t)(k0 + u) * W] = prev;
      }
  }
  o[(size_t)(H - 1) * W] = (float)prev;
  for (int k1 = H - 2; k1 >= 0; k1 -= U) {
    double yv[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k1 - u;
      yv[u] = k >= 0 ? d[(size_t)k * W] : 0.0;
      cv[u] = k >= 0 ? th[k].x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k1 - u >= 0) {
        prev = yv[u] - cv[u] * prev;
        o[(size_t)(k1 - u) * W] = (float)prev;
      }
  }
}

// Reference spline at the undisplaced nodes: rho_i = s_Re(V_i - 1/2).
__global__ __launch_bounds__(256) void k_sample_rho(const NodeItem *__restrict__ items,
                                                    const DevPair *__restrict__ pairs,
                                                    const int2 *__restrict__ xy,
                                                    const float *__restrict__ coef_re,
                                                    float *__restrict__ rho) {
  const NodeItem it = items[blockIdx.x];
  const int i = it.begin + threadIdx.x;
  if (i >= it.end) return;
  const DevPair P = pairs[it.pair];
  const int2 v = xy[i];
  rho[i] = spline_value(coef_re + P.pix_off, P.height, P.width, v.x - 1, 0.5f, v.y - 1, 0.5f);
}

// ---------------------------------------------------------------------------
// Hot path
// ---------------------------------------------------------------------------

// Work item of block b (0 <= b < G) of a launch range whose blocks take one
// item each: workgroups go to the 8 XCDs round-robin by block id, so blocks
// b, b + 8, b + 16, ... share an XCD; they take one contiguous run of items
// (neighbouring items touch the same cache lines, which then stay in that
// XCD's L2).  A bijection for any G.
__device__ __forceinline__ int xcd_item(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Second pass of the MSD: workgroup `group` finishes pairs 4 group .. 4 group + 3,
// one wavefront per pair summing that pair's tile partials in a fixed order
// (deterministic) and dividing by its pixel count.
__device__ __forceinline__ void msd_finish_group(const DevPair *__restrict__ pairs, int n_pairs,
                                                 const double *__restrict__ partials,
                                                 double *__restrict__ msd, int group) {
  const int lane = threadIdx.x & 63;
  const int p = group * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  if (p >= n_pairs) return;
  const DevPair Q = pairs[p];
  if (!Q.active) return;                      // retired pair: its MSD is left as it is
  const double s = wave_sum(lane_strided_sum(partials + Q.tile_off, Q.n_tiles, lane));
  if (lane == 0) msd[p] = s / ((double)Q.height * (double)Q.width);
}

// FP32 cubic B-spline weights of fraction t in [0, 1); w[2] is formed from the
// other three so the four sum to 1 up to the last rounding (no systematic
// scaling of the sample, which would bias a mean of squared differences).
__device__ __forceinline__ void bs_weights_unit(float t, float w[4]) {
  const float s = 1.0f - t, t2 = t * t, s2 = s * s;
  w[0] = s2 * (s * (1.0f / 6.0f));
  w[3] = t2 * (t * (1.0f / 6.0f));
  w[1] = fmaf(t2, fmaf(t, 0.5f, -1.0f), 2.0f / 3.0f);
  w[2] = ((1.0f - w[0]) - w[1]) - w[3];
}

// Element at byte offset `off` (unsigned 32-bit, cannot overflow) of an array
// at a workgroup-uniform base: the load takes the scalar base plus a 32-bit
// vector offset, with no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T load_at(const T *__restrict__ base, unsigned off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// The records of NT consecutive tiles from tile0 (a tile past the end or of a
// retired pair is off and has no entries); the group's triangle entries are
// numbered tile after tile, tile q's from base[q] on, total in all.
template <int NT>
struct WarpGroup {
  TileItem it[NT];
  int tl[NT], base[NT], total;
  bool on[NT];
};

template <int NT>
__device__ __forceinline__ void warp_group(WarpGroup<NT> &g, int tile0, int n_tiles,
                                           const TileItem *__restrict__ tiles) {
  g.total = 0;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const bool valid = tile0 + q < n_tiles;
    g.tl[q] = valid ? tile0 + q : tile0;
    g.it[q] = tiles[g.tl[q]];
  }
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const bool valid = tile0 + q < n_tiles;
    g.on[q] = valid & (g.it[q].active != 0);
    g.base[q] = g.total;
    g.total += g.on[q] ? g.it[q].n_ent : 0;
  }
}

// The thread's pixel (rx, ry) of each tile: its triangle's slot in the group's
// entry numbering, its offset in the pair's image, whether it lies inside the
// image and its reference sample.  None of it depends on the maps.
template <int NT>
struct WarpPixels {
  int slot[NT];
  float rv[NT];
  unsigned po[NT];
  bool in[NT];
};

template <int NT>
__device__ __forceinline__ void warp_pixels(WarpPixels<NT> &p, const WarpGroup<NT> &g, int tid,
                                            int rx, int ry, const uint8_t *__restrict__ tile_loc,
                                            const float *__restrict__ re) {
  constexpr int kPix = kTile * kTile;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int i = g.it[q].y0 + ry, j = g.it[q].x0 + rx;
    p.in[q] = g.on[q] && i < g.it[q].height && j < g.it[q].width;
    p.po[q] = __umul24((unsigned)min(i, g.it[q].height - 1), (unsigned)g.it[q].width) +
              (unsigned)min(j, g.it[q].width - 1);
    p.slot[q] = g.base[q] + (int)tile_loc[(size_t)g.tl[q] * kPix + tid];
    p.rv[q] = load_at(re + g.it[q].pix_off, p.po[q] << 2);
  }
}

// Stage 1: the maps of the group's entries [r0, r1) (at most kTile^2), entry e
// by thread e - r0, into map[.][e - r0].
template <int NT>
__device__ __forceinline__ void warp_maps(const WarpGroup<NT> &g, int r0, int r1, int tid,
                                          const double2 *__restrict__ u,
                                          const int4 *__restrict__ tile_nodes,
                                          const int2 *__restrict__ tile_pbc, unsigned *flags,
                                          double2 (*map)[kTile * kTile]) {
  const int e = r0 + tid;
  if (e >= r1) return;
  // the entry's tile: the last with base <= e (off tiles have no entries)
  int x0 = g.it[0].x0, y0 = g.it[0].y0, k = g.it[0].ent_off + e;
#pragma unroll
  for (int q = 1; q < NT; ++q)
    if (e >= g.base[q]) {
      x0 = g.it[q].x0;
      y0 = g.it[q].y0;
      k = g.it[q].ent_off - g.base[q] + e;
    }
  const int4 nd = tile_nodes[k];               // corner nodes, packed first corner
  const int2 pbc = tile_pbc[k];                // packed other corners
  double2 ua = load_at(u, (unsigned)nd.x << 4);
  const double2 ub = load_at(u, (unsigned)nd.y << 4);
  const double2 uc = load_at(u, (unsigned)nd.z << 4);
  // corners relative to the tile origin (exact)
  const int ax = (nd.w & 0xffff) - x0, ay = (int)((unsigned)nd.w >> 16) - y0;
  const double e1x = (double)((pbc.x & 0xffff) - x0 - ax);
  const double e1y = (double)((int)((unsigned)pbc.x >> 16) - y0 - ay);
  const double e2x = (double)((pbc.y & 0xffff) - x0 - ax);
  const double e2y = (double)((int)((unsigned)pbc.y >> 16) - y0 - ay);
  const double det = e1x * e2y - e1y * e2x;    // twice the area: exact, positive
  // 1 / det: the FP32 estimate and two Newton steps
  double inv = (double)__builtin_amdgcn_rcpf((float)det);
  inv = fma(inv, fma(-det, inv, 1.0), inv);
  inv = fma(inv, fma(-det, inv, 1.0), inv);
  const bool ok = fabs(ua.x) < 1.0e6 && fabs(ua.y) < 1.0e6 && fabs(ub.x) < 1.0e6 &&
                  fabs(ub.y) < 1.0e6 && fabs(uc.x) < 1.0e6 && fabs(uc.y) < 1.0e6;
  // formed unconditionally (a branch around them would sink the corner
  // coordinate load behind the displacement loads)
  const double d1x = ub.x - ua.x, d1y = ub.y - ua.y, d2x = uc.x - ua.x, d2y = uc.y - ua.y;
  double gxx = (d1x * e2y - d2x * e1y) * inv;
  double gxy = (d2x * e1x - d1x * e2x) * inv;
  double gyx = (d1y * e2y - d2y * e1y) * inv;
  double gyy = (d2y * e1x - d1y * e2x) * inv;
  if (!ok) {
    gxx = gxy = gyx = gyy = 0.0;
    ua = make_double2(0.0, 0.0);
    atomicOr(flags, kFlagNonFinitePixel);
  }
  // displacement at the origin pixel's centre, (1/2, 1/2) in the tile frame
  const double ox = 0.5 - (double)ax, oy = 0.5 - (double)ay;
  map[0][tid] = make_double2(ua.x + gxx * ox + gxy * oy, ua.y + gyx * ox + gyy * oy);
  map[1][tid] = make_double2(1.0 + gxx, gxy);
  map[2][tid] = make_double2(gyx, 1.0 + gyy);
}

// Stage 2, first half: the pixels whose slots lie in the round [r0, r1)
// evaluate their map and issue their coefficient loads (both tiles' together).
template <int NT>
struct WarpTaps {
  float tap[NT][4][4];
  float fx[NT], fy[NT];
  bool act[NT];
};

template <int NT>
__device__ __forceinline__ void warp_taps(WarpTaps<NT> &t, const WarpGroup<NT> &g,
                                          const WarpPixels<NT> &p, int r0, int r1, double rxd,
                                          double ryd, const double2 (*map)[kTile * kTile],
                                          const float *__restrict__ coef) {
  int qx[NT], qy[NT];
  bool inside = true;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    t.act[q] = p.slot[q] >= r0 && p.slot[q] < r1;
    const int sl = t.act[q] ? p.slot[q] - r0 : 0;
    const double2 c = map[0][sl], gx = map[1][sl], gy = map[2][sl];
    const double vx = fma(gx.x, rxd, fma(gx.y, ryd, c.x));
    const double vy = fma(gy.x, rxd, fma(gy.y, ryd, c.y));
    const double flx = floor(vx), fly = floor(vy);
    qx[q] = g.it[q].x0 + (int)flx;
    qy[q] = g.it[q].y0 + (int)fly;
    t.fx[q] = (float)(vx - flx);
    t.fy[q] = (float)(vy - fly);
    // positions outside the image or the round take the window of cell
    // (1, 1) (inside the image when both sides are at least 4)
    if (!(p.in[q] && t.act[q])) {
      qx[q] = qy[q] = 1;
      t.fx[q] = t.fy[q] = 0.0f;
    }
    inside = inside && taps_inside(g.it[q].height, g.it[q].width, qx[q], qy[q]);
  }
  if (__all(inside)) {
#pragma unroll
    for (int q = 0; q < NT; ++q)
      load_taps_inside(coef + g.it[q].pix_off, g.it[q].width, qx[q], qy[q], t.tap[q]);
  } else {
#pragma unroll
    for (int q = 0; q < NT; ++q)
      load_taps(coef + g.it[q].pix_off, g.it[q].height, g.it[q].width, qx[q], qy[q], t.tap[q]);
  }
}

// Stage 2, second half: the samples of the round's pixels, the warped image
// and the squared differences (each pixel is in exactly one round).
template <int NT>
__device__ __forceinline__ void warp_samples(const WarpTaps<NT> &t, const WarpGroup<NT> &g,
                                             const WarpPixels<NT> &p, float *__restrict__ warped,
                                             double (&sq)[NT]) {
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    float wx[4], wy[4];
    bs_weights_unit(t.fx[q], wx);
    bs_weights_unit(t.fy[q], wy);
    float w = 0.0f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float rs = t.tap[q][m][0] * wx[0] + t.tap[q][m][1] * wx[1] +
                       t.tap[q][m][2] * wx[2] + t.tap[q][m][3] * wx[3];
      w += wy[m] * rs;
    }
    if (t.act[q]) {
      if (warped && p.in[q]) (warped + g.it[q].pix_off)[p.po[q]] = w;
      const double d = (double)(w - p.rv[q]);
      sq[q] = p.in[q] ? d * d : 0.0;
    }
  }
}

// Warp + MSD of NT kTile x kTile pixel tiles, tile0 .. tile0 + NT - 1 (those
// below n_tiles), with a workgroup of kTile^2 threads, the thread taking the
// same pixel position in each tile.
//
// Every pixel of a triangle has the same affine displacement map (P1
// interpolation), so the work is split in two stages.  First each distinct
// triangle of a tile (the tile's list, built at init from T6: corner node ids
// in tile_nodes, in the node order of u, and packed corner coordinates) gets
// its map in the tile's frame, one thread per triangle, into LDS: for the
// pixel at tile position r = (rx, ry) the sampling position in spline
// coordinates is (x0, y0) + c + G' r, with G' = I + grad d and c the displaced
// position of the tile origin's pixel (FP64; the map is formed from the
// corners' exact integer coordinates and displacements).  Then each pixel
// reads its triangle's slot (a byte per pixel) and samples the template
// spline there (FP32 weights with the partition of unity kept and FP32 tap
// sums).  A triangle with a non-finite displacement, or one of 10^6 pixels or
// more, at a corner raises the flag and is warped with zero displacement.
// Windows wholly inside the image take four row loads per pixel; a wavefront
// with a lane whose window crosses the border folds its taps one by one.
// Each tile's FP64 sum of squared differences (a fixed order over the
// workgroup's threads) goes to partials[tile].  Offsets within a pair's image
// are 32-bit (fewer than 2^31 pixels).
template <int NT>
__device__ __forceinline__ void warp_tiles(int tile0, int n_tiles, const TileItem *__restrict__ tiles,
                                           const double2 *__restrict__ u,
                                           const int4 *__restrict__ tile_nodes,
                                           const int2 *__restrict__ tile_pbc,
                                           const uint8_t *__restrict__ tile_loc,
                                           const float *__restrict__ coef,
                                           const float *__restrict__ re,
                                           float *__restrict__ warped,
                                           double *__restrict__ partials, unsigned *flags) {
  constexpr int kPix = kTile * kTile;
  // maps of up to kPix triangles at a time: c, (G'xx, G'xy), (G'yx, G'yy)
  __shared__ double2 map[3][kPix];
  const int tid = (int)threadIdx.x;
  WarpGroup<NT> g;
  warp_group(g, tile0, n_tiles, tiles);
  // Tiles of retired pairs are not warped (the workgroup returns when all of
  // its tiles are retired).
  bool any = false;
#pragma unroll
  for (int q = 0; q < NT; ++q) any = any || g.on[q];
  if (!any) return;

  // The pixels' slots and reference samples do not depend on the maps:
  // their loads go out first.
  const int rx = tid % kTile, ry = tid / kTile;
  WarpPixels<NT> p;
  warp_pixels(p, g, tid, rx, ry, tile_loc, re);
  const double rxd = (double)rx, ryd = (double)ry;
  double sq[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) sq[q] = 0.0;

  // The tiles' triangles in rounds of up to kPix (one round unless two dense
  // tiles share the workgroup); each pixel is evaluated in its slot's round.
  for (int r0 = 0; r0 < g.total; r0 += kPix) {
    const int r1 = min(g.total, r0 + kPix);
    if (r0 > 0) __syncthreads();                  // the previous round's maps are read
    warp_maps(g, r0, r1, tid, u, tile_nodes, tile_pbc, flags, map);
    __syncthreads();
    WarpTaps<NT> t;
    warp_taps(t, g, p, r0, r1, rxd, ryd, map, coef);
    warp_samples(t, g, p, warped, sq);
  }

  // Tile sums in a fixed order: the threads' values through LDS (the maps'
  // storage), then one wavefront adds kPix / (64 / NT) of them per lane and
  // reduces within its 64 / NT lanes.
  __syncthreads();
  double *red = reinterpret_cast<double *>(&map[0][0]);
#pragma unroll
  for (int q = 0; q < NT; ++q) red[q * kPix + tid] = sq[q];
  __syncthreads();
  if (tid < 64) {
    constexpr int kLanes = 64 / NT;
    const int q = tid / kLanes, j = tid % kLanes;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPix / kLanes; ++k) s += red[q * kPix + j + k * kLanes];
#pragma unroll
    for (int off = kLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    bool onq = g.on[0];
    int tq = g.tl[0];
#pragma unroll
    for (int p2 = 1; p2 < NT; ++p2)
      if (q == p2) {
        onq = g.on[p2];
        tq = g.tl[p2];
      }
    if (j == 0 && onq) partials[tq] = s;
  }
}

// Node sampling of NT node items at once (the thread's node in each; a
// thread past an item's end re-reads its first node and writes nothing):
// r_i = s(V_i - 1/2 + u_i) - rho_i and h_i = r_i grad s, in FP32.  The NT
// nodes go through each step together so their dependent loads overlap.
template <int NT>
__device__ __forceinline__ void sample_nodes(const NodeItem (&it)[NT], const DevPair (&P)[NT],
                                             const double2 *__restrict__ u,
                                             const int2 *__restrict__ xy,
                                             const float *__restrict__ coef,
                                             const float *__restrict__ rho,
                                             float2 *__restrict__ h, unsigned *flags) {
  int i[NT];
  bool on[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    i[q] = it[q].begin + (int)threadIdx.x;
    on[q] = i[q] < it[q].end;
    if (!on[q]) i[q] = it[q].begin;
  }
  double2 ui[NT];
  int2 v[NT];
  float rh[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    ui[q] = u[i[q]];
    v[q] = xy[i[q]];
    rh[q] = rho[i[q]];
  }
  int cx[NT], cy[NT];
  float fx[NT], fy[NT];
  bool inside = true;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const bool okx = split_coord(v[q].x, ui[q].x - 0.5, cx[q], fx[q]);
    const bool ok = split_coord(v[q].y, ui[q].y - 0.5, cy[q], fy[q]) && okx;
    if (on[q] && !ok) atomicOr(flags, kFlagNonFiniteNode);
    inside = inside && taps_inside(P[q].height, P[q].width, cx[q], cy[q]);
  }
  float tap[NT][4][4];
  if (inside) {
#pragma unroll
    for (int q = 0; q < NT; ++q)
      load_taps_inside(coef + P[q].pix_off, P[q].width, cx[q], cy[q], tap[q]);
  } else {
#pragma unroll
    for (int q = 0; q < NT; ++q)
      load_taps(coef + P[q].pix_off, P[q].height, P[q].width, cx[q], cy[q], tap[q]);
  }
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    float val, gx, gy;
    spline_value_grad_taps(tap[q], fx[q], fy[q], val, gx, gy);
    const float r = val - rh[q];
    if (on[q]) h[i[q]] = make_float2(r * gx, r * gy);
  }
}

// Node sampling (one workgroup per node item) of the node displacements un
// with the node tables xy, rho and the output h, all in one node order (the
// iteration uses solve order).  When `n_tiles` > 0 the workgroups after the
// node items warp the pixel grid by u (natural node order, the same
// displacements) into the MSD partials (one tile each: this launch is short,
// and a workgroup's latency matters more than overlap), so the MSD of the
// previous iteration's result shares it.
__global__ __launch_bounds__(256) void k_sample(const NodeItem *__restrict__ items, int n_items,
                                                const DevPair *__restrict__ pairs,
                                                const double2 *__restrict__ un,
                                                const int2 *__restrict__ xy,
                                                const float *__restrict__ coef,
                                                const float *__restrict__ rho,
                                                float2 *__restrict__ h, unsigned *flags,
                                                const TileItem *__restrict__ tiles,
                                                const double2 *__restrict__ u,
                                                const int4 *__restrict__ tile_nodes,
                                                const int2 *__restrict__ tile_pbc,
                                                const uint8_t *__restrict__ tile_loc,
                                                const float *__restrict__ re,
                                                double *__restrict__ partials, int n_tiles) {
  if ((int)blockIdx.x >= n_items) {
    warp_tiles<1>(xcd_item((int)blockIdx.x - n_items, n_tiles), n_tiles, tiles, u, tile_nodes,
                  tile_pbc, tile_loc, coef, re, nullptr, partials, flags);
    return;
  }
  const NodeItem it[1] = {items[xcd_item((int)blockIdx.x, n_items)]};
  if (!it[0].active || it[0].begin + (int)threadIdx.x >= it[0].end) return;
  const DevPair P[1] = {pairs[it[0].pair]};
  sample_nodes<1>(it, P, un, xy, coef, rho, h, flags);
}

// Entry q of a one-word force-operator row of solve row k: its column (k plus
// the signed 16-bit offset in the high half) and its integer numerator.
__device__ __forceinline__ int ment_col(uint32_t e, int k) { return k + ((int32_t)e >> 16); }
__device__ __forceinline__ float ment_num(uint32_t e) { return (float)(e & 0xffffu); }

// b for solve row k: u_k - tau f_k, f_k = (sum_q a_q h(col_q)) / (4 * 6 m_k)
// over the force operator row k (integer numerators a_q; FP32 sum in row
// order), loads issued in batches of U.  Node data in solve order (u, h and
// the operator's columns).  Rows flagged by bit 31 of mptr hold two words per
// entry (column, FP32 numerator).
__device__ __forceinline__ double2 assemble_b(int k, const int32_t *__restrict__ mptr,
                                              const uint32_t *__restrict__ ment,
                                              const float *__restrict__ minv,
                                              const float2 *__restrict__ h,
                                              const double2 *__restrict__ u, double tau) {
  const double2 ui = u[k];
  const int32_t p0 = mptr[k];
  const int q0 = p0 & 0x7fffffff, q1 = mptr[k + 1] & 0x7fffffff;
  const float inv = minv[k];
  float fx = 0.0f, fy = 0.0f;
  constexpr int U = 8;
  if (p0 >= 0) {
    for (int q = q0; q < q1; q += U) {
      uint32_t e[U];
#pragma unroll
      for (int j = 0; j < U; ++j) e[j] = q + j < q1 ? ment[q + j] : 0u;
      float2 hv[U];
#pragma unroll
      for (int j = 0; j < U; ++j) hv[j] = h[ment_col(e[j], k)];
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (q + j < q1) {
          fx += ment_num(e[j]) * hv[j].x;
          fy += ment_num(e[j]) * hv[j].y;
        }
    }
  } else {
    for (int q = q0; q < q1; q += 2) {
      const int c = (int)ment[q];
      const float a = __uint_as_float(ment[q + 1]);
      const float2 hv = h[c];
      fx += a * hv.x;
      fy += a * hv.y;
    }
  }
  return make_double2(ui.x - tau * (double)(fx * inv), ui.y - tau * (double)(fy * inv));
}

// Whether solve row `row` belongs to an active pair.  active[n_pairs] is
// nonzero once some pair is retired (until then no lookup is made); the pair
// is found by bisection over the pairs' first rows (rows are packed pair by
// pair in solve order).
__device__ __forceinline__ bool row_active(const DevPair *__restrict__ pairs, int n_pairs,
                                           const int32_t *__restrict__ active, int row) {
  if (!active || active[n_pairs] == 0) return true;
  int lo = 0, hi = n_pairs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pairs[mid].node_off <= row) lo = mid;
    else hi = mid - 1;
  }
  return active[lo] != 0;
}

// Workgroup g of those after a fused first level's block items: the first
// ceil(n_rows / blockDim) assemble b of the other solve rows (b stays in x,
// read by later levels), the rest finish the MSD.  Rows of retired pairs keep
// their x (the displacement).
__device__ __forceinline__ void fused_tail(const AssembleArgs &A, double2 *x, int g) {
  const int nt = (int)blockDim.x;
  const int row_groups = (A.n_rows + nt - 1) / nt;
  if (g < row_groups) {
    const int k = g * nt + (int)threadIdx.x;
    if (k < A.n_rows) {
      const int row = A.rows[k];
      if (row_active(A.pairs, A.n_pairs, A.active, row))
        x[row] = assemble_b(row, A.mptr, A.ment, A.minv, A.h, A.u, A.tau);
    }
  } else {
    msd_finish_group(A.pairs, A.n_pairs, A.partials, A.finish_msd, g - row_groups);
  }
}

// Force assembly (a thread per solve row: at 38 VGPRs the workgroups fill
// the CUs, which beat two rows per thread with their gathers interleaved at
// 76), b written in solve order; u and h in solve order too, and x may be u
// itself (each thread reads its row of u before writing it).  When `finish_msd` is given, the workgroups after
// the node range finish the MSD of the partials written by the preceding
// sample launch.
__global__ __launch_bounds__(256) void k_assemble(int n, const int32_t *__restrict__ mptr,
                                                  const uint32_t *__restrict__ ment,
                                                  const float *__restrict__ minv,
                                                  const float2 *__restrict__ h,
                                                  const double2 *u, double2 *x, double tau,
                                                  const DevPair *__restrict__ pairs, int n_pairs,
                                                  const double *__restrict__ partials,
                                                  double *__restrict__ finish_msd,
                                                  const int32_t *__restrict__ active) {
  const int node_groups = (n + 255) / 256;
  if ((int)blockIdx.x >= node_groups) {
    msd_finish_group(pairs, n_pairs, partials, finish_msd, (int)blockIdx.x - node_groups);
    return;
  }
  const int k = (int)blockIdx.x * 256 + (int)threadIdx.x;
  // rows of retired pairs keep their x (the displacement)
  if (k < n && row_active(pairs, n_pairs, active, k))
    x[k] = assemble_b(k, mptr, ment, minv, h, u, tau);
}

// Smallest power of two >= b (b <= kBlockMax).
__device__ __forceinline__ int pow2_at_least(int b) {
  int p = 1;
  while (p < b) p <<= 1;
  return p;
}

// Sums red[o + q * stride] for q < nparts in order (deterministic combine).
__device__ __forceinline__ double2 combine_parts(const double2 *red, int o, int stride,
                                                 int nparts) {
  double sx = 0.0, sy = 0.0;
  for (int q = 0; q < nparts; ++q) {
    sx += red[o + q * stride].x;
    sy += red[o + q * stride].y;
  }
  return make_double2(sx, sy);
}

// Forward solve, one level of the block tree (supernodal, push form).  Work
// item = (block, slice).  Every slice of a block computes
//   t = b_rows - (update entries that descendant blocks wrote for these rows)
//   y = D^-1 t              (dense inverse, column-major packed)
// and then its slice of the block's own update entries
//   upd[k] = sum_j P[k][j] y_j   for panel rows k of the slice (P = L(below, block),
//                                 read from its column-major copy).
// Slice 0 also writes y to ybuf (b stays in x for the other slices).  D and P
// are read straight from global memory in coalesced order, U loads per thread
// in flight (each entry is used once, so nothing is staged); only t, y and
// the partial sums live in LDS, which keeps the workgroup's LDS independent
// of the block size.  Each phase spreads its sums over all threads and
// combines the partial sums in a fixed order (deterministic).
// With FUSED (first level only, no contributions) the workgroup forms b of
// its rows itself, and the workgroups after the `count` block items assemble
// the other rows and finish the MSD (AssembleArgs).
template <int NT, bool FUSED>
__global__ __launch_bounds__(NT) void k_solve_fwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
    const double *__restrict__ dcol, const double *__restrict__ pcol, double2 *x, double2 *ybuf,
    double2 *upd, AssembleArgs A) {
  extern __shared__ double2 sv[];           // t[b], y[b], red[NT]
  if (FUSED && (int)blockIdx.x >= count) {
    fused_tail(A, x, (int)blockIdx.x - count);
    return;
  }
  const int2 it = items[blockIdx.x];
  const DevBlock B = blocks[it.x];
  const int b = B.r1 - B.r0;
  if (b == 0 || !B.active) return;
  const int tid = threadIdx.x;
  const int m = B.m;
  const int k0 = it.y * B.rslice;
  const int kn = max(0, min(B.rslice, m - k0));
  double2 *t = sv;
  double2 *yv = sv + b;
  double2 *red = sv + 2 * b;
  const int bp = pow2_at_least(b);
  const int np = NT / bp;          // threads per row
  const int r = tid & (bp - 1), part = tid / bp;
  constexpr int U = 8;
  // D(r, j), j <= r, at doff + j b - j (j - 1) / 2 + (r - j); the first batch
  // is in flight during phase 1
  auto dload = [&](int j) {
    return (r < b && j <= r)
               ? dcol[B.doff + (int64_t)j * b - (int64_t)j * (j - 1) / 2 + (r - j)]
               : 0.0;
  };
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = dload(part + u * np);
  // phase 1: gathers of the contributions, all loads of a thread in flight
  if (FUSED) {
    if (part == 0 && r < b) {
      const int row = B.r0 + r;
      t[r] = assemble_b(row, A.mptr, A.ment, A.minv, A.h, A.u, A.tau);
    }
  } else {
    double ax = 0.0, ay = 0.0;
    if (r < b) {
      const int row = B.r0 + r;
      const int64_t q1 = cptr[row + 1];
      for (int64_t q = cptr[row] + part; q < q1; q += (int64_t)np * U) {
        int idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t qq = q + (int64_t)u * np;
          idx[u] = qq < q1 ? cidx[qq] : -1;
        }
        double2 cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cv[u] = idx[u] >= 0 ? upd[idx[u]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ax += cv[u].x;
          ay += cv[u].y;
        }
      }
    }
    red[tid] = make_double2(ax, ay);
    __syncthreads();
    if (part == 0 && r < b) {
      const double2 c = combine_parts(red, r, bp, np);
      const double2 bb = x[B.r0 + r];
      t[r] = make_double2(bb.x - c.x, bb.y - c.y);
    }
  }
  __syncthreads();
  // phase 2: y_r = sum_{j <= r} D(r, j) t_j, j = part, part + np, ...
  {
    double ax = 0.0, ay = 0.0;
    for (int j0 = part; j0 < b; j0 += U * np) {
      if (j0 != part) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = dload(j0 + u * np);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * np;
        if (r < b && j <= r) {
          const double2 tj = t[j];
          ax += v[u] * tj.x;
          ay += v[u] * tj.y;
        }
      }
    }
    red[tid] = make_double2(ax, ay);
  }
  __syncthreads();
  if (part == 0 && r < b) {
    const double2 y = combine_parts(red, r, bp, np);
    yv[r] = y;
    if (it.y == 0) ybuf[B.r0 + r] = y;
  }
  __syncthreads();
  // phase 3: the slice's update entries, kParts partial sums per panel row
  // (one pass over a 64-row slice); P(k0 + kk, j) at poff + j m + k0 + kk
  constexpr int kParts = NT / 64;
  constexpr int kRows = NT / kParts;
  for (int base = 0; base < kn; base += kRows) {
    const int kk = base + tid % kRows;
    const int pp = tid / kRows;
    const bool on = kk < kn;
    double ax = 0.0, ay = 0.0;
    for (int j0 = pp; j0 < b; j0 += U * kParts) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * kParts;
        v[u] = (on && j < b) ? pcol[B.poff + (int64_t)j * m + k0 + kk] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * kParts;
        if (on && j < b) {
          const double2 yj = yv[j];
          ax += v[u] * yj.x;
          ay += v[u] * yj.y;
        }
      }
    }
    red[tid] = make_double2(ax, ay);
    __syncthreads();
    if (pp == 0 && on) upd[B.boff + k0 + kk] = combine_parts(red, tid, kRows, kParts);
    __syncthreads();
  }
}

// Backward solve, one level of the block tree.  Work item = (block, slice);
// a block is split into B.bslice workgroups, each covering a contiguous run of
// panel rows that it walks in chunks of B.rslice rows (z of the chunk's rows
// gathered into LDS), forming the partial sums s_j = sum_k P[k][j] z(below_k).
// A block with one workgroup finishes at once; otherwise each workgroup
// writes its partials, and the last to arrive (device-scope counter) adds
// them in slice order.  The finishing workgroup forms t = y_block - s (y from
// ybuf) and z = D^-T t (row-major packed inverse), writes z in place and,
// when `out` is given, scatters it to natural order.  The finisher resets the
// counter.  P and D are read straight from global memory in coalesced order
// (each entry is used once), U loads per thread in flight.
template <int NT>
__global__ __launch_bounds__(NT) void k_solve_bwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items,
    const int32_t *__restrict__ below_idx, const double *__restrict__ drow,
    const double *__restrict__ prow, double2 *x, const double2 *__restrict__ ybuf,
    const int32_t *__restrict__ perm,
    double2 *__restrict__ out, double2 *partials, unsigned *counters) {
  extern __shared__ double2 sv[];           // zb[cap], red[NT], t[b]
  __shared__ int last;
  const int2 it = items[blockIdx.x];
  const DevBlock B = blocks[it.x];
  const int b = B.r1 - B.r0;
  if (b == 0 || !B.active) return;
  const int tid = threadIdx.x;
  const int rs = B.rslice;
  // panel rows [kb, ke) of this workgroup
  const int per = (B.m + B.bslice - 1) / B.bslice;
  const int kb = min(B.m, it.y * per), ke = min(B.m, kb + per);
  const int cap = min(rs, B.m);   // chunk of panel rows whose z is held in LDS
  double2 *zb = sv;
  double2 *red = zb + cap;
  double2 *t = red + NT;
  const int bp = pow2_at_least(b);
  const int np = NT / bp;
  const int j = tid & (bp - 1), g = tid / bp;
  constexpr int U = 8;
  double v[U];
  double ax = 0.0, ay = 0.0;
  for (int c0 = kb; c0 < ke; c0 += cap) {
    const int kn = min(cap, ke - c0);
    // P(c0 + k, j) at poff + (c0 + k) b + j; the first batch is in flight
    // during the z gather
    auto pload = [&](int k) {
      return (j < b && k < kn) ? prow[B.poff + (int64_t)(c0 + k) * b + j] : 0.0;
    };
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pload(g + u * np);
    for (int k = tid; k < kn; k += NT) zb[k] = x[below_idx[B.boff + c0 + k]];
    __syncthreads();
    for (int q0 = g; q0 < kn; q0 += U * np) {
      if (q0 != g) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = pload(q0 + u * np);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = q0 + u * np;
        if (j < b && k < kn) {
          const double2 zk = zb[k];
          ax += v[u] * zk.x;
          ay += v[u] * zk.y;
        }
      }
    }
    __syncthreads();
  }
  red[tid] = make_double2(ax, ay);
  __syncthreads();
  double2 sum = make_double2(0.0, 0.0);
  if (g == 0 && j < b) sum = combine_parts(red, j, bp, np);
  if (B.bslice > 1) {
    if (g == 0 && j < b) partials[B.part_off + it.y * b + j] = sum;
    __threadfence();
    __syncthreads();
    if (tid == 0) last = (atomicAdd(&counters[B.cnt_idx], 1u) == (unsigned)(B.bslice - 1));
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (g == 0 && j < b) {
      double sx = 0.0, sy = 0.0;
      for (int q = 0; q < B.bslice; ++q) {
        const double2 pq = partials[B.part_off + q * b + j];
        sx += pq.x;
        sy += pq.y;
      }
      sum = make_double2(sx, sy);
    }
    if (tid == 0) atomicExch(&counters[B.cnt_idx], 0u);
  }
  if (g == 0 && j < b) {
    const double2 yy = ybuf[B.r0 + j];
    t[j] = make_double2(yy.x - sum.x, yy.y - sum.y);
  }
  __syncthreads();
  // z_j = sum_{i >= j} D(i, j) t_i over i = g, g + np, ...; D(i, j) at
  // doff + i (i + 1) / 2 + j (a row per step: coalesced over j)
  {
    auto dload = [&](int i) {
      return (j < b && i < b && i >= j) ? drow[B.doff + (int64_t)i * (i + 1) / 2 + j] : 0.0;
    };
    double zx = 0.0, zy = 0.0;
    for (int i0 = g; i0 < b; i0 += U * np) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = dload(i0 + u * np);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * np;
        if (j < b && i < b && i >= j) {
          const double2 ti = t[i];
          zx += v[u] * ti.x;
          zy += v[u] * ti.y;
        }
      }
    }
    red[tid] = make_double2(zx, zy);
  }
  __syncthreads();
  if (g == 0 && j < b) {
    const double2 z = combine_parts(red, j, bp, np);
    x[B.r0 + j] = z;
    if (out) out[perm[B.r0 + j]] = z;
  }
}

// ---------------------------------------------------------------------------
// Wavefront-per-block level kernels: one wavefront solves one block of at
// most 64 rows (lane r holds row r), reading the dense inverse and the panel straight
// from global memory in coalesced order (each entry is used once, so nothing
// is staged in LDS) and broadcasting the vector entries across lanes.  Four
// independent wavefronts per workgroup, no barriers.
// ---------------------------------------------------------------------------

// v of lane `src` (uniform) in every lane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double2 lane_bcast2(double2 v, int src) {
  return make_double2(lane_bcast(v.x, src), lane_bcast(v.y, src));
}

// Sum of the update entries upd[cidx[q]], q in [q0, q1), loads in batches.
__device__ __forceinline__ double2 gather_updates(int64_t q0, int64_t q1,
                                                  const int32_t *__restrict__ cidx,
                                                  const double2 *__restrict__ upd) {
  double ax = 0.0, ay = 0.0;
  constexpr int U = 8;
  for (int64_t q = q0; q < q1; q += U) {
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = q + u < q1 ? cidx[q + u] : -1;
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = idx[u] >= 0 ? upd[idx[u]] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ax += v[u].x;
      ay += v[u].y;
    }
  }
  return make_double2(ax, ay);
}

// Forward, one level (blocks of at most 64 rows): per item (block, slice)
//   t = b_rows - contributions,  y = D t (D packed column-major),
//   upd[k] = sum_j P(k, j) y_j for the slice's panel rows (P column-major),
// slice 0 writes y to ybuf.  Lane r holds row r for the first two steps and
// panel row k0 + kc + r for the third.  Loads are issued C per lane at a
// time (all independent); D's first C columns before the right-hand side is
// formed.  With FUSED (first level) b is assembled here and the workgroups
// after the items assemble the other rows and finish the MSD.
template <bool FUSED, int C>
__global__ __launch_bounds__(256) void k_wave_fwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
    const double *__restrict__ dcol, const double *__restrict__ pcol, double2 *x,
    double2 *__restrict__ ybuf, double2 *__restrict__ upd, AssembleArgs A) {
  const int item_groups = (count + 3) / 4;
  if (FUSED && (int)blockIdx.x >= item_groups) {
    fused_tail(A, x, (int)blockIdx.x - item_groups);
    return;
  }
  const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (w >= count) return;
  const int lane = threadIdx.x & 63;
  const int2 it = items[w];
  const DevBlock B = blocks[it.x];
  if (!B.active) return;
  const int b = B.r1 - B.r0, m = B.m;
  const int k0 = it.y * B.rslice;
  const int kn = max(0, min(B.rslice, m - k0));
  // D(r, j), r >= j, at doff + j b - j (j - 1) / 2 + (r - j)
  auto dload = [&](int j) {
    return (j < b && j <= lane && lane < b)
               ? dcol[B.doff + (int64_t)j * b - (int64_t)j * (j - 1) / 2 + (lane - j)]
               : 0.0;
  };
  double v[C];
#pragma unroll
  for (int u = 0; u < C; ++u) v[u] = dload(u);
  double2 t = make_double2(0.0, 0.0);
  if (lane < b) {
    const int row = B.r0 + lane;
    if (FUSED) {
      t = assemble_b(row, A.mptr, A.ment, A.minv, A.h, A.u, A.tau);
    } else {
      const double2 c = gather_updates(cptr[row], cptr[row + 1], cidx, upd);
      const double2 bb = x[row];
      t = make_double2(bb.x - c.x, bb.y - c.y);
    }
  }
  // y_r = sum_{j <= r} D(r, j) t_j
  double2 y = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < b; j0 += C) {
    if (j0 > 0) {
#pragma unroll
      for (int u = 0; u < C; ++u) v[u] = dload(j0 + u);
    }
#pragma unroll
    for (int u = 0; u < C; ++u)
      if (j0 + u < b) {
        const double2 tj = lane_bcast2(t, j0 + u);
        y.x += v[u] * tj.x;
        y.y += v[u] * tj.y;
      }
  }
  // upd[k] = sum_j P(k, j) y_j, panel entry (k, j) at poff + j m + k
  for (int kc = 0; kc < kn; kc += 64) {
    const int kk = k0 + kc + lane;
    const bool on = kc + lane < kn;
    double2 acc = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < b; j0 += C) {
#pragma unroll
      for (int u = 0; u < C; ++u)
        v[u] = (j0 + u < b && on) ? pcol[B.poff + (int64_t)(j0 + u) * m + kk] : 0.0;
#pragma unroll
      for (int u = 0; u < C; ++u)
        if (j0 + u < b) {
          const double2 yj = lane_bcast2(y, j0 + u);
          acc.x += v[u] * yj.x;
          acc.y += v[u] * yj.y;
        }
    }
    if (on) upd[B.boff + kk] = acc;
  }
  if (it.y == 0 && lane < b) ybuf[B.r0 + lane] = y;
}

// Backward, one level (blocks of at most 64 rows, not split): per block
//   s_j = sum_k P(k, j) z(below_k)   (P row-major; z gathered 64 rows at a time),
//   t = y - s,  z_j = sum_{i >= j} D(i, j) t_i   (D packed row-major),
// z written to x and, when `out` is given, to natural node order.  Lane j holds
// column j.  Loads are issued C per lane at a time; the first panel chunk's
// with the z gather.
template <int C>
__global__ __launch_bounds__(256) void k_wave_bwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int32_t *__restrict__ below_idx, const double *__restrict__ drow,
    const double *__restrict__ prow, double2 *x, const double2 *__restrict__ ybuf,
    const int32_t *__restrict__ perm, double2 *__restrict__ out) {
  const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (w >= count) return;
  const int lane = threadIdx.x & 63;
  const int2 it = items[w];
  const DevBlock B = blocks[it.x];
  if (!B.active) return;
  const int b = B.r1 - B.r0, m = B.m;
  const bool col = lane < b;
  auto pload = [&](int k) { return (k < m && col) ? prow[B.poff + (int64_t)k * b + lane] : 0.0; };
  double v[C];
#pragma unroll
  for (int u = 0; u < C; ++u) v[u] = pload(u);
  double2 s = make_double2(0.0, 0.0);
  for (int kc = 0; kc < m; kc += 64) {
    const double2 zl = kc + lane < m ? x[below_idx[B.boff + kc + lane]] : make_double2(0.0, 0.0);
    const int kend = min(64, m - kc);
    for (int k0 = 0; k0 < kend; k0 += C) {
      if (kc > 0 || k0 > 0) {
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = pload(kc + k0 + u);
      }
#pragma unroll
      for (int u = 0; u < C; ++u)
        if (k0 + u < kend) {
          const double2 zk = lane_bcast2(zl, k0 + u);
          s.x += v[u] * zk.x;
          s.y += v[u] * zk.y;
        }
    }
  }
  double2 t = make_double2(0.0, 0.0);
  if (col) {
    const double2 y = ybuf[B.r0 + lane];
    t = make_double2(y.x - s.x, y.y - s.y);
  }
  // z_j = sum_{i >= j} D(i, j) t_i, D(i, j) at doff + i (i + 1) / 2 + j
  double2 z = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < b; i0 += C) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int i = i0 + u;
      v[u] = (i < b && lane <= i && col) ? drow[B.doff + (int64_t)i * (i + 1) / 2 + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < C; ++u)
      if (i0 + u < b) {
        const double2 ti = lane_bcast2(t, i0 + u);
        z.x += v[u] * ti.x;
        z.y += v[u] * ti.y;
      }
  }
  if (col) {
    x[B.r0 + lane] = z;
    if (out) out[perm[B.r0 + lane]] = z;
  }
}

// ---------------------------------------------------------------------------
// Half-wavefront-per-block level kernels for levels whose blocks have at most
// 32 rows (the leaves of the dissection): each wavefront solves two blocks,
// one per 32-lane half, so a load instruction moves twice the data of the
// wavefront-per-block form.  The vector entries a half broadcasts go through
// its own 32-entry LDS slot (one read per entry, same address for the whole
// half); within a wavefront LDS operations complete in issue order, so a slot
// is rewritten only after the reads issued before it.
// ---------------------------------------------------------------------------

// Forward, one level: per item (block, slice) t = b_rows - contributions (or
// the assembled b with FUSED), y = D t, upd = P y for the slice's panel rows
// (D packed column-major, P column-major), y to ybuf by slice 0.  Lane r of a
// half holds row r, then panel rows k0 + kc + r.
template <bool FUSED, int C>
__global__ __launch_bounds__(256) void k_half_fwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
    const double *__restrict__ dcol, const double *__restrict__ pcol, double2 *x,
    double2 *__restrict__ ybuf, double2 *__restrict__ upd, AssembleArgs A) {
  const int item_groups = (count + 7) / 8;
  if (FUSED && (int)blockIdx.x >= item_groups) {
    fused_tail(A, x, (int)blockIdx.x - item_groups);
    return;
  }
  __shared__ double2 vec[8][32];
  const int hw = (int)threadIdx.x >> 5, r = (int)threadIdx.x & 31;
  const int w = (int)blockIdx.x * 8 + hw;
  if ((int)blockIdx.x * 8 + (hw & ~1) >= count) return;    // both halves idle
  DevBlock B{};
  int b = 0, m = 1, k0 = 0, kn = 0, slice = 1;
  if (w < count) {
    const int2 it = items[w];
    B = blocks[it.x];
    // a retired pair's half idles; selects rather than a branch, so that the
    // record's fields and the item arrive in one round of loads
    const bool on = B.active != 0;
    b = on ? B.r1 - B.r0 : 0;
    m = on ? B.m : 1;
    slice = on ? it.y : 1;
    k0 = on ? it.y * B.rslice : 0;
    kn = on ? max(0, min(B.rslice, m - k0)) : 0;
  }
  double2 *v2 = vec[hw];
  // D(r, j), r >= j, at doff + j b - j (j - 1) / 2 + (r - j)
  auto dload = [&](int j) {
    return (j < b && j <= r && r < b)
               ? dcol[B.doff + (int64_t)j * b - (int64_t)j * (j - 1) / 2 + (r - j)]
               : 0.0;
  };
  double v[C];
#pragma unroll
  for (int u = 0; u < C; ++u) v[u] = dload(u);
  double2 t = make_double2(0.0, 0.0);
  if (r < b) {
    const int row = B.r0 + r;
    if (FUSED) {
      t = assemble_b(row, A.mptr, A.ment, A.minv, A.h, A.u, A.tau);
    } else {
      const double2 c = gather_updates(cptr[row], cptr[row + 1], cidx, upd);
      const double2 bb = x[row];
      t = make_double2(bb.x - c.x, bb.y - c.y);
    }
  }
  v2[r] = t;
  __builtin_amdgcn_wave_barrier();
  // y_r = sum_{j <= r} D(r, j) t_j
  double2 y = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < b; j0 += C) {
    if (j0 > 0) {
#pragma unroll
      for (int u = 0; u < C; ++u) v[u] = dload(j0 + u);
    }
    // no guard on j0 + u < b: the slot holds t_j = 0 and D(r, j) = 0 past
    // the block (j0 + u < 32), so all C reads go out together
    double2 tj[C];
#pragma unroll
    for (int u = 0; u < C; ++u) tj[u] = v2[j0 + u];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      y.x += v[u] * tj[u].x;
      y.y += v[u] * tj[u].y;
    }
  }
  __builtin_amdgcn_wave_barrier();
  v2[r] = y;
  __builtin_amdgcn_wave_barrier();
  // upd[k] = sum_j P(k, j) y_j, panel entry (k, j) at poff + j m + k
  for (int kc = 0; kc < kn; kc += 32) {
    const int kk = k0 + kc + r;
    const bool on = kc + r < kn;
    double2 acc = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < b; j0 += C) {
#pragma unroll
      for (int u = 0; u < C; ++u)
        v[u] = (j0 + u < b && on) ? pcol[B.poff + (int64_t)(j0 + u) * m + kk] : 0.0;
      double2 yj[C];                 // y_j = 0 and P(k, j) = 0 past the block
#pragma unroll
      for (int u = 0; u < C; ++u) yj[u] = v2[j0 + u];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        acc.x += v[u] * yj[u].x;
        acc.y += v[u] * yj[u].y;
      }
    }
    if (on) upd[B.boff + kk] = acc;
  }
  if (slice == 0 && r < b) ybuf[B.r0 + r] = y;
}

// Backward, one level (blocks of at most 32 rows, not split): per block
//   s_j = sum_k P(k, j) z(below_k)   (P row-major; z gathered 32 rows at a time),
//   t = y - s,  z_j = sum_{i >= j} D(i, j) t_i   (D packed row-major),
// z written to x and, when `out` is given, to natural node order.  Lane r of a
// half holds column r.
template <int C>
__global__ __launch_bounds__(256) void k_half_bwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int32_t *__restrict__ below_idx, const double *__restrict__ drow,
    const double *__restrict__ prow, double2 *x, const double2 *__restrict__ ybuf,
    const int32_t *__restrict__ perm, double2 *__restrict__ out) {
  __shared__ double2 vec[8][32];
  const int hw = (int)threadIdx.x >> 5, r = (int)threadIdx.x & 31;
  const int w = (int)blockIdx.x * 8 + hw;
  if ((int)blockIdx.x * 8 + (hw & ~1) >= count) return;    // both halves idle
  DevBlock B{};
  int b = 0, m = 0;
  if (w < count) {
    B = blocks[items[w].x];
    const bool on = B.active != 0;             // a retired pair's half idles
    b = on ? B.r1 - B.r0 : 0;
    m = on ? B.m : 0;
  }
  double2 *v2 = vec[hw];
  const bool col = r < b;
  auto pload = [&](int k) { return (k < m && col) ? prow[B.poff + (int64_t)k * b + r] : 0.0; };
  double v[C];
#pragma unroll
  for (int u = 0; u < C; ++u) v[u] = pload(u);
  double2 s = make_double2(0.0, 0.0);
  for (int kc = 0; kc < m; kc += 32) {
    const double2 zl = kc + r < m ? x[below_idx[B.boff + kc + r]] : make_double2(0.0, 0.0);
    __builtin_amdgcn_wave_barrier();
    v2[r] = zl;
    __builtin_amdgcn_wave_barrier();
    const int kend = min(32, m - kc);
    for (int k0 = 0; k0 < kend; k0 += C) {
      if (kc > 0 || k0 > 0) {
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = pload(kc + k0 + u);
      }
      double2 zk[C];                 // z = 0 and P(k, j) = 0 past the panel
#pragma unroll
      for (int u = 0; u < C; ++u) zk[u] = v2[k0 + u];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        s.x += v[u] * zk[u].x;
        s.y += v[u] * zk[u].y;
      }
    }
  }
  double2 t = make_double2(0.0, 0.0);
  if (col) {
    const double2 yv = ybuf[B.r0 + r];
    t = make_double2(yv.x - s.x, yv.y - s.y);
  }
  __builtin_amdgcn_wave_barrier();
  v2[r] = t;
  __builtin_amdgcn_wave_barrier();
  // z_j = sum_{i >= j} D(i, j) t_i, D(i, j) at doff + i (i + 1) / 2 + j
  double2 z = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < b; i0 += C) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int i = i0 + u;
      v[u] = (i < b && r <= i && col) ? drow[B.doff + (int64_t)i * (i + 1) / 2 + r] : 0.0;
    }
    double2 ti[C];                   // t_i = 0 and D(i, j) = 0 past the block
#pragma unroll
    for (int u = 0; u < C; ++u) ti[u] = v2[i0 + u];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      z.x += v[u] * ti[u].x;
      z.y += v[u] * ti[u].y;
    }
  }
  if (col) {
    x[B.r0 + r] = z;
    if (out) out[perm[B.r0 + r]] = z;
  }
}

// ---------------------------------------------------------------------------
// LDS-staged wavefront-per-block level kernels: one wavefront (the whole
// workgroup) per block of at most 64 rows whose panel is not split; the
// block's dense inverse and panel are copied straight from global memory into
// LDS with 16-byte direct loads (all in flight at once, no registers held)
// while the right-hand side is gathered, then read back in conflict-free
// order (consecutive lanes, consecutive doubles).
// ---------------------------------------------------------------------------

// Copies `bytes` from 16-byte aligned global memory into this wavefront's LDS
// (16-byte aligned), 16 bytes per lane and instruction; completion is waited
// for by the caller.
__device__ __forceinline__ void stage_direct(const void *src, void *lds, int bytes, int lane) {
  const int nch = (bytes + 15) >> 4;
  for (int c0 = 0; c0 < nch; c0 += 64)
    if (c0 + lane < nch)
      __builtin_amdgcn_global_load_lds(
          static_cast<const char *>(src) + (size_t)(c0 + lane) * 16,
          (__attribute__((address_space(3))) void *)(static_cast<char *>(lds) + (size_t)c0 * 16),
          16, 0, 0);
}

// Waits for every outstanding load (direct LDS copies included) of the wavefront.
__device__ __forceinline__ void wait_all_loads() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Forward, one level: per block, t = b_rows - contributions (or the assembled
// b with FUSED), y = D t, upd = P y (D packed column-major, P column-major,
// both staged in LDS), y to ybuf.  The item of slice 0 takes the whole panel
// (the other slices' items return at once).  With FUSED the workgroups after the blocks
// assemble the other rows (64 per workgroup) and finish the MSD.
template <bool FUSED>
__global__ __launch_bounds__(64) void k_lds_fwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
    const double *__restrict__ dcol, const double *__restrict__ pcol, double2 *x,
    double2 *__restrict__ ybuf, double2 *__restrict__ upd, AssembleArgs A) {
  extern __shared__ double smem[];
  if (FUSED && (int)blockIdx.x >= count) {
    fused_tail(A, x, (int)blockIdx.x - count);
    return;
  }
  const int lane = threadIdx.x;
  const int2 it = items[blockIdx.x];
  if (it.y != 0) return;                      // slice 0 takes the whole panel
  const DevBlock B = blocks[it.x];
  if (!B.active) return;
  const int b = B.r1 - B.r0, m = B.m;
  const int nd = b * (b + 1) / 2;
  double *D = smem;
  double *P = smem + (nd + 1) / 2 * 2;
  stage_direct(dcol + B.doff, D, 8 * nd, lane);
  stage_direct(pcol + B.poff, P, 8 * m * b, lane);
  double2 t = make_double2(0.0, 0.0);
  if (lane < b) {
    const int row = B.r0 + lane;
    if (FUSED) {
      t = assemble_b(row, A.mptr, A.ment, A.minv, A.h, A.u, A.tau);
    } else {
      const double2 c = gather_updates(cptr[row], cptr[row + 1], cidx, upd);
      const double2 bb = x[row];
      t = make_double2(bb.x - c.x, bb.y - c.y);
    }
  }
  wait_all_loads();
  // y_r = sum_{j <= r} D(r, j) t_j, D(r, j) at j b - j (j - 1) / 2 + (r - j)
  double2 y = make_double2(0.0, 0.0);
  for (int j = 0; j < b; ++j) {
    const double2 tj = lane_bcast2(t, j);
    if (lane >= j && lane < b) {
      const double d = D[j * b - j * (j - 1) / 2 + (lane - j)];
      y.x += d * tj.x;
      y.y += d * tj.y;
    }
  }
  // upd[k] = sum_j P(k, j) y_j, P(k, j) at j m + k
  for (int kc = 0; kc < m; kc += 64) {
    const int kk = kc + lane;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < b; ++j) {
      const double2 yj = lane_bcast2(y, j);
      if (kk < m) {
        const double v = P[j * m + kk];
        acc.x += v * yj.x;
        acc.y += v * yj.y;
      }
    }
    if (kk < m) upd[B.boff + kk] = acc;
  }
  if (lane < b) ybuf[B.r0 + lane] = y;
}

// Backward, one level: per block, s = P^T z(below) (P row-major in LDS, z
// gathered 64 rows at a time), t = y - s, z = D^-T t (D packed row-major in
// LDS); z to x and, when `out` is given, to natural node order.
__global__ __launch_bounds__(64) void k_lds_bwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items, int count,
    const int32_t *__restrict__ below_idx, const double *__restrict__ drow,
    const double *__restrict__ prow, double2 *x, const double2 *__restrict__ ybuf,
    const int32_t *__restrict__ perm, double2 *__restrict__ out) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x;
  const int2 it = items[blockIdx.x];
  const DevBlock B = blocks[it.x];
  if (!B.active) return;
  const int b = B.r1 - B.r0, m = B.m;
  const int nd = b * (b + 1) / 2;
  double *D = smem;
  double *P = smem + (nd + 1) / 2 * 2;
  stage_direct(drow + B.doff, D, 8 * nd, lane);
  stage_direct(prow + B.poff, P, 8 * m * b, lane);
  const double2 y = lane < b ? ybuf[B.r0 + lane] : make_double2(0.0, 0.0);
  double2 zl = lane < m ? x[below_idx[B.boff + lane]] : make_double2(0.0, 0.0);
  wait_all_loads();
  // s_j = sum_k P(k, j) z_k, P(k, j) at k b + j
  double2 s = make_double2(0.0, 0.0);
  for (int kc = 0; kc < m; kc += 64) {
    if (kc > 0) zl = kc + lane < m ? x[below_idx[B.boff + kc + lane]] : make_double2(0.0, 0.0);
    const int kend = min(64, m - kc);
    for (int k = 0; k < kend; ++k) {
      const double2 zk = lane_bcast2(zl, k);
      if (lane < b) {
        const double v = P[(kc + k) * b + lane];
        s.x += v * zk.x;
        s.y += v * zk.y;
      }
    }
  }
  const double2 t = make_double2(y.x - s.x, y.y - s.y);
  // z_j = sum_{i >= j} D(i, j) t_i, D(i, j) at i (i + 1) / 2 + j
  double2 z = make_double2(0.0, 0.0);
  for (int i = 0; i < b; ++i) {
    const double2 ti = lane_bcast2(t, i);
    if (lane <= i && lane < b) {
      const double d = D[i * (i + 1) / 2 + lane];
      z.x += d * ti.x;
      z.y += d * ti.y;
    }
  }
  if (lane < b) {
    x[B.r0 + lane] = z;
    if (out) out[perm[B.r0 + lane]] = z;
  }
}

// Apex of the forward solve, step 1: t = b - (update entries of the non-apex
// blocks) for every apex row of every pair (thread per row, global list).
__global__ __launch_bounds__(256) void k_apex_rhs(int n_rows, const int32_t *__restrict__ rows,
                                                  const int64_t *__restrict__ acptr,
                                                  const int32_t *__restrict__ acidx,
                                                  const double2 *__restrict__ upd,
                                                  const double2 *__restrict__ x,
                                                  double2 *__restrict__ tbuf) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_rows) return;
  const int64_t q1 = acptr[g + 1];
  double ax = 0.0, ay = 0.0;
  constexpr int U = 8;
  for (int64_t q = acptr[g]; q < q1; q += U) {
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = q + u < q1 ? acidx[q + u] : -1;
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = idx[u] >= 0 ? upd[idx[u]] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ax += v[u].x;
      ay += v[u].y;
    }
  }
  const double2 bb = x[rows[g]];
  tbuf[g] = make_double2(bb.x - ax, bb.y - ay);
}

// Dot products of one wavefront's two rows against an LDS vector: row A has
// entries q in [qa, la), row B in [qb, lb), each at base[q] of its own pointer
// (position q of the LDS vector).  The first batch of loads is issued by the
// caller (before its LDS staging); U loads per lane per row and batch.
template <int U>
struct RowPair {
  double va[U], vb[U];
  __device__ __forceinline__ void load(const double *pa, int qa, int la, const double *pb, int qb,
                                       int lb, int lane) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q0 = qa + lane + 64 * u, q1 = qb + lane + 64 * u;
      va[u] = q0 < la ? pa[q0] : 0.0;
      vb[u] = q1 < lb ? pb[q1] : 0.0;
    }
  }
  __device__ __forceinline__ void fma(const double2 *v, int qa, int la, int qb, int lb, int lane,
                                      double2 &sa, double2 &sb) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q0 = qa + lane + 64 * u, q1 = qb + lane + 64 * u;
      if (q0 < la) {
        const double2 t = v[q0];
        sa.x += va[u] * t.x;
        sa.y += va[u] * t.y;
      }
      if (q1 < lb) {
        const double2 t = v[q1];
        sb.x += vb[u] * t.x;
        sb.y += vb[u] * t.y;
      }
    }
  }
};

// Apex forward, y = X t with X = L(apex, apex)^-1: row r of X is nonzero
// only on columns [c0, r] (its block's subtree).  A work item takes up to 8
// rows of one block against one segment of at most kApexSeg columns: each
// wavefront loads its two rows' entries of the segment, the segment of t is
// staged in LDS meanwhile, and the dot products (fixed-order reduction) go to
// the item's partial slots.
__global__ __launch_bounds__(256) void k_apex_fwd(const ApexFwdItem *__restrict__ items,
                                                  const double *__restrict__ xf,
                                                  const double2 *__restrict__ tbuf,
                                                  double2 *__restrict__ part) {
  __shared__ double2 tl[kApexSeg];
  const ApexFwdItem it = items[blockIdx.x];
  if (!it.active) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // rows ra, rb; entries of row r in the segment: columns k0 .. min(k1, r+1)-1,
  // stored from xoff0 + sum_{a0 <= s < r} (s - c0 + 1) + (k0 - c0) on
  const int ra = it.a0 + wave, rb = ra + 4;
  const int la = ra < it.a1 ? max(0, min(it.k1, ra + 1) - it.k0) : 0;
  const int lb = rb < it.a1 ? max(0, min(it.k1, rb + 1) - it.k0) : 0;
  const int64_t w0 = it.a0 - it.c0 + 1;                 // length of row a0
  const int64_t da = ra - it.a0, db = rb - it.a0;
  const double *pa = xf + it.xoff0 + da * w0 + da * (da - 1) / 2 + (it.k0 - it.c0);
  const double *pb = xf + it.xoff0 + db * w0 + db * (db - 1) / 2 + (it.k0 - it.c0);
  constexpr int U = 8;
  RowPair<U> rp;
  rp.load(pa, 0, la, pb, 0, lb, lane);
  const int kn = it.k1 - it.k0;
  for (int j = threadIdx.x; j < kn; j += blockDim.x) tl[j] = tbuf[it.k0 + j];
  __syncthreads();
  double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
  rp.fma(tl, 0, la, 0, lb, lane, sa, sb);
  for (int o = 64 * U; o < la || o < lb; o += 64 * U) {
    rp.load(pa, o, la, pb, o, lb, lane);
    rp.fma(tl, o, la, o, lb, lane, sa, sb);
  }
  sa.x = wave_sum(sa.x);
  sa.y = wave_sum(sa.y);
  sb.x = wave_sum(sb.x);
  sb.y = wave_sum(sb.y);
  if (lane == 0) {
    if (la > 0) part[it.part + (ra - it.a0)] = sa;
    if (lb > 0) part[it.part + (rb - it.a0)] = sb;
  }
}

// y_a = sum of row a's forward segment partials, in segment order (thread per
// apex position).
__global__ __launch_bounds__(256) void k_apex_combine(int n, const ApexRow *__restrict__ arow,
                                                      const double2 *__restrict__ part,
                                                      double2 *__restrict__ y) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const ApexRow R = arow[a];
  double2 s = make_double2(0.0, 0.0);
  constexpr int U = 4;
  for (int g0 = 0; g0 < R.nseg; g0 += U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = g0 + u < R.nseg ? part[R.part + (int64_t)(g0 + u) * R.stride] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s.x += v[u].x;
      s.y += v[u].y;
    }
  }
  y[a] = s;
}

// Apex backward, z = X^T y: z_r is the dot product of column r of X over r's
// path (its block's rows from r on, then the ancestor blocks' rows) with y on
// the same rows.  A work item takes up to 8 rows of one block: each
// wavefront loads its two columns' first entries while the path list of the
// first row is staged in LDS from y; row r uses the list from position
// r - a0 on.  z goes to x and, when `out` is given, to natural node order.
__global__ __launch_bounds__(256) void k_apex_bwd(const ApexBwdItem *__restrict__ items,
                                                  const int2 *__restrict__ rng,
                                                  const int32_t *__restrict__ rows,
                                                  const double2 *__restrict__ y,
                                                  const double *__restrict__ xb, double2 *x,
                                                  const int32_t *__restrict__ perm,
                                                  double2 *__restrict__ out) {
  extern __shared__ double2 yl[];              // the longest path of the launch
  __shared__ int2 rl[kApexMaxRanges];          // the item's ancestor ranges
  const ApexBwdItem it = items[blockIdx.x];
  if (!it.active) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ra = it.a0 + wave, rb = ra + 4;
  const int qa = ra - it.a0, qb = rb - it.a0;
  const int la = ra < it.a1 ? it.len : 0, lb = rb < it.a1 ? it.len : 0;
  // column r stores list positions r - a0 .. len - 1, columns back to back
  const int64_t da = qa, db = qb;
  const double *pa = xb + (it.xoff0 + da * it.len - da * (da - 1) / 2 - qa);
  const double *pb = xb + (it.xoff0 + db * it.len - db * (db - 1) / 2 - qb);
  constexpr int U = 8;
  RowPair<U> rp;
  rp.load(pa, qa, la, pb, qb, lb, lane);
  const int own = it.e - it.a0;
  if ((int)threadIdx.x < it.n_rng) rl[threadIdx.x] = rng[it.rng_off + threadIdx.x];
  __syncthreads();
  for (int q = threadIdx.x; q < it.len; q += blockDim.x) {
    int a;
    if (q < own) {
      a = it.a0 + q;
    } else {
      int r = q - own, k = 0;
      while (k + 1 < it.n_rng && r >= rl[k].y - rl[k].x) {
        r -= rl[k].y - rl[k].x;
        ++k;
      }
      a = rl[k].x + r;
    }
    yl[q] = y[a];
  }
  __syncthreads();
  double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
  rp.fma(yl, qa, la, qb, lb, lane, sa, sb);
  for (int o = 64 * U; qa + o < la || qb + o < lb; o += 64 * U) {
    rp.load(pa, qa + o, la, pb, qb + o, lb, lane);
    rp.fma(yl, qa + o, la, qb + o, lb, lane, sa, sb);
  }
  sa.x = wave_sum(sa.x);
  sa.y = wave_sum(sa.y);
  sb.x = wave_sum(sb.x);
  sb.y = wave_sum(sb.y);
  if (lane == 0) {
    if (la > 0) {
      const int row = rows[ra];
      x[row] = sa;
      if (out) out[perm[row]] = sa;
    }
    if (lb > 0) {
      const int row = rows[rb];
      x[row] = sb;
      if (out) out[perm[row]] = sb;
    }
  }
}

// Two tiles per workgroup: their loads overlap, and the launch's workgroups
// stay within the LDS and register budget of eight per CU (64 VGPRs).
__global__ __launch_bounds__(256) void k_warp_msd(
    const TileItem *__restrict__ tiles, const double2 *__restrict__ u,
    const int4 *__restrict__ tile_nodes, const int2 *__restrict__ tile_pbc,
    const uint8_t *__restrict__ tile_loc, const float *__restrict__ coef,
    const float *__restrict__ re, float *__restrict__ warped, double *__restrict__ partials,
    unsigned *flags, int n_tiles) {
  const int t0 = 2 * xcd_item((int)blockIdx.x, (int)gridDim.x);
  warp_tiles<2>(t0, n_tiles, tiles, u, tile_nodes, tile_pbc, tile_loc, coef, re, warped, partials,
                flags);
}

__global__ __launch_bounds__(256) void k_msd_finish(const DevPair *__restrict__ pairs, int n_pairs,
                                                    const double *__restrict__ partials,
                                                    double *__restrict__ msd) {
  msd_finish_group(pairs, n_pairs, partials, msd, blockIdx.x);
}

// Gather / scatter between the natural node order and the solve order.
__global__ void k_to_solve_order(int n, const double2 *__restrict__ src,
                                 const int32_t *__restrict__ iperm, double2 *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[iperm[i]] = src[i];
}

__global__ void k_from_solve_order(int n, const double2 *__restrict__ x,
                                   const int32_t *__restrict__ iperm, double2 *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = x[iperm[i]];
}

__global__ void k_h_from_solve_order(int n, const float2 *__restrict__ hs,
                                     const int32_t *__restrict__ iperm, float2 *__restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = hs[iperm[i]];
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------

thread_local LaunchTimer *tl_launch_timer = nullptr;

hipError_t launch_prefilter(const float *src_f, const double *src_d, double *tmp, float *out,
                            int H, int W, const double2 *tab_w, const double2 *tab_h,
                            hipStream_t s) {
  const int tb = 64;
  hipError_t e = src_f ? launch(k_prefilter_rows<float>, (H + tb - 1) / tb, tb, 0, s, src_f, tmp,
                                H, W, tab_w)
                       : launch(k_prefilter_rows<double>, (H + tb - 1) / tb, tb, 0, s, src_d, tmp,
                                H, W, tab_w);
  if (e != hipSuccess) return e;
  return launch(k_prefilter_cols, (W + tb - 1) / tb, tb, 0, s, tmp, out, H, W, tab_h);
}

hipError_t launch_prefilter_all(const PrefItem *row_items, int n_row_items,
                                const PrefItem *col_items, int n_col_items, const DevPair *pairs,
                                double *img, float *out, const double2 *tab, hipStream_t s) {
  if (n_row_items == 0 || n_col_items == 0) return hipSuccess;
  hipError_t e = launch(k_prefilter_rows_all, n_row_items, 64, 0, s, row_items, pairs,
                        (const double *)img, img, tab);
  if (e != hipSuccess) return e;
  return launch(k_prefilter_cols_all, n_col_items, 64, 0, s, col_items, pairs, img, out, tab);
}

hipError_t launch_sample_rho(const NodeItem *items, int n_items, const DevPair *pairs,
                             const int2 *xy, const float *coef_re, float *rho, hipStream_t s) {
  return launch(k_sample_rho, n_items, kNodeChunk, 0, s, items, pairs, xy, coef_re, rho);
}

hipError_t launch_sample(const NodeItem *items, int n_items, const DevPair *pairs,
                         const double2 *un, const int2 *xy, const float *coef, const float *rho,
                         float2 *h, unsigned *flags, const TileItem *tiles, int n_tiles,
                         const double2 *u, const int4 *tile_nodes, const int2 *tile_pbc,
                         const uint8_t *tile_loc, const float *re, double *partials,
                         hipStream_t s) {
  return launch(k_sample, n_items + n_tiles, kNodeChunk, 0, s, items, n_items, pairs, un, xy,
                coef, rho, h, flags, tiles, u, tile_nodes, tile_pbc, tile_loc, re, partials,
                n_tiles);
}

hipError_t launch_assemble(int n, const int32_t *mptr, const uint32_t *ment, const float *minv,
                           const float2 *h, const double2 *u, double2 *x, double tau,
                           const DevPair *pairs, int n_pairs, const double *partials,
                           double *finish_msd, const int32_t *active, hipStream_t s) {
  const int groups = (n + 255) / 256 + (finish_msd ? (n_pairs + 3) / 4 : 0);
  return launch(k_assemble, groups, 256, 0, s, n, mptr, ment, minv, h, u, x, tau, pairs, n_pairs,
                partials, finish_msd, active);
}

hipError_t launch_solve_fwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int64_t *cptr, const int32_t *cidx,
                                  const double *dcol, const double *prow, const double *pcol,
                                  double2 *x, double2 *ybuf, double2 *upd,
                                  const AssembleArgs *fuse, hipStream_t s) {
  if (nt == 1) {                              // wavefront per block, LDS staged
    int groups = count;
    if (fuse) groups += (fuse->n_rows + 63) / 64 + (fuse->finish_msd ? fuse->n_pairs : 0);
    if (groups == 0) return hipSuccess;
    return fuse ? launch(k_lds_fwd<true>, groups, 64, lds_bytes, s, blocks, items, count, cptr,
                         cidx, dcol, pcol, x, ybuf, upd, *fuse)
                : launch(k_lds_fwd<false>, groups, 64, lds_bytes, s, blocks, items, count, cptr,
                         cidx, dcol, pcol, x, ybuf, upd, AssembleArgs{});
  }
  if (nt == 32 || nt == 33 || nt == 34) {     // half-wavefront per block (at most 32 rows),
                                              // 8 (32), 16 (33) or 4 (34) loads per batch
    int groups = (count + 7) / 8;
    if (fuse)
      groups += (fuse->n_rows + 255) / 256 + (fuse->finish_msd ? (fuse->n_pairs + 3) / 4 : 0);
    if (groups == 0) return hipSuccess;
    if (nt == 33)
      return fuse ? launch(k_half_fwd<true, 16>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, *fuse)
                  : launch(k_half_fwd<false, 16>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, AssembleArgs{});
    if (nt == 34)
      return fuse ? launch(k_half_fwd<true, 4>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, *fuse)
                  : launch(k_half_fwd<false, 4>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, AssembleArgs{});
    return fuse ? launch(k_half_fwd<true, 8>, groups, 256, 0, s, blocks, items, count, cptr, cidx,
                         dcol, pcol, x, ybuf, upd, *fuse)
                : launch(k_half_fwd<false, 8>, groups, 256, 0, s, blocks, items, count, cptr,
                         cidx, dcol, pcol, x, ybuf, upd, AssembleArgs{});
  }
  if (nt == 8 || nt == 16) {                  // wavefront per block, nt loads per batch
    int groups = (count + 3) / 4;
    if (fuse)
      groups += (fuse->n_rows + 255) / 256 + (fuse->finish_msd ? (fuse->n_pairs + 3) / 4 : 0);
    if (groups == 0) return hipSuccess;
    const AssembleArgs none{};
    if (nt == 8)
      return fuse ? launch(k_wave_fwd<true, 8>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, *fuse)
                  : launch(k_wave_fwd<false, 8>, groups, 256, 0, s, blocks, items, count, cptr,
                           cidx, dcol, pcol, x, ybuf, upd, none);
    return fuse ? launch(k_wave_fwd<true, 16>, groups, 256, 0, s, blocks, items, count, cptr, cidx,
                         dcol, pcol, x, ybuf, upd, *fuse)
                : launch(k_wave_fwd<false, 16>, groups, 256, 0, s, blocks, items, count, cptr,
                         cidx, dcol, pcol, x, ybuf, upd, none);
  }
  nt = nt == 64 || nt == 128 || nt == 512 || nt == 1024 ? nt : 256;
  if (!fuse) {
    auto k = nt == 64    ? k_solve_fwd<64, false>
             : nt == 128 ? k_solve_fwd<128, false>
             : nt == 512 ? k_solve_fwd<512, false>
             : nt == 1024 ? k_solve_fwd<1024, false>
                          : k_solve_fwd<256, false>;
    if (count == 0) return hipSuccess;
    return launch(k, count, nt, lds_bytes, s, blocks, items, count, cptr, cidx, dcol, pcol, x,
                  ybuf, upd, AssembleArgs{});
  }
  auto k = nt == 64    ? k_solve_fwd<64, true>
           : nt == 128 ? k_solve_fwd<128, true>
           : nt == 512 ? k_solve_fwd<512, true>
           : nt == 1024 ? k_solve_fwd<1024, true>
                        : k_solve_fwd<256, true>;
  const int groups = count + (fuse->n_rows + nt - 1) / nt +
                     (fuse->finish_msd ? (fuse->n_pairs + nt / 64 - 1) / (nt / 64) : 0);
  if (groups == 0) return hipSuccess;
  return launch(k, groups, nt, lds_bytes, s, blocks, items, count, cptr, cidx, dcol, pcol, x,
                ybuf, upd, *fuse);
}

hipError_t launch_solve_bwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int32_t *below_idx,
                                  const double *drow, const double *prow, double2 *x,
                                  const double2 *ybuf, const int32_t *perm, double2 *out,
                                  double2 *partials, unsigned *counters, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (nt == 1)
    return launch(k_lds_bwd, count, 64, lds_bytes, s, blocks, items, count, below_idx, drow, prow,
                  x, ybuf, perm, out);
  if (nt == 32 || nt == 33 || nt == 34)
    return launch(nt == 32 ? k_half_bwd<8> : nt == 33 ? k_half_bwd<16> : k_half_bwd<4>,
                  (count + 7) / 8, 256, 0, s, blocks, items, count, below_idx, drow, prow, x,
                  ybuf, perm, out);
  if (nt == 8 || nt == 16)
    return launch(nt == 8 ? k_wave_bwd<8> : k_wave_bwd<16>, (count + 3) / 4, 256, 0, s, blocks,
                  items, count, below_idx, drow, prow, x, ybuf, perm, out);
  nt = nt == 64 || nt == 128 || nt == 512 || nt == 1024 ? nt : 256;
  auto k = nt == 64    ? k_solve_bwd<64>
           : nt == 128 ? k_solve_bwd<128>
           : nt == 512 ? k_solve_bwd<512>
           : nt == 1024 ? k_solve_bwd<1024>
                        : k_solve_bwd<256>;
  return launch(k, count, nt, lds_bytes, s, blocks, items, below_idx, drow, prow, x, ybuf, perm,
                out, partials, counters);
}

hipError_t launch_apex_solve(int n_rows, const int32_t *rows, const int64_t *acptr,
                             const int32_t *acidx, const double2 *upd, double2 *x, double2 *tbuf,
                             const ApexFwdItem *fitems, int n_fitems, const double *xf,
                             double2 *part, const ApexRow *arow, double2 *ybuf,
                             const ApexBwdItem *bitems, int n_bitems, const int2 *rng, int bwd_lds,
                             const double *xb, const int32_t *perm, double2 *out, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  hipError_t e = launch(k_apex_rhs, (n_rows + 255) / 256, 256, 0, s, n_rows, rows, acptr, acidx,
                        upd, x, tbuf);
  if (e == hipSuccess) e = launch(k_apex_fwd, n_fitems, 256, 0, s, fitems, xf, tbuf, part);
  if (e == hipSuccess)
    e = launch(k_apex_combine, (n_rows + 255) / 256, 256, 0, s, n_rows, arow, part, ybuf);
  if (e == hipSuccess)
    e = launch(k_apex_bwd, n_bitems, 256, bwd_lds, s, bitems, rng, rows, (const double2 *)ybuf, xb,
               x, perm, out);
  return e;
}

hipError_t launch_warp_partials(const TileItem *tiles, int n_tiles, const double2 *u,
                                const int4 *tile_nodes, const int2 *tile_pbc,
                                const uint8_t *tile_loc, const float *coef, const float *re,
                                float *warped, double *partials, unsigned *flags,
                                hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return launch(k_warp_msd, (n_tiles + 1) / 2, kTile * kTile, 0, s, tiles, u, tile_nodes, tile_pbc,
                tile_loc, coef, re, warped, partials, flags, n_tiles);
}

hipError_t launch_msd_finish(const DevPair *pairs, int n_pairs, const double *partials,
                             double *msd, hipStream_t s) {
  return launch(k_msd_finish, (n_pairs + 3) / 4, 256, 0, s, pairs, n_pairs, partials, msd);
}

// ---------------------------------------------------------------------------
// Algorithm 1 as printed: explicit update with the mesh gradient (eq. 5, 6,
// 9, 10) and umbrella smoothing (eq. 11-14).  Node data in natural order.
// ---------------------------------------------------------------------------

// Smoothing and sampling (one workgroup per node item).  With `smooth` set,
// u_i = (1 - lambda) u0_i + lambda * mean of u0 over the 1-ring of i (eq. 14;
// the 1-ring as CSR r_ptr / r_idx, global node ids, its sum in CSR order);
// otherwise u is left as it is.  With `sample` set, t_i = s_Te(V_i - 1/2 + u_i)
// (FP32 spline value, eq. 3) and the node's record (deformed position V + u,
// t, r = t - rho) is written for the update.  The workgroups after the node
// items finish the MSD of `partials` into finish_msd (when given).
__global__ __launch_bounds__(256) void k_explicit_smooth(
    const NodeItem *__restrict__ items, int n_items, const DevPair *__restrict__ pairs,
    int n_pairs, const double2 *__restrict__ u0, double2 *__restrict__ u,
    const int32_t *__restrict__ r_ptr, const int32_t *__restrict__ r_idx, double lambda,
    int smooth, int sample, const int2 *__restrict__ xy, const float *__restrict__ coef,
    const float *__restrict__ rho, NodeRec *__restrict__ rec, unsigned *flags,
    const double *__restrict__ partials, double *__restrict__ finish_msd) {
  if ((int)blockIdx.x >= n_items) {
    msd_finish_group(pairs, n_pairs, partials, finish_msd, (int)blockIdx.x - n_items);
    return;
  }
  const NodeItem it = items[xcd_item((int)blockIdx.x, n_items)];
  const int i = it.begin + (int)threadIdx.x;
  if (i >= it.end) return;
  double2 ui;
  if (smooth) {
    const int q0 = r_ptr[i], q1 = r_ptr[i + 1];
    double sx = 0.0, sy = 0.0;
    constexpr int U = 4;
    for (int q = q0; q < q1; q += U) {
      int j[U];
#pragma unroll
      for (int k = 0; k < U; ++k) j[k] = q + k < q1 ? r_idx[q + k] : -1;
      double2 v[U];
#pragma unroll
      for (int k = 0; k < U; ++k) v[k] = j[k] >= 0 ? u0[j[k]] : make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < U; ++k) {
        sx += v[k].x;
        sy += v[k].y;
      }
    }
    const double2 a = u0[i];
    const double inv_m = 1.0 / (double)(q1 - q0);
    ui = make_double2((1.0 - lambda) * a.x + lambda * (sx * inv_m),
                      (1.0 - lambda) * a.y + lambda * (sy * inv_m));
    u[i] = ui;
  } else {
    ui = u[i];
  }
  if (sample) {
    const DevPair P = pairs[it.pair];
    const int2 v = xy[i];
    int cx, cy;
    float fx, fy;
    const bool okx = split_coord(v.x, ui.x - 0.5, cx, fx);
    const bool ok = split_coord(v.y, ui.y - 0.5, cy, fy) && okx;
    if (!ok) atomicOr(flags, kFlagNonFiniteNode);
    const float tv = spline_value(coef + P.pix_off, P.height, P.width, cx, fx, cy, fy);
    NodeRec R;
    R.px = (double)v.x + ui.x;
    R.py = (double)v.y + ui.y;
    R.t = (double)tv;
    R.r = (double)tv - (double)rho[i];
    rec[i] = R;
  }
}

// Update (one workgroup per node item): the gradient of the nodal samples t
// on the deformed mesh V + u, eq. 9 per triangle and the area-weighted mean of
// eq. 10 per node, then u0_i = u_i - tau (t_i - rho_i) g_i (eq. 5-6).  With
// cr the doubled signed area of a deformed triangle and
// S = sum_v t_v R(P_{v+2} - P_{v+1}), R(x, y) = (-y, x), the triangle's
// gradient is S / cr and its area |cr| / 2, so the node's mean is
// sum sign(cr) S / sum |cr| over its triangles (a zero-area triangle adds
// nothing; a node with none left gets g = 0).  FP64 throughout, from the
// node records the smoothing launch wrote.  Node i's triangles are given by
// their other two corners (j, k), in the triangle's cyclic order after i, in
// the list o_ptr / o_jk (global ids, triangle order): one record gather per
// other corner.  The workgroups after the node items warp the pixel grid by u
// into the MSD partials (when n_tiles > 0).
__global__ __launch_bounds__(256) void k_explicit_update(
    const NodeItem *__restrict__ items, int n_items, const DevPair *__restrict__ pairs,
    const double2 *__restrict__ u, const NodeRec *__restrict__ rec,
    const int4 *__restrict__ tri, const int32_t *__restrict__ o_ptr,
    const int2 *__restrict__ o_jk, double tau, double2 *__restrict__ u0, unsigned *flags,
    const TileItem *__restrict__ tiles, const int4 *__restrict__ tile_nodes,
    const int2 *__restrict__ tile_pbc, const uint8_t *__restrict__ tile_loc,
    const float *__restrict__ coef, const float *__restrict__ re,
    double *__restrict__ partials, int n_tiles) {
  if ((int)blockIdx.x >= n_items) {
    warp_tiles<1>(xcd_item((int)blockIdx.x - n_items, n_tiles), n_tiles, tiles, u, tile_nodes,
                  tile_pbc, tile_loc, coef, re, nullptr, partials, flags);
    return;
  }
  const NodeItem it = items[xcd_item((int)blockIdx.x, n_items)];
  const int i = it.begin + (int)threadIdx.x;
  if (i >= it.end) return;
  const int q0 = o_ptr[i], q1 = o_ptr[i + 1];
  const NodeRec Ri = rec[i];
  double nx = 0.0, ny = 0.0, den = 0.0;
  // U triangles per batch, their corner-record gathers issued together; the
  // sums run in list order
  constexpr int U = 2;
  for (int q = q0; q < q1; q += U) {
    int2 o[U];
#pragma unroll
    for (int k = 0; k < U; ++k) o[k] = q + k < q1 ? o_jk[q + k] : make_int2(i, i);
    double jx[U], jy[U], jt[U], kx[U], ky[U], kt[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const NodeRec Rj = rec[o[k].x], Rk = rec[o[k].y];
      jx[k] = Rj.px;
      jy[k] = Rj.py;
      jt[k] = Rj.t;
      kx[k] = Rk.px;
      ky[k] = Rk.py;
      kt[k] = Rk.t;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (q + k >= q1) continue;
      const double cr = (jx[k] - Ri.px) * (ky[k] - Ri.py) - (jy[k] - Ri.py) * (kx[k] - Ri.px);
      const double sx = -(Ri.t * (ky[k] - jy[k]) + jt[k] * (Ri.py - ky[k]) + kt[k] * (jy[k] - Ri.py));
      const double sy = Ri.t * (kx[k] - jx[k]) + jt[k] * (Ri.px - kx[k]) + kt[k] * (jx[k] - Ri.px);
      if (cr > 0.0) {
        nx += sx;
        ny += sy;
      } else if (cr < 0.0) {
        nx -= sx;
        ny -= sy;
      }
      den += fabs(cr);
    }
  }
  const double gx = den > 0.0 ? nx / den : 0.0;
  const double gy = den > 0.0 ? ny / den : 0.0;
  const double r = Ri.r;
  const double2 ui = u[i];
  u0[i] = make_double2(ui.x - tau * r * gx, ui.y - tau * r * gy);
}

hipError_t launch_explicit_smooth(const NodeItem *items, int n_items, const DevPair *pairs,
                                  int n_pairs, const double2 *u0, double2 *u,
                                  const int32_t *r_ptr, const int32_t *r_idx, double lambda,
                                  bool smooth, bool sample, const int2 *xy, const float *coef,
                                  const float *rho, NodeRec *rec, unsigned *flags,
                                  const double *partials, double *finish_msd, hipStream_t s) {
  const int groups = n_items + (finish_msd ? (n_pairs + 3) / 4 : 0);
  return launch(k_explicit_smooth, groups, kNodeChunk, 0, s, items, n_items, pairs, n_pairs, u0, u,
                r_ptr, r_idx, lambda, (int)smooth, (int)sample, xy, coef, rho, rec, flags,
                partials, finish_msd);
}

hipError_t launch_explicit_update(const NodeItem *items, int n_items, const DevPair *pairs,
                                  const double2 *u, const NodeRec *rec, const int4 *tri,
                                  const int32_t *o_ptr, const int2 *o_jk, double tau,
                                  double2 *u0, unsigned *flags, const TileItem *tiles, int n_tiles,
                                  const int4 *tile_nodes, const int2 *tile_pbc,
                                  const uint8_t *tile_loc, const float *coef, const float *re,
                                  double *partials, hipStream_t s) {
  return launch(k_explicit_update, n_items + n_tiles, kNodeChunk, 0, s, items, n_items, pairs, u,
                rec, tri, o_ptr, o_jk, tau, u0, flags, tiles, tile_nodes, tile_pbc, tile_loc, coef,
                re, partials, n_tiles);
}

// Copies the per-pair activity flags into every work descriptor (pairs,
// blocks, node items, tiles, apex items): a retired pair's work items return
// at once in every kernel.
__global__ void k_set_active(const int32_t *__restrict__ flags, DevPair *pairs, int n_pairs,
                             DevBlock *blocks, const int32_t *__restrict__ block_pair,
                             int n_blocks, NodeItem *items, int n_items, TileItem *tiles,
                             int n_tiles, ApexFwdItem *af, int n_af, ApexBwdItem *ab, int n_ab) {
  const int stride = (int)(gridDim.x * blockDim.x);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x;; k += stride) {
    bool any = false;
    if (k < n_pairs) pairs[k].active = flags[k], any = true;
    if (k < n_blocks) blocks[k].active = flags[block_pair[k]], any = true;
    if (k < n_items) items[k].active = flags[items[k].pair], any = true;
    if (k < n_tiles) tiles[k].active = flags[tiles[k].pair], any = true;
    if (k < n_af) af[k].active = flags[af[k].pair], any = true;
    if (k < n_ab) ab[k].active = flags[ab[k].pair], any = true;
    if (!any) break;
  }
}

hipError_t launch_set_active(const int32_t *flags, DevPair *pairs, int n_pairs, DevBlock *blocks,
                             const int32_t *block_pair, int n_blocks, NodeItem *items,
                             int n_items, TileItem *tiles, int n_tiles, ApexFwdItem *af, int n_af,
                             ApexBwdItem *ab, int n_ab, hipStream_t s) {
  const int n = std::max({n_pairs, n_blocks, n_items, n_tiles, n_af, n_ab});
  const int groups = std::min(std::max(1, (n + 255) / 256), 4096);
  return launch(k_set_active, groups, 256, 0, s, flags, pairs, n_pairs, blocks, block_pair,
                n_blocks, items, n_items, tiles, n_tiles, af, n_af, ab, n_ab);
}

hipError_t launch_to_solve_order(int n, const double2 *src, const int32_t *iperm, double2 *x,
                                 hipStream_t s) {
  return launch(k_to_solve_order, (n + 255) / 256, 256, 0, s, n, src, iperm, x);
}

hipError_t launch_from_solve_order(int n, const double2 *x, const int32_t *iperm, double2 *dst,
                                   hipStream_t s) {
  return launch(k_from_solve_order, (n + 255) / 256, 256, 0, s, n, x, iperm, dst);
}

hipError_t launch_h_from_solve_order(int n, const float2 *hs, const int32_t *iperm, float2 *h,
                                     hipStream_t s) {
  return launch(k_h_from_solve_order, (n + 255) / 256, 256, 0, s, n, hs, iperm, h);
}

}  // namespace mr
