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
//   k_warp_msd  pixel-tile-parallel: piecewise-linear displacement of each
//               pixel's triangle, template sample at the displaced pixel centre,
//               squared error, deterministic FP64 reduction to the MSD
// All node-, tile- and block-parallel launches cover every pair of a batch
// through work lists, so one launch per kernel family advances all pairs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>

#include "device.h"
#include "kernels.h"
#include "spline.h"

namespace mr {

// ---------------------------------------------------------------------------
// Pre-computation kernels (run once per pair, and for the template adjoint)
// ---------------------------------------------------------------------------

// Solve B c = s along each row (thread per row) with the Thomas algorithm;
// `cp` holds the eliminated super-diagonal, which depends only on the length.
template <typename Tin>
__global__ void k_prefilter_rows(const Tin *__restrict__ src, double *__restrict__ dst, int H,
                                 int W, const double *__restrict__ cp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= H) return;
  const Tin *s = src + (size_t)r * W;
  double *d = dst + (size_t)r * W;
  if (W == 1) {
    d[0] = (double)s[0];
    return;
  }
  const double off = 1.0 / 6.0;
  double prev = (double)s[0] / (5.0 / 6.0);
  d[0] = prev;
  for (int k = 1; k < W; ++k) {
    const double diag = (k == W - 1) ? 5.0 / 6.0 : 4.0 / 6.0;
    const double den = diag - off * cp[k - 1];
    prev = ((double)s[k] - off * prev) / den;
    d[k] = prev;
  }
  for (int k = W - 2; k >= 0; --k) {
    prev = d[k] - cp[k] * prev;
    d[k] = prev;
  }
}

// Column pass (thread per column, coalesced across threads), in place on
// `tmp`, writing the FP32 coefficients.
__global__ void k_prefilter_cols(double *__restrict__ tmp, float *__restrict__ out, int H, int W,
                                 const double *__restrict__ cp) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= W) return;
  double *d = tmp + col;
  if (H == 1) {
    out[col] = (float)d[0];
    return;
  }
  const double off = 1.0 / 6.0;
  double prev = d[0] / (5.0 / 6.0);
  d[0] = prev;
  for (int k = 1; k < H; ++k) {
    const double diag = (k == H - 1) ? 5.0 / 6.0 : 4.0 / 6.0;
    const double den = diag - off * cp[k - 1];
    prev = (d[(size_t)k * W] - off * prev) / den;
    d[(size_t)k * W] = prev;
  }
  out[(size_t)(H - 1) * W + col] = (float)prev;
  for (int k = H - 2; k >= 0; --k) {
    prev = d[(size_t)k * W] - cp[k] * prev;
    out[(size_t)k * W + col] = (float)prev;
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

// Second pass of the MSD, run by one workgroup: per pair, the tile partials
// summed in tile order by one wavefront (deterministic) over the pixel count.
__device__ __forceinline__ void msd_finish_block(const DevPair *__restrict__ pairs, int n_pairs,
                                                 const double *__restrict__ partials,
                                                 double *__restrict__ msd) {
  const int lane = threadIdx.x & 63;
  for (int p = threadIdx.x >> 6; p < n_pairs; p += blockDim.x >> 6) {
    const DevPair Q = pairs[p];
    double s = 0.0;
    for (int k = lane; k < Q.n_tiles; k += 64) s += partials[Q.tile_off + k];
    s = wave_sum(s);
    if (lane == 0) msd[p] = s / ((double)Q.height * (double)Q.width);
  }
}


// Node sampling.  When `finish_msd` is set, one extra workgroup (the last)
// completes the MSD of the previous warp instead (saves a launch per iteration).
__global__ __launch_bounds__(256) void k_sample(const NodeItem *__restrict__ items, int n_items,
                                                const DevPair *__restrict__ pairs, int n_pairs,
                                                const double2 *__restrict__ u,
                                                const int2 *__restrict__ xy,
                                                const float *__restrict__ coef,
                                                const float *__restrict__ rho,
                                                float2 *__restrict__ h, unsigned *flags,
                                                const double *__restrict__ partials,
                                                double *__restrict__ finish_msd) {
  if ((int)blockIdx.x == n_items) {
    msd_finish_block(pairs, n_pairs, partials, finish_msd);
    return;
  }
  const NodeItem it = items[blockIdx.x];
  const int i = it.begin + threadIdx.x;
  if (i >= it.end) return;
  const DevPair P = pairs[it.pair];
  const double2 ui = u[i];
  const int2 v = xy[i];
  int cx, cy;
  float fx, fy;
  const bool okx = split_coord(v.x, ui.x - 0.5, cx, fx);
  const bool ok = split_coord(v.y, ui.y - 0.5, cy, fy) && okx;
  if (!ok) atomicOr(flags, kFlagNonFiniteNode);
  float val, gx, gy;
  spline_value_grad(coef + P.pix_off, P.height, P.width, cx, fx, cy, fy, val, gx, gy);
  const float r = val - rho[i];
  h[i] = make_float2(r * gx, r * gy);
}

__global__ __launch_bounds__(256) void k_assemble(int n, const int32_t *__restrict__ mptr,
                                                  const int32_t *__restrict__ mcol,
                                                  const float *__restrict__ mwt,
                                                  const float2 *__restrict__ h,
                                                  const double2 *__restrict__ u,
                                                  const int32_t *__restrict__ iperm,
                                                  double2 *__restrict__ x, double tau) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float fx = 0.0f, fy = 0.0f;
  const int q1 = mptr[i + 1];
  for (int q = mptr[i]; q < q1; ++q) {
    const float w = mwt[q];
    const float2 hj = h[mcol[q]];
    fx += w * hj.x;
    fy += w * hj.y;
  }
  const double2 ui = u[i];
  x[iperm[i]] = make_double2(ui.x - tau * (double)fx, ui.y - tau * (double)fy);
}

// Copies n doubles from global memory to LDS with all of a thread's loads of
// a batch in flight before the first LDS store (predicated, no serial tail).
template <int NT>
__device__ __forceinline__ void stage_to_lds(double *__restrict__ dst, const double *__restrict__ src,
                                             int n) {
  constexpr int U = 16;
  for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      v[u] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      if (e < n) dst[e] = v[u];
    }
  }
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
//   y = D^-1 t              (dense inverse, column-major packed, staged in LDS)
// and then its slice of the block's own update entries
//   upd[k] = sum_j P[k][j] y_j   for panel rows k of the slice (P = L(below, block)).
// Slice 0 also writes y to x (in place).  Each phase spreads its sums over all
// threads and combines the partial sums in a fixed order (deterministic).
template <int NT>
__global__ __launch_bounds__(NT) void k_solve_fwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items,
    const int64_t *__restrict__ cptr, const int32_t *__restrict__ cidx,
    const double *__restrict__ dcol, const double *__restrict__ prow, double2 *x, double2 *upd) {
  extern __shared__ double smem[];
  const int2 it = items[blockIdx.x];
  const DevBlock B = blocks[it.x];
  const int b = B.r1 - B.r0;
  if (b == 0) return;
  const int tid = threadIdx.x;
  const int nd = b * (b + 1) / 2;
  const int k0 = it.y * B.rslice;
  const int kn = max(0, min(B.rslice, B.m - k0));
  double *D = smem;
  double *Ps = D + nd;
  double2 *t = reinterpret_cast<double2 *>(smem + (nd + kn * b + 1) / 2 * 2);
  double2 *yv = t + b;
  double2 *red = yv + b;
  stage_to_lds<NT>(D, dcol + B.doff, nd);
  stage_to_lds<NT>(Ps, prow + B.poff + (int64_t)k0 * b, kn * b);
  const int bp = pow2_at_least(b);
  const int np = NT / bp;          // threads per row
  const int r = tid & (bp - 1), part = tid / bp;
  // phase 1: gathers of the contributions, all loads of a thread in flight
  {
    double ax = 0.0, ay = 0.0;
    if (r < b) {
      const int row = B.r0 + r;
      const int64_t q1 = cptr[row + 1];
      constexpr int U = 8;
      for (int64_t q = cptr[row] + part; q < q1; q += (int64_t)np * U) {
        int idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t qq = q + (int64_t)u * np;
          idx[u] = qq < q1 ? cidx[qq] : -1;
        }
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = idx[u] >= 0 ? upd[idx[u]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ax += v[u].x;
          ay += v[u].y;
        }
      }
    }
    red[tid] = make_double2(ax, ay);
  }
  __syncthreads();
  if (part == 0 && r < b) {
    const double2 c = combine_parts(red, r, bp, np);
    const double2 bb = x[B.r0 + r];
    t[r] = make_double2(bb.x - c.x, bb.y - c.y);
  }
  __syncthreads();
  // phase 2: y_i = sum_{j <= i} D(i, j) t_j, j split over the row's threads
  {
    double ax = 0.0, ay = 0.0;
    if (r < b) {
#pragma unroll 8
      for (int j = part; j <= r; j += np) {
        // element (r, j) of the packed column-major lower triangle
        const double v = D[j * b - j * (j - 1) / 2 + (r - j)];
        ax += v * t[j].x;
        ay += v * t[j].y;
      }
    }
    red[tid] = make_double2(ax, ay);
  }
  __syncthreads();
  if (part == 0 && r < b) {
    const double2 y = combine_parts(red, r, bp, np);
    yv[r] = y;
    if (it.y == 0) x[B.r0 + r] = y;
  }
  __syncthreads();
  // phase 3: the slice's update entries, 4 partial sums per panel row
  constexpr int kParts = 4;
  constexpr int kRows = NT / kParts;
  for (int base = 0; base < kn; base += kRows) {
    const int kk = base + tid % kRows;
    const int pp = tid / kRows;
    double ax = 0.0, ay = 0.0;
    if (kk < kn) {
      const double *Pr = Ps + kk * b;
#pragma unroll 8
      for (int j = pp; j < b; j += kParts) {
        const double v = Pr[j];
        ax += v * yv[j].x;
        ay += v * yv[j].y;
      }
    }
    red[tid] = make_double2(ax, ay);
    __syncthreads();
    if (pp == 0 && kk < kn) upd[B.boff + k0 + kk] = combine_parts(red, tid, kRows, kParts);
    __syncthreads();
  }
}

// Backward solve, one level of the block tree.  Work item = (block, slice);
// a block is split into B.bslice workgroups, each covering a contiguous run of
// panel rows that it walks in LDS chunks of B.rslice rows, forming the partial
// sums s_j = sum_k P[k][j] z(below_k).  A block with one workgroup finishes at
// once; otherwise each workgroup writes its partials, and the last to arrive
// (device-scope counter) adds them in slice order.  The finishing workgroup
// forms t = y_block - s and z = D^-T t (row-major packed inverse in LDS),
// writes z in place and, when `out` is given, scatters it to natural order.
// The finisher resets the counter.
template <int NT>
__global__ __launch_bounds__(NT) void k_solve_bwd(
    const DevBlock *__restrict__ blocks, const int2 *__restrict__ items,
    const int32_t *__restrict__ below_idx, const double *__restrict__ drow,
    const double *__restrict__ prow, double2 *x, const int32_t *__restrict__ perm,
    double2 *__restrict__ out, double2 *partials, unsigned *counters) {
  extern __shared__ double smem[];
  __shared__ int last;
  const int2 it = items[blockIdx.x];
  const DevBlock B = blocks[it.x];
  const int b = B.r1 - B.r0;
  if (b == 0) return;
  const int tid = threadIdx.x;
  const int nd = b * (b + 1) / 2;
  const int rs = B.rslice;
  // panel rows [kb, ke) of this workgroup
  const int per = (B.m + B.bslice - 1) / B.bslice;
  const int kb = min(B.m, it.y * per), ke = min(B.m, kb + per);
  const int cap = min(rs, B.m);   // LDS chunk capacity in panel rows
  double *Ps = smem;
  double2 *zb = reinterpret_cast<double2 *>(smem + (cap * b + 1) / 2 * 2);
  double2 *red = zb + cap;
  double2 *t = red + NT;
  double *D = reinterpret_cast<double *>(t + b);
  if (B.bslice == 1) stage_to_lds<NT>(D, drow + B.doff, nd);
  const int bp = pow2_at_least(b);
  const int np = NT / bp;
  const int j = tid & (bp - 1), g = tid / bp;
  double ax = 0.0, ay = 0.0;
  for (int c0 = kb; c0 < ke; c0 += cap) {
    const int kn = min(cap, ke - c0);
    stage_to_lds<NT>(Ps, prow + B.poff + (int64_t)c0 * b, kn * b);
    for (int k = tid; k < kn; k += NT) zb[k] = x[below_idx[B.boff + c0 + k]];
    __syncthreads();
    if (j < b) {
#pragma unroll 8
      for (int k = g; k < kn; k += np) {
        const double v = Ps[k * b + j];
        ax += v * zb[k].x;
        ay += v * zb[k].y;
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
    stage_to_lds<NT>(D, drow + B.doff, nd);
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
    const double2 yy = x[B.r0 + j];
    t[j] = make_double2(yy.x - sum.x, yy.y - sum.y);
  }
  __syncthreads();
  // z_j = sum_{i >= j} D(i, j) t_i, i split over the column's threads
  {
    double zx = 0.0, zy = 0.0;
    if (j < b) {
#pragma unroll 8
      for (int i = j + g; i < b; i += np) {
        // element (i, j) of the packed row-major lower triangle
        const double v = D[i * (i + 1) / 2 + j];
        zx += v * t[i].x;
        zy += v * t[i].y;
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

// Apex, step 2: z = G t with G = L(apex,apex)^-T L(apex,apex)^-1 (dense,
// symmetric, row-major), i.e. both triangular solves of the apex at once; one
// wavefront per row (t staged in LDS); z goes to x and, when `out` is given,
// to natural node order.  Work item = (pair, first row).
__global__ __launch_bounds__(256) void k_apex_solve(const int2 *__restrict__ items,
                                                    const ApexDesc *__restrict__ apex,
                                                    const double *__restrict__ gram,
                                                    const int32_t *__restrict__ rows,
                                                    const double2 *__restrict__ tbuf, double2 *x,
                                                    const int32_t *__restrict__ perm,
                                                    double2 *__restrict__ out) {
  extern __shared__ double smem[];
  double2 *tl = reinterpret_cast<double2 *>(smem);
  const int2 it = items[blockIdx.x];
  const ApexDesc A = apex[it.x];
  for (int j = threadIdx.x; j < A.n; j += blockDim.x) tl[j] = tbuf[A.rows_off + j];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int i = it.y + (threadIdx.x >> 6);
  if (i >= A.n) return;
  const double *row = gram + A.inv_off + (int64_t)i * A.n;
  double ax = 0.0, ay = 0.0;
  constexpr int U = 8;
  for (int j0 = lane; j0 < A.n; j0 += 64 * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + 64 * u;
      v[u] = j < A.n ? row[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + 64 * u;
      if (j < A.n) {
        ax += v[u] * tl[j].x;
        ay += v[u] * tl[j].y;
      }
    }
  }
  ax = wave_sum(ax);
  ay = wave_sum(ay);
  if (lane == 0) {
    const double2 z = make_double2(ax, ay);
    const int r = rows[A.rows_off + i];
    x[r] = z;
    if (out) out[perm[r]] = z;
  }
}

// G = X^T X for the lower-triangular X = L(apex,apex)^-1 given as a packed
// row-major triangle (init / re-factorisation only): 16x16 output tiles,
// k-tiles staged in LDS.
__global__ __launch_bounds__(256) void k_apex_gram(int n, const double *__restrict__ xrow,
                                                   double *__restrict__ g) {
  __shared__ double Xi[16][17], Xj[16][17];
  const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
  const int r = threadIdx.x / 16, c = threadIdx.x % 16;
  double acc = 0.0;
  for (int k0 = max(ti, tj); k0 < n; k0 += 16) {
    const int k = k0 + r;
    // X[k][col] for col = ti + c and tj + c (zero above the diagonal)
    const int ci = ti + c, cj = tj + c;
    Xi[r][c] = (k < n && ci <= k) ? xrow[(int64_t)k * (k + 1) / 2 + ci] : 0.0;
    Xj[r][c] = (k < n && cj <= k) ? xrow[(int64_t)k * (k + 1) / 2 + cj] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += Xi[q][r] * Xj[q][c];
    __syncthreads();
  }
  if (ti + r < n && tj + c < n) g[(int64_t)(ti + r) * n + (tj + c)] = acc;
}

// Warp + MSD over kTile x kTile pixel tiles.  Each workgroup writes its FP64
// partial sum; the last workgroup to finish sums every pair's partials in a
// fixed order (deterministic) and resets the counter for the next launch.
__global__ __launch_bounds__(256) void k_warp_msd(
    const TileItem *__restrict__ tiles, const DevPair *__restrict__ pairs, int n_pairs,
    const double2 *__restrict__ u, const int2 *__restrict__ xy, const int4 *__restrict__ tri,
    const int32_t *__restrict__ t6, const float *__restrict__ coef, const float *__restrict__ re,
    float *__restrict__ warped, double *__restrict__ partials, unsigned *flags) {
  const TileItem it = tiles[blockIdx.x];
  const DevPair P = pairs[it.pair];
  const int i = it.y0 + (int)(threadIdx.x / kTile);
  const int j = it.x0 + (int)(threadIdx.x % kTile);
  double acc = 0.0;
  if (i < P.height && j < P.width) {
    const size_t pix = (size_t)P.pix_off + (size_t)i * P.width + j;
    const int4 nd = tri[P.tri_off + t6[pix]];
    const int2 a = xy[nd.x], b = xy[nd.y], c = xy[nd.z];
    // barycentric weights in doubled coordinates (exact integer cross products)
    const double px = 2.0 * j + 1.0, py = 2.0 * i + 1.0;
    const double ax = 2.0 * a.x - px, ay = 2.0 * a.y - py;
    const double bx = 2.0 * b.x - px, by = 2.0 * b.y - py;
    const double cx = 2.0 * c.x - px, cy = 2.0 * c.y - py;
    const double ca = bx * cy - by * cx, cb = cx * ay - cy * ax, cc = ax * by - ay * bx;
    const double inv = 1.0 / (ca + cb + cc);
    const double wa = ca * inv, wb = cb * inv, wc = cc * inv;
    const double2 ua = u[nd.x], ub = u[nd.y], uc = u[nd.z];
    const double dx = wa * ua.x + wb * ub.x + wc * uc.x;
    const double dy = wa * ua.y + wb * ub.y + wc * uc.y;
    int qx, qy;
    double fx, fy;
    const bool okx = split_coord_d(j, dx, qx, fx);
    const bool ok = split_coord_d(i, dy, qy, fy) && okx;
    if (!ok) atomicOr(flags, kFlagNonFinitePixel);
    const double w = spline_value_d(coef + P.pix_off, P.height, P.width, qx, fx, qy, fy);
    if (warped) warped[pix] = (float)w;
    const double e = w - (double)re[pix];
    acc = e * e;
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_msd_finish(const DevPair *__restrict__ pairs, int n_pairs,
                                                    const double *__restrict__ partials,
                                                    double *__restrict__ msd) {
  msd_finish_block(pairs, n_pairs, partials, msd);
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

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------

hipError_t launch_prefilter(const float *src_f, const double *src_d, double *tmp, float *out,
                            int H, int W, const double *cp_w, const double *cp_h,
                            hipStream_t s) {
  const int tb = 64;
  if (src_f)
    k_prefilter_rows<float><<<(H + tb - 1) / tb, tb, 0, s>>>(src_f, tmp, H, W, cp_w);
  else
    k_prefilter_rows<double><<<(H + tb - 1) / tb, tb, 0, s>>>(src_d, tmp, H, W, cp_w);
  k_prefilter_cols<<<(W + tb - 1) / tb, tb, 0, s>>>(tmp, out, H, W, cp_h);
  return hipGetLastError();
}

hipError_t launch_sample_rho(const NodeItem *items, int n_items, const DevPair *pairs,
                             const int2 *xy, const float *coef_re, float *rho, hipStream_t s) {
  k_sample_rho<<<n_items, kNodeChunk, 0, s>>>(items, pairs, xy, coef_re, rho);
  return hipGetLastError();
}

hipError_t launch_sample(const NodeItem *items, int n_items, const DevPair *pairs, int n_pairs,
                         const double2 *u, const int2 *xy, const float *coef, const float *rho,
                         float2 *h, unsigned *flags, const double *partials, double *finish_msd,
                         hipStream_t s) {
  k_sample<<<n_items + (finish_msd ? 1 : 0), kNodeChunk, 0, s>>>(
      items, n_items, pairs, n_pairs, u, xy, coef, rho, h, flags, partials, finish_msd);
  return hipGetLastError();
}

hipError_t launch_assemble(int n, const int32_t *mptr, const int32_t *mcol, const float *mwt,
                           const float2 *h, const double2 *u, const int32_t *iperm, double2 *x,
                           double tau, hipStream_t s) {
  k_assemble<<<(n + 255) / 256, 256, 0, s>>>(n, mptr, mcol, mwt, h, u, iperm, x, tau);
  return hipGetLastError();
}

hipError_t launch_solve_fwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int64_t *cptr, const int32_t *cidx,
                                  const double *dcol, const double *prow, double2 *x,
                                  double2 *upd, hipStream_t s) {
  switch (nt) {
    case 64:
      k_solve_fwd<64><<<count, 64, lds_bytes, s>>>(blocks, items, cptr, cidx, dcol, prow, x, upd);
      break;
    case 128:
      k_solve_fwd<128><<<count, 128, lds_bytes, s>>>(blocks, items, cptr, cidx, dcol, prow, x, upd);
      break;
    default:
      k_solve_fwd<256><<<count, 256, lds_bytes, s>>>(blocks, items, cptr, cidx, dcol, prow, x, upd);
  }
  return hipGetLastError();
}

hipError_t launch_solve_bwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int32_t *below_idx,
                                  const double *drow, const double *prow, double2 *x,
                                  const int32_t *perm, double2 *out, double2 *partials,
                                  unsigned *counters, hipStream_t s) {
  switch (nt) {
    case 64:
      k_solve_bwd<64><<<count, 64, lds_bytes, s>>>(blocks, items, below_idx, drow, prow, x, perm,
                                                   out, partials, counters);
      break;
    case 128:
      k_solve_bwd<128><<<count, 128, lds_bytes, s>>>(blocks, items, below_idx, drow, prow, x, perm,
                                                     out, partials, counters);
      break;
    default:
      k_solve_bwd<256><<<count, 256, lds_bytes, s>>>(blocks, items, below_idx, drow, prow, x, perm,
                                                     out, partials, counters);
  }
  return hipGetLastError();
}

hipError_t launch_apex_solve(int n_rows, const int32_t *rows, const int64_t *acptr,
                             const int32_t *acidx, const double2 *upd, double2 *x, double2 *tbuf,
                             const int2 *items, int n_items, int lds_bytes, const ApexDesc *apex,
                             const double *gram, const int32_t *perm, double2 *out,
                             hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  k_apex_rhs<<<(n_rows + 255) / 256, 256, 0, s>>>(n_rows, rows, acptr, acidx, upd, x, tbuf);
  k_apex_solve<<<n_items, 64 * kApexRowsPerGroup, lds_bytes, s>>>(items, apex, gram, rows, tbuf, x,
                                                                  perm, out);
  return hipGetLastError();
}

hipError_t launch_apex_gram(int n, const double *xrow, double *g, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int t = (n + 15) / 16;
  k_apex_gram<<<dim3(t, t), 256, 0, s>>>(n, xrow, g);
  return hipGetLastError();
}

hipError_t launch_warp_partials(const TileItem *tiles, int n_tiles, const DevPair *pairs,
                                int n_pairs, const double2 *u, const int2 *xy, const int4 *tri,
                                const int32_t *t6, const float *coef, const float *re,
                                float *warped, double *partials, unsigned *flags, hipStream_t s) {
  k_warp_msd<<<n_tiles, kTile * kTile, 0, s>>>(tiles, pairs, n_pairs, u, xy, tri, t6, coef, re,
                                               warped, partials, flags);
  return hipGetLastError();
}

hipError_t launch_msd_finish(const DevPair *pairs, int n_pairs, const double *partials,
                             double *msd, hipStream_t s) {
  k_msd_finish<<<1, 256, 0, s>>>(pairs, n_pairs, partials, msd);
  return hipGetLastError();
}

hipError_t launch_to_solve_order(int n, const double2 *src, const int32_t *iperm, double2 *x,
                                 hipStream_t s) {
  k_to_solve_order<<<(n + 255) / 256, 256, 0, s>>>(n, src, iperm, x);
  return hipGetLastError();
}

hipError_t launch_from_solve_order(int n, const double2 *x, const int32_t *iperm, double2 *dst,
                                   hipStream_t s) {
  k_from_solve_order<<<(n + 255) / 256, 256, 0, s>>>(n, x, iperm, dst);
  return hipGetLastError();
}

}  // namespace mr
