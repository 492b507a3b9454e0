// Reverse mode of the unrolled registration: gradient of
//   L = sum_p g_msd[p] * MSD_p(u^N)
// with respect to the initial displacements, each pair's alpha and the
// template intensities (the objective of eq. 1 unrolled by Algorithm 1 in its
// semi-implicit form).  With S = I + tau alpha K, u^{k+1} = S^-1 b^k and
// b^k = u^k - tau (M h(u^k)) / m, h_i = r_i g_i:
//
//   warp:   lambda^N_v += (2 g/P) e_p w_v(p) grad s(q_p),  cbar += (2 g/P) e_p beta(x) beta(y)
//   step k: mu = S^-1 lambda^{k+1}                        (same factor, same kernels)
//           gbar_alpha -= tau mu^T K u^{k+1}
//           eta = -tau M (mu / m)                        (-tau mu in the nodal mode)
//           lambda^k_i = mu_i + (g_i . eta_i) g_i + r_i H_i eta_i
//           cbar += (eta_i . g_i) beta beta + r_i (eta_x beta' beta + eta_y beta beta')
//   end:    gbar_Te = B^-1 cbar                           (the prefilter is symmetric)
//
// The iterates are recomputed from checkpoints every `ckpt_every` iterations
// (each segment's last iterate is the next checkpoint and is not recomputed)
// with the forward kernels, so they equal the forward pass bit for bit.  The
// checkpoints come from a forward pass that writes them as it goes (the
// caller's, or one the reverse call runs itself).  The
// adjoint arithmetic is FP64; lambda^N is summed in a fixed order (per tile
// entry, then per node), the scatter into cbar uses FP64 atomic adds (its
// summation order is not fixed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "../../include/meshreg.h"
#include "ctx.h"
#include "kernels.h"
#include "launch.h"
#include "spline.h"

namespace mr {

// FP64 spline value and gradient with FP32 coefficients.
__device__ __forceinline__ void spline_vg_d(const float *__restrict__ c, int H, int W, int cx,
                                            double fx, int cy, double fy, double &val, double &gx,
                                            double &gy) {
  double wx[4], dx[4], wy[4], dy[4];
  bs_weights_d(fx, wx);
  bs_deriv_d(fx, dx);
  bs_weights_d(fy, wy);
  bs_deriv_d(fy, dy);
  float t[4][4];
  load_taps(c, H, W, cx, cy, t);
  val = gx = gy = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double rv = 0.0, rd = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const double cv = (double)t[m][n];
      rv += cv * wx[n];
      rd += cv * dx[n];
    }
    val += wy[m] * rv;
    gx += wy[m] * rd;
    gy += dy[m] * rv;
  }
}

// Coefficient-adjoint contributions of a wavefront's nodes: node (lane) adds
// cv beta(x) beta(y) + cgx beta'(x) beta(y) + cgy beta(x) beta'(y) at its 16
// taps (cell cx, cy; fractions fx, fy) into cbar (one pair's [H][W] FP64
// array).  When the taps of the wavefront's nodes fit a box of at most
// kAdjBox coefficients, they are first summed in `box` (this wavefront's LDS,
// FP64 LDS atomics) and the box is then added to cbar with one global atomic
// per touched coefficient; otherwise each tap is a global atomic.  Every
// wavefront of the workgroup must call this once (it holds two workgroup
// barriers); lanes with `on` false add nothing.
constexpr int kAdjBox = 512;
__device__ __forceinline__ void scatter_taps_wave(double *__restrict__ cbar, int H, int W, bool on,
                                                  int cx, double fx, int cy, double fy, double cv,
                                                  double cgx, double cgy, double *box) {
  const int lane = (int)threadIdx.x & 63;
  int mnx = on ? cx : INT_MAX, mxx = on ? cx : INT_MIN;
  int mny = on ? cy : INT_MAX, mxy = on ? cy : INT_MIN;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mnx = min(mnx, __shfl_xor(mnx, off));
    mxx = max(mxx, __shfl_xor(mxx, off));
    mny = min(mny, __shfl_xor(mny, off));
    mxy = max(mxy, __shfl_xor(mxy, off));
  }
  const bool any = mxx >= mnx;                      // uniform in the wavefront
  const int bx0 = mnx - 1, by0 = mny - 1;
  const int bw = any ? mxx - mnx + 4 : 0, bh = any ? mxy - mny + 4 : 0;
  const bool staged = any && bw <= 64 && bw * bh <= kAdjBox;
  if (staged)
    for (int e = lane; e < bw * bh; e += 64) box[e] = 0.0;
  __syncthreads();
  double wx[4], dx[4], wy[4], dy[4];
  bs_weights_d(fx, wx);
  bs_deriv_d(fx, dx);
  bs_weights_d(fy, wy);
  bs_deriv_d(fy, dy);
  if (on && staged) {
    double *b = box + (cy - 1 - by0) * bw + (cx - 1 - bx0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
        atomicAdd(b + m * bw + n, cv * wy[m] * wx[n] + cgx * wy[m] * dx[n] + cgy * dy[m] * wx[n]);
  } else if (on) {
    unsigned col[4], row[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      col[k] = (unsigned)fold_index(cx - 1 + k, W);
      row[k] = (unsigned)fold_index(cy - 1 + k, H) * (unsigned)W;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
        unsafeAtomicAdd(cbar + (row[m] + col[n]),
                        cv * wy[m] * wx[n] + cgx * wy[m] * dx[n] + cgy * dy[m] * wx[n]);
  }
  __syncthreads();
  if (staged) {
    // box rows, 64 / (32 or 64) rows per pass
    const int per = bw <= 32 ? 32 : 64, rpp = 64 / per, c = lane % per;
    for (int r = lane / per; r < bh; r += rpp)
      if (c < bw) {
        const double v = box[r * bw + c];
        if (v != 0.0)
          unsafeAtomicAdd(cbar + ((unsigned)fold_index(by0 + r, H) * (unsigned)W +
                                  (unsigned)fold_index(bx0 + c, W)),
                          v);
      }
  }
}

// Warp adjoint (and the forward MSD partials of the same pixels), one 16 x 16
// tile per workgroup: the coefficient adjoint of each pixel's sample
// (pre-summed per wavefront in LDS before the global atomics,
// scatter_taps_wave) and, for lambda^N, each pixel's contributions to the
// three corners of its triangle summed per entry of the tile's triangle list
// in pixel order (thread e adds the pixels whose slot is e) into
// lam_part[3 (ent_off + e) + corner]; k_lambda_gather then adds each node's
// entries in a fixed order, so lambda^N does not depend on the order in
// which workgroups run.
__global__ __launch_bounds__(256) void k_warp_adjoint(
    const TileItem *__restrict__ tiles, const DevPair *__restrict__ pairs,
    const double2 *__restrict__ u, const int2 *__restrict__ xy, const int4 *__restrict__ tri,
    const int32_t *__restrict__ t6, const uint8_t *__restrict__ tile_loc,
    const float *__restrict__ coef, const float *__restrict__ re,
    const double *__restrict__ g_msd, double2 *__restrict__ lam_part, double *cbar,
    double *__restrict__ partials) {
  constexpr int kPix = kTile * kTile;
  __shared__ double box[4][kAdjBox];
  __shared__ double2 cont[3][kPix];
  __shared__ uint8_t slot[kPix];
  const int tid = (int)threadIdx.x, wave = tid >> 6;
  const TileItem it = tiles[blockIdx.x];
  const DevPair P = pairs[it.pair];
  const int i = it.y0 + tid / kTile;
  const int j = it.x0 + tid % kTile;
  const bool in = i < P.height && j < P.width;
  const int I = min(i, P.height - 1), J = min(j, P.width - 1);
  const size_t pix = (size_t)P.pix_off + (size_t)I * P.width + J;
  const int4 nd = tri[P.tri_off + t6[pix]];
  const int2 a = xy[nd.x], b = xy[nd.y], c = xy[nd.z];
  const double px = 2.0 * J + 1.0, py = 2.0 * I + 1.0;
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
  split_coord_d(J, dx, qx, fx);
  split_coord_d(I, dy, qy, fy);
  const float *cp = coef + P.pix_off;
  double val, gx, gy;
  spline_vg_d(cp, P.height, P.width, qx, fx, qy, fy, val, gx, gy);
  const double e = val - (double)re[pix];
  const double acc = in ? e * e : 0.0;
  const double s = in ? 2.0 * g_msd[it.pair] / ((double)P.height * (double)P.width) * e : 0.0;
  // the pixel's entry in the tile's triangle list (the triangle of T6 above)
  slot[tid] = tile_loc[(size_t)blockIdx.x * kPix + tid];
  cont[0][tid] = in ? make_double2(s * wa * gx, s * wa * gy) : make_double2(0.0, 0.0);
  cont[1][tid] = in ? make_double2(s * wb * gx, s * wb * gy) : make_double2(0.0, 0.0);
  cont[2][tid] = in ? make_double2(s * wc * gx, s * wc * gy) : make_double2(0.0, 0.0);
  // (its barriers also make slot and cont visible to the whole workgroup)
  scatter_taps_wave(cbar + P.pix_off, P.height, P.width, in, qx, fx, qy, fy, s, 0.0, 0.0,
                    box[wave]);
  if (tid < it.n_ent) {
    double2 sa = make_double2(0.0, 0.0), sb = sa, sc = sa;
    for (int q = 0; q < kPix; ++q)
      if (slot[q] == tid) {
        sa.x += cont[0][q].x;
        sa.y += cont[0][q].y;
        sb.x += cont[1][q].x;
        sb.y += cont[1][q].y;
        sc.x += cont[2][q].x;
        sc.y += cont[2][q].y;
      }
    double2 *o = lam_part + 3 * ((int64_t)it.ent_off + tid);
    o[0] = sa;
    o[1] = sb;
    o[2] = sc;
  }
  __shared__ double red[4];
  const double sum = wave_sum(acc);
  if ((tid & 63) == 0) red[wave] = sum;
  __syncthreads();
  if (tid == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// lambda^N of node v: its (tile entry, corner) sums lam_part[lidx[q]],
// q = lptr[v] .. lptr[v + 1] - 1, added in that (ascending) order.
__global__ __launch_bounds__(256) void k_lambda_gather(int n, const int32_t *__restrict__ lptr,
                                                       const int32_t *__restrict__ lidx,
                                                       const double2 *__restrict__ lam_part,
                                                       double2 *__restrict__ lam) {
  const int v = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (v >= n) return;
  double sx = 0.0, sy = 0.0;
  for (int q = lptr[v]; q < lptr[v + 1]; ++q) {
    const double2 c = lam_part[lidx[q]];
    sx += c.x;
    sy += c.y;
  }
  lam[v] = make_double2(sx, sy);
}

// One reverse step per node i, given mu = S^-1 lambda^{k+1}:
//   the alpha partial (K u^{k+1})_i . mu_i (summed per node item in a fixed order),
//   eta_i = -tau (M (mu / m))_i (-tau mu_i in the nodal mode),
//   lambda^k_i = mu_i + (g_i . eta_i) g_i + r_i H_i eta_i at u^k, written in natural
//   and in solve order (the right-hand side of the next step's solve),
//   and the coefficient adjoint of the force density scattered into cbar.
// The stiffness / mass row is read in batches of 4 entries (indices and
// weights, then the gathers of u^{k+1} and mu), the template taps at u^k in
// the same batch as the row's first indices.
__global__ __launch_bounds__(256) void k_adjoint_step(
    const NodeItem *__restrict__ items, const DevPair *__restrict__ pairs,
    const int32_t *__restrict__ kptr, const int32_t *__restrict__ kcol,
    const double *__restrict__ kval, const double *__restrict__ mwt_t,
    const double2 *__restrict__ mu, const double2 *__restrict__ u1, const double2 *__restrict__ u,
    const int2 *__restrict__ xy, const float *__restrict__ coef, const float *__restrict__ rho,
    const int32_t *__restrict__ iperm, double2 *__restrict__ lam, double2 *__restrict__ lam_solve,
    double *cbar, double *__restrict__ alpha_part, double tau, int nodal) {
  __shared__ double box[4][kAdjBox];
  const NodeItem it = items[blockIdx.x];
  const int i = it.begin + threadIdx.x;
  const bool on = i < it.end;
  const int ii = on ? i : it.begin;               // idle lanes read a valid node
  const DevPair P = pairs[it.pair];
  const double2 ui = u[ii];
  const int2 v = xy[ii];
  const double2 mi = mu[ii];
  const float rh = rho[ii];
  const int q0 = kptr[ii], q1 = kptr[ii + 1];
  int cx, cy;
  double fx, fy;
  split_coord_d(v.x, ui.x - 0.5, cx, fx);
  split_coord_d(v.y, ui.y - 0.5, cy, fy);
  const float *c = coef + P.pix_off;
  float t[4][4];
  load_taps(c, P.height, P.width, cx, cy, t);
  double kx = 0.0, ky = 0.0, ex = 0.0, ey = 0.0;
  constexpr int U = 4;
  for (int q = q0; q < q1; q += U) {
    int jn[U];
    double kv[U], mw[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const bool in = q + k < q1;
      jn[k] = in ? kcol[q + k] : ii;
      kv[k] = in ? kval[q + k] : 0.0;
      mw[k] = (in && !nodal) ? mwt_t[q + k] : 0.0;
    }
    double2 uj[U], mj[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      uj[k] = u1[jn[k]];
      mj[k] = nodal ? make_double2(0.0, 0.0) : mu[jn[k]];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      kx += kv[k] * uj[k].x;
      ky += kv[k] * uj[k].y;
      ex += mw[k] * mj[k].x;
      ey += mw[k] * mj[k].y;
    }
  }
  double da = on ? mi.x * kx + mi.y * ky : 0.0;
  const double2 et = nodal ? make_double2(-tau * mi.x, -tau * mi.y)
                           : make_double2(-tau * ex, -tau * ey);
  // spline value, gradient and Hessian of the template at u^k
  double wx[4], dx[4], exw[4], wy[4], dy[4], eyw[4];
  bs_weights_d(fx, wx);
  bs_deriv_d(fx, dx);
  bs_deriv2_d(fx, exw);
  bs_weights_d(fy, wy);
  bs_deriv_d(fy, dy);
  bs_deriv2_d(fy, eyw);
  double val = 0.0, gx = 0.0, gy = 0.0, hxx = 0.0, hxy = 0.0, hyy = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double rv = 0.0, rd = 0.0, re2 = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const double cv = (double)t[m][n];
      rv += cv * wx[n];
      rd += cv * dx[n];
      re2 += cv * exw[n];
    }
    val += wy[m] * rv;
    gx += wy[m] * rd;
    gy += dy[m] * rv;
    hxx += wy[m] * re2;
    hxy += dy[m] * rd;
    hyy += eyw[m] * rv;
  }
  const double r = val - (double)rh;
  const double ge = gx * et.x + gy * et.y;
  if (on) {
    const double2 l = make_double2(mi.x + ge * gx + r * (hxx * et.x + hxy * et.y),
                                   mi.y + ge * gy + r * (hxy * et.x + hyy * et.y));
    lam[i] = l;
    lam_solve[iperm[i]] = l;
  }
  scatter_taps_wave(cbar + P.pix_off, P.height, P.width, on, cx, fx, cy, fy, ge, r * et.x,
                    r * et.y, box[threadIdx.x >> 6]);
  __shared__ double red[4];
  da = wave_sum(da);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = da;
  __syncthreads();
  if (threadIdx.x == 0) alpha_part[blockIdx.x] += -tau * ((red[0] + red[1]) + (red[2] + red[3]));
}

// Per pair: the alpha partials of its node items summed in item order.
__global__ void k_alpha_finish(const DevPair *__restrict__ pairs, int n_pairs,
                               const double *__restrict__ alpha_part, double *__restrict__ g_alpha) {
  const int lane = threadIdx.x & 63;
  for (int p = threadIdx.x >> 6; p < n_pairs; p += blockDim.x >> 6) {
    const DevPair Q = pairs[p];
    const double s = wave_sum(lane_strided_sum(alpha_part + Q.item_off, Q.n_items, lane));
    if (lane == 0) g_alpha[p] = s;
  }
}

}  // namespace mr

using namespace mr;

static int bfail(int code, const std::string &msg) { return mr_set_error(code, msg); }

#define HIP_OK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return bfail(MR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Buffers of the reverse sweep (allocated on first use, grown when needed).
int mr_ctx::reserve_adjoint(int32_t n_iter, int32_t ckpt_every, hipStream_t s) {
  const int64_t N = n_nodes;
  // recomputed iterates strictly inside a segment: at most min(ckpt_every, n_iter) - 1
  const int64_t seg_slots = std::max(0, std::min(ckpt_every, n_iter) - 1);
  if (seg_slots > 0 && (int64_t)d_seg.count < seg_slots * N) HIP_OK(d_seg.alloc((size_t)(seg_slots * N)));
  if ((int64_t)d_lam.count < N) {
    HIP_OK(d_lam.alloc(N));
    HIP_OK(d_lam_s.alloc(N));
    HIP_OK(d_mu.alloc(N));
  }
  if ((int64_t)d_cbar.count < n_pix) HIP_OK(d_cbar.alloc(n_pix));
  if (d_lam_part.count < 3 * d_tile_nodes.count) HIP_OK(d_lam_part.alloc(3 * d_tile_nodes.count));
  if ((int)d_alpha_part.count < n_node_items) HIP_OK(d_alpha_part.alloc(n_node_items));
  if (!d_mwt_t.ptr) {                         // uploaded last: present after a complete upload
    const int rc = upload_adjoint_operators(s);
    if (rc) return rc;
  }
  return MR_OK;
}

// n_iter iterations from ck[0] (which holds u^0) writing the checkpoints
// ck[q] = u^{q ckpt_every} for 0 < q < n_seg and ck[n_seg] = u^N; the solve
// writes u in natural order only at those iterations (the iteration state
// stays in the solve vector in between).
hipError_t mr_ctx::forward_ckpt(double2 *ck, int32_t n_iter, int32_t ckpt_every, hipStream_t s) {
  const int n_seg = (n_iter + ckpt_every - 1) / ckpt_every;
  const size_t N = (size_t)n_nodes;
  hipError_t e = hipSuccess;
  if (n_iter > 0) e = launch_to_solve_order((int)N, ck, d_iperm.ptr, d_x.ptr, s);
  double *pending = nullptr;
  for (int k = 0; k < n_iter && e == hipSuccess; ++k) {
    const bool last = k + 1 == n_iter, boundary = last || (k + 1) % ckpt_every == 0;
    double2 *dst = ck + (last ? (size_t)n_seg : (size_t)((k + 1) / ckpt_every)) * N;
    e = iterate(dst, nullptr, &pending, true, boundary, s);
  }
  return e;
}

// Reverse sweep from the checkpoints ck (as forward_ckpt leaves them).
int mr_ctx::reverse(const double2 *ck, int32_t n_iter, int32_t ckpt_every, const double *g_msd,
                    double *g_u0, double *g_alpha, float *g_te, double *msd, hipStream_t s) {
  const int64_t N = n_nodes;
  const int n_seg = (n_iter + ckpt_every - 1) / ckpt_every;
  const size_t nb = sizeof(double2) * (size_t)N;
  int rc = reserve_adjoint(n_iter, ckpt_every, s);
  if (rc) return rc;
  double2 *seg = d_seg.ptr;
  auto ckpt = [&](int q) { return ck + (size_t)q * N; };
  // warp adjoint at u^N: lambda^N per (tile entry, corner), then per node
  HIP_OK(hipMemsetAsync(d_cbar.ptr, 0, sizeof(double) * n_pix, s));
  HIP_OK(hipMemsetAsync(d_alpha_part.ptr, 0, sizeof(double) * n_node_items, s));
  timed_begin(MR_KF_WARP, s);
  hipError_t ew = launch(k_warp_adjoint, n_tiles, kTile * kTile, 0, s, d_tiles.ptr, d_pairs.ptr,
                         ckpt(n_seg), d_xy.ptr, d_tri.ptr, d_t6.ptr, d_tile_loc.ptr, d_coef.ptr,
                         d_re.ptr, g_msd, d_lam_part.ptr, d_cbar.ptr, d_partials.ptr);
  if (ew == hipSuccess && N > 0)
    ew = launch(k_lambda_gather, (int)((N + 255) / 256), 256, 0, s, (int)N, d_lam_ptr.ptr,
                d_lam_idx.ptr, (const double2 *)d_lam_part.ptr, d_lam.ptr);
  timed_end(s);          // before any return, so no timer stays attached to the thread
  HIP_OK(ew);
  if (msd) HIP_OK(launch_msd_finish(d_pairs.ptr, n_pairs, d_partials.ptr, msd, s));
  // lambda^N in solve order (its own buffer: the recomputed iterations use x)
  // for the first reverse solve; every reverse step writes the next one there
  if (n_iter > 0) HIP_OK(launch_to_solve_order((int)N, d_lam.ptr, d_iperm.ptr, d_lam_s.ptr, s));
  // reverse sweep, one checkpoint segment at a time: u^{k0} and u^{k1} are
  // checkpoints, the iterates between are recomputed into seg[0 ..]
  double *pending = nullptr;
  for (int sg = n_seg - 1; sg >= 0; --sg) {
    const int k0 = sg * ckpt_every, k1 = std::min(n_iter, k0 + ckpt_every);
    auto iterate_at = [&](int k) -> const double2 * {
      return k == k0 ? ckpt(sg) : k == k1 ? ckpt(sg + 1) : seg + (size_t)(k - k0 - 1) * N;
    };
    for (int k = k0; k + 1 < k1; ++k) {
      double2 *dst = seg + (size_t)(k - k0) * N;
      // x still holds u^k from the previous recomputed iteration, except at
      // the segment's start (a checkpoint): permute it in there
      if (k == k0) HIP_OK(launch_to_solve_order((int)N, ckpt(sg), d_iperm.ptr, d_x.ptr, s));
      HIP_OK(iterate(dst, nullptr, &pending, true, true, s));
    }
    for (int k = k1 - 1; k >= k0; --k) {
      // mu = S^-1 lambda^{k+1} (right-hand side in solve order, consumed in place)
      HIP_OK(solve(d_lam_s.ptr, d_mu.ptr, s, nullptr));
      timed_begin(MR_KF_ASSEMBLE, s);
      const hipError_t ea =
          launch(k_adjoint_step, n_node_items, kNodeChunk, 0, s, d_node_items.ptr, d_pairs.ptr,
                 d_kptr.ptr, d_kcol.ptr, d_kval.ptr, d_mwt_t.ptr, (const double2 *)d_mu.ptr,
                 iterate_at(k + 1), iterate_at(k), d_xy.ptr, d_coef.ptr, d_rho.ptr, d_iperm.ptr,
                 d_lam.ptr, d_lam_s.ptr, d_cbar.ptr, d_alpha_part.ptr, params.tau,
                 params.force_mode == MR_FORCE_NODAL ? 1 : 0);
      timed_end(s);
      HIP_OK(ea);
    }
  }
  if (g_u0) HIP_OK(hipMemcpyAsync(g_u0, d_lam.ptr, nb, hipMemcpyDeviceToDevice, s));
  if (g_alpha) {
    HIP_OK(launch(k_alpha_finish, 1, 256, 0, s, d_pairs.ptr, n_pairs, d_alpha_part.ptr,
                  g_alpha));
  }
  // gbar_Te = B^-1 cbar for every pair in two launches (cbar is overwritten)
  if (g_te)
    HIP_OK(launch_prefilter_all(d_pref_rows.ptr, (int)d_pref_rows.count, d_pref_cols.ptr,
                                (int)d_pref_cols.count, d_pairs.ptr, d_cbar.ptr, g_te,
                                d_thomas.ptr, s));
  post_flags(s);
  return MR_OK;
}

static bool args_ok(int32_t n_iter, int32_t ckpt_every) { return n_iter >= 0 && ckpt_every >= 1; }

int mr_ctx::backward(const double *u0, int32_t n_iter, int32_t ckpt_every, const double *g_msd,
                     double *g_u0, double *g_alpha, float *g_te, double *msd, hipStream_t s) {
  if (!u0 || !g_msd || !args_ok(n_iter, ckpt_every) || ((uintptr_t)u0 & 15) ||
      (g_u0 && ((uintptr_t)g_u0 & 15)))
    return bfail(MR_EINVAL, "backward: need aligned u0, g_msd, n_iter >= 0, ckpt_every >= 1");
  int rc = check_flags();
  if (rc) return rc;
  const int64_t N = n_nodes;
  const int n_ck = (n_iter + ckpt_every - 1) / ckpt_every + 1;
  if ((int64_t)d_ck.count < (int64_t)n_ck * N) HIP_OK(d_ck.alloc((size_t)n_ck * N));
  HIP_OK(hipMemcpyAsync(d_ck.ptr, u0, sizeof(double2) * (size_t)N, hipMemcpyDeviceToDevice, s));
  HIP_OK(forward_ckpt(d_ck.ptr, n_iter, ckpt_every, s));
  return reverse(d_ck.ptr, n_iter, ckpt_every, g_msd, g_u0, g_alpha, g_te, msd, s);
}

int mr_ctx::forward_with_ckpt(double *u, int32_t n_iter, int32_t ckpt_every, double *ckpt,
                              double *msd, hipStream_t s) {
  if (!u || !ckpt || !args_ok(n_iter, ckpt_every) || ((uintptr_t)u & 15) || ((uintptr_t)ckpt & 15))
    return bfail(MR_EINVAL, "forward_ckpt: need aligned u and ckpt, n_iter >= 0, ckpt_every >= 1");
  int rc = check_flags();
  if (rc) return rc;
  const size_t nb = sizeof(double2) * (size_t)n_nodes;
  const int n_seg = (n_iter + ckpt_every - 1) / ckpt_every;
  double2 *ck = reinterpret_cast<double2 *>(ckpt);
  HIP_OK(hipMemcpyAsync(ck, u, nb, hipMemcpyDeviceToDevice, s));
  HIP_OK(forward_ckpt(ck, n_iter, ckpt_every, s));
  if (n_seg > 0) HIP_OK(hipMemcpyAsync(u, ck + (size_t)n_seg * n_nodes, nb, hipMemcpyDeviceToDevice, s));
  if (msd) HIP_OK(warp(ck + (size_t)n_seg * n_nodes, msd, nullptr, s));
  post_flags(s);
  return MR_OK;
}

int mr_ctx::backward_from_ckpt(const double *ckpt, int32_t n_iter, int32_t ckpt_every,
                               const double *g_msd, double *g_u0, double *g_alpha, float *g_te,
                               double *msd, hipStream_t s) {
  if (!ckpt || !g_msd || !args_ok(n_iter, ckpt_every) || ((uintptr_t)ckpt & 15) ||
      (g_u0 && ((uintptr_t)g_u0 & 15)))
    return bfail(MR_EINVAL, "backward_ckpt: need aligned ckpt, g_msd, n_iter >= 0, ckpt_every >= 1");
  int rc = check_flags();
  if (rc) return rc;
  return reverse(reinterpret_cast<const double2 *>(ckpt), n_iter, ckpt_every, g_msd, g_u0, g_alpha,
                 g_te, msd, s);
}

// Stiffness rows (FP64) and the column-normalised mass M_ij / m_j on the
// operator pattern, for the adjoint kernels.
int mr_ctx::upload_adjoint_operators(hipStream_t s) {
  std::vector<int32_t> kptr(n_nodes + 1, 0), kcol;
  std::vector<double> kval, mwt_t;
  for (int p = 0; p < n_pairs; ++p) {
    const PairHost &h = host[p];
    const int32_t no = dpairs[p].node_off;
    for (int i = 0; i < h.n; ++i) {
      for (int64_t q = h.tab.t3_ptr[i]; q < h.tab.t3_ptr[i + 1]; ++q) {
        const int32_t jn = (int32_t)h.tab.t3_idx[q];
        kcol.push_back(no + jn);
        kval.push_back(h.kval[q]);
        mwt_t.push_back((double)h.mval[q] / (4.0 * (double)h.tab.t5[jn]));
      }
      kptr[no + i + 1] = (int32_t)kcol.size();
    }
  }
  auto put = [&](auto &dst, const auto &v) -> hipError_t {
    hipError_t e = dst.alloc(v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(dst.ptr, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice, s);
  };
  HIP_OK(put(d_kptr, kptr));
  HIP_OK(put(d_kcol, kcol));
  HIP_OK(put(d_kval, kval));
  HIP_OK(put(d_mwt_t, mwt_t));
  HIP_OK(hipStreamSynchronize(s));
  return MR_OK;
}
