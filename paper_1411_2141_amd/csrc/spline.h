// Device-side cubic B-spline sampling shared by the forward and adjoint
// kernels (the abstract: spline interpolation of both images).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace mr {

// ---------------------------------------------------------------------------
// Cubic B-spline pieces.  For a point at integer cell `c` plus fraction t in
// [0, 1), the taps are c-1 .. c+2 and their weights are beta(t+1), beta(t),
// beta(t-1), beta(t-2) of the centred cubic B-spline, with the derivatives
// below.  Index folding is half-sample symmetric with period 2N.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int fold_index(int n, int N) {
  if ((unsigned)n < (unsigned)N) return n;
  // one reflection covers -N <= n < 2N
  const int r = n < 0 ? -1 - n : 2 * N - 1 - n;
  if ((unsigned)r < (unsigned)N) return r;
  const int P = 2 * N;
  int m = n % P;
  if (m < 0) m += P;
  return m >= N ? P - 1 - m : m;
}

__device__ __forceinline__ void bs_weights(float t, float w[4]) {
  const float s = 1.0f - t, t2 = t * t, t3 = t2 * t;
  w[0] = s * s * s * (1.0f / 6.0f);
  w[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
  w[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * (1.0f / 6.0f);
  w[3] = t3 * (1.0f / 6.0f);
}

// FP64 weights (the adjoint kernels).
__device__ __forceinline__ void bs_weights_d(double t, double w[4]) {
  const double s = 1.0 - t, t2 = t * t, t3 = t2 * t;
  w[0] = s * s * s * (1.0 / 6.0);
  w[1] = (3.0 * t3 - 6.0 * t2 + 4.0) * (1.0 / 6.0);
  w[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * (1.0 / 6.0);
  w[3] = t3 * (1.0 / 6.0);
}

__device__ __forceinline__ void bs_deriv(float t, float d[4]) {
  const float s = 1.0f - t, t2 = t * t;
  d[0] = -0.5f * s * s;
  d[1] = 1.5f * t2 - 2.0f * t;
  d[2] = -1.5f * t2 + t + 0.5f;
  d[3] = 0.5f * t2;
}

// Integer cell and fraction of base + off.  Non-finite or absurd offsets are
// replaced by 0 (so no tap leaves the image) and reported through the result.
__device__ __forceinline__ bool split_coord(int base, double off, int &cell, float &frac) {
  const bool ok = (off == off) && fabs(off) < 1.0e6;
  if (!ok) off = 0.0;
  const double fl = floor(off);
  cell = base + (int)fl;
  frac = (float)(off - fl);
  return ok;
}

// Same split, keeping the fraction in FP64.
__device__ __forceinline__ bool split_coord_d(int base, double off, int &cell, double &frac) {
  const bool ok = (off == off) && fabs(off) < 1.0e6;
  if (!ok) off = 0.0;
  const double fl = floor(off);
  cell = base + (int)fl;
  frac = off - fl;
  return ok;
}

// Four consecutive floats from a 4-byte aligned address as one 16-byte load
// (a vector type, so the load is neither split nor merged with the scalar
// loads of the folded path).
typedef float float4_a4 __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ void load_row4(const float *__restrict__ p, float (&t)[4]) {
  const float4_a4 q = *reinterpret_cast<const float4_a4 *>(p);
  t[0] = q.x;
  t[1] = q.y;
  t[2] = q.z;
  t[3] = q.w;
}

// The 4x4 taps of cell (cx, cy) when the whole window lies inside the image
// (1 <= cx, cx + 2 < W, likewise y): four row loads at one 32-bit offset from
// c, one pair's coefficient image (fewer than 2^31 pixels).
__device__ __forceinline__ bool taps_inside(int H, int W, int cx, int cy) {
  return cx >= 1 && cx + 2 < W && cy >= 1 && cy + 2 < H;
}
__device__ __forceinline__ void load_taps_inside(const float *__restrict__ c, int W, int cx, int cy,
                                                 float (&t)[4][4]) {
  // byte offsets from c (sides below 2^16, so the 24-bit product is exact)
  const unsigned o = (__umul24((unsigned)(cy - 1), (unsigned)W) + (unsigned)(cx - 1)) << 2;
  const unsigned row = (unsigned)W << 2;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float4_a4 q = *reinterpret_cast<const float4_a4 *>(
        reinterpret_cast<const char *>(c) + (o + (unsigned)m * row));
    t[m][0] = q.x;
    t[m][1] = q.y;
    t[m][2] = q.z;
    t[m][3] = q.w;
  }
}

// The 4x4 coefficient taps around cell (cx, cy), t[m][n] = c(cy - 1 + m,
// cx - 1 + n) with folded indices: the row loads above when the window lies
// inside the image (the common case), else each tap folded and loaded on its
// own.
__device__ __forceinline__ void load_taps(const float *__restrict__ c, int H, int W, int cx, int cy,
                                          float (&t)[4][4]) {
  if (taps_inside(H, W, cx, cy)) {
    load_taps_inside(c, W, cx, cy, t);
  } else {
    unsigned col[4], row[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      col[k] = (unsigned)fold_index(cx - 1 + k, W);
      row[k] = (unsigned)fold_index(cy - 1 + k, H) * (unsigned)W;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) t[m][n] = c[row[m] + col[n]];
  }
}

__device__ __forceinline__ float spline_value(const float *__restrict__ c, int H, int W, int cx,
                                              float fx, int cy, float fy) {
  float wx[4], wy[4];
  bs_weights(fx, wx);
  bs_weights(fy, wy);
  float t[4][4];
  load_taps(c, H, W, cx, cy, t);
  float v = 0.0f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float rv = t[m][0] * wx[0] + t[m][1] * wx[1] + t[m][2] * wx[2] + t[m][3] * wx[3];
    v += wy[m] * rv;
  }
  return v;
}


// Value and gradient from the 16 taps t (as load_taps gives them).
__device__ __forceinline__ void spline_value_grad_taps(const float (&t)[4][4], float fx, float fy,
                                                       float &val, float &gx, float &gy) {
  float wx[4], dx[4], wy[4], dy[4];
  bs_weights(fx, wx);
  bs_deriv(fx, dx);
  bs_weights(fy, wy);
  bs_deriv(fy, dy);
  val = gx = gy = 0.0f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float c0 = t[m][0], c1 = t[m][1], c2 = t[m][2], c3 = t[m][3];
    const float rv = c0 * wx[0] + c1 * wx[1] + c2 * wx[2] + c3 * wx[3];
    const float rd = c0 * dx[0] + c1 * dx[1] + c2 * dx[2] + c3 * dx[3];
    val += wy[m] * rv;
    gx += wy[m] * rd;
    gy += dy[m] * rv;
  }
}


// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Lane `lane`'s share of a wavefront's sum over a[0 .. n): a[lane],
// a[lane + 64], ... added in that order, with sixteen loads in flight at a
// time (the order, and so the result, does not depend on the batching).
__device__ __forceinline__ double lane_strided_sum(const double *__restrict__ a, int n, int lane) {
  constexpr int U = 16;
  double s = 0.0;
  int k = lane;
  for (; k + (U - 1) * 64 < n; k += U * 64) {
    double v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = a[k + j * 64];
#pragma unroll
    for (int j = 0; j < U; ++j) s += v[j];
  }
  for (; k < n; k += 64) s += a[k];
  return s;
}


// FP64 first and second derivative weights (adjoint kernels).
__device__ __forceinline__ void bs_deriv_d(double t, double d[4]) {
  const double s = 1.0 - t, t2 = t * t;
  d[0] = -0.5 * s * s;
  d[1] = 1.5 * t2 - 2.0 * t;
  d[2] = -1.5 * t2 + t + 0.5;
  d[3] = 0.5 * t2;
}

__device__ __forceinline__ void bs_deriv2_d(double t, double e[4]) {
  e[0] = 1.0 - t;
  e[1] = 3.0 * t - 2.0;
  e[2] = 1.0 - 3.0 * t;
  e[3] = t;
}

}  // namespace mr
