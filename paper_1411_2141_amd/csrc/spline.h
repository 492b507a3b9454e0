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

// FP64 weights for the pixel warp: the MSD is a mean of squared differences
// of nearly equal numbers, so a systematic FP32 weight rounding (at t = 0 the
// FP32 weights sum to 1 + 3e-8 per axis) would bias it by ~1e-6 relative.
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

__device__ __forceinline__ void bs_deriv2(float t, float e[4]) {
  e[0] = 1.0f - t;
  e[1] = 3.0f * t - 2.0f;
  e[2] = 1.0f - 3.0f * t;
  e[3] = t;
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

struct Taps {
  int col[4];
  const float *row[4];
};

// The four taps of one coefficient row around cell cx: one 16-byte load when
// all four lie inside the row (the common case), else the folded taps one by
// one.
struct __attribute__((aligned(4))) Row4 {
  float v[4];
};
__device__ __forceinline__ void row_taps(const float *__restrict__ r, const Taps &tp, int cx, int W,
                                         float t[4]) {
  if (cx >= 1 && cx + 2 < W) {
    Row4 q;
    __builtin_memcpy(&q, r + (cx - 1), sizeof(Row4));
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = q.v[k];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = r[tp.col[k]];
  }
}

__device__ __forceinline__ void make_taps(const float *__restrict__ c, int H, int W, int cx,
                                          int cy, Taps &tp) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    tp.col[k] = fold_index(cx - 1 + k, W);
    tp.row[k] = c + (size_t)fold_index(cy - 1 + k, H) * W;
  }
}

__device__ __forceinline__ float spline_value(const float *__restrict__ c, int H, int W, int cx,
                                              float fx, int cy, float fy) {
  float wx[4], wy[4];
  bs_weights(fx, wx);
  bs_weights(fy, wy);
  Taps tp;
  make_taps(c, H, W, cx, cy, tp);
  float v = 0.0f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    float c[4];
    row_taps(tp.row[m], tp, cx, W, c);
    const float rv = c[0] * wx[0] + c[1] * wx[1] + c[2] * wx[2] + c[3] * wx[3];
    v += wy[m] * rv;
  }
  return v;
}

// Value with FP32 coefficients, FP64 weights and FP64 accumulation.
__device__ __forceinline__ double spline_value_d(const float *__restrict__ c, int H, int W,
                                                 int cx, double fx, int cy, double fy) {
  double wx[4], wy[4];
  bs_weights_d(fx, wx);
  bs_weights_d(fy, wy);
  Taps tp;
  make_taps(c, H, W, cx, cy, tp);
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    float c[4];
    row_taps(tp.row[m], tp, cx, W, c);
    const double rv = (double)c[0] * wx[0] + (double)c[1] * wx[1] + (double)c[2] * wx[2] +
                      (double)c[3] * wx[3];
    v += wy[m] * rv;
  }
  return v;
}

__device__ __forceinline__ void spline_value_grad(const float *__restrict__ c, int H, int W,
                                                  int cx, float fx, int cy, float fy, float &val,
                                                  float &gx, float &gy) {
  float wx[4], dx[4], wy[4], dy[4];
  bs_weights(fx, wx);
  bs_deriv(fx, dx);
  bs_weights(fy, wy);
  bs_deriv(fy, dy);
  Taps tp;
  make_taps(c, H, W, cx, cy, tp);
  val = gx = gy = 0.0f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    float c[4];
    row_taps(tp.row[m], tp, cx, W, c);
    const float c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
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
