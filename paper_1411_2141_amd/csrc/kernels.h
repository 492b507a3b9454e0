// Launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mr {

// B-spline prefilter (B^-1 along rows, then columns) of an FP32 or FP64 image;
// tab_w / tab_h: Thomas tables (cp_k, 1 / pivot_k) of the row / column length.
hipError_t launch_prefilter(const float *src_f, const double *src_d, double *tmp, float *out,
                            int H, int W, const double2 *tab_w, const double2 *tab_h,
                            hipStream_t s);
hipError_t launch_sample_rho(const NodeItem *items, int n_items, const DevPair *pairs,
                             const int2 *xy, const float *coef_re, float *rho, hipStream_t s);
// Sample launch (node displacements un with node tables xy, rho and output
// h, one node order); with n_tiles > 0 it also writes the warp/MSD partials
// of u (in the node order of tile_nodes).
hipError_t launch_sample(const NodeItem *items, int n_items, const DevPair *pairs,
                         const double2 *un, const int2 *xy, const float *coef, const float *rho,
                         float2 *h, unsigned *flags, const TileItem *tiles, int n_tiles,
                         const double2 *u, const int4 *tile_nodes, const int2 *tile_pbc,
                         const uint8_t *tile_loc, const float *re, double *partials,
                         hipStream_t s);
// Assemble launch (solve order; x may be u); with finish_msd it also finishes
// the MSD of `partials`.
hipError_t launch_assemble(int n, const int32_t *mptr, const uint32_t *ment, const float *minv,
                           const float2 *h, const double2 *u, double2 *x, double tau,
                           const DevPair *pairs, int n_pairs, const double *partials,
                           double *finish_msd, const int32_t *active, hipStream_t s);
// One level of the forward / backward block solve; nt = 1 selects the
// wavefront-per-block kernels with direct global-to-LDS staging (blocks of at
// most 64 rows, panels not split), nt = 8 or 16 the wavefront-per-block
// kernels issuing nt loads per lane at a time (blocks of at most 64 rows),
// 64 / 128 / 256 the workgroup-per-block ones with that many threads (LDS
// staged); lds_bytes is the launch's dynamic LDS.
hipError_t launch_solve_fwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int64_t *cptr, const int32_t *cidx,
                                  const double *dcol, const double *prow, const double *pcol,
                                  double2 *x, double2 *ybuf, double2 *upd,
                                  const AssembleArgs *fuse, hipStream_t s);
hipError_t launch_solve_bwd_level(const DevBlock *blocks, const int2 *items, int count,
                                  int lds_bytes, int nt, const int32_t *below_idx,
                                  const double *drow, const double *prow, double2 *x,
                                  const double2 *ybuf, const int32_t *perm, double2 *out,
                                  double2 *partials, unsigned *counters, hipStream_t s);
// The apex of the solve: t = b - (non-apex updates), segment partials of
// y = X t, y, then z = X^T y written to x (and out[perm] when out is given).
hipError_t launch_apex_solve(int n_rows, const int32_t *rows, const int64_t *acptr,
                             const int32_t *acidx, const double2 *upd, double2 *x, double2 *tbuf,
                             const ApexFwdItem *fitems, int n_fitems, const double *xf,
                             double2 *part, const ApexRow *arow, double2 *ybuf,
                             const ApexBwdItem *bitems, int n_bitems, const int2 *rng, int bwd_lds,
                             const double *xb, const int32_t *perm, double2 *out, hipStream_t s);
// Warp partials of u; tpos holds each triangle's corners packed as x | y << 16.
// B^-1 along rows then columns of every pair of a context (img: FP64, all
// pairs' pixels, overwritten by the row pass; out: FP32 coefficients).
hipError_t launch_prefilter_all(const PrefItem *row_items, int n_row_items,
                                const PrefItem *col_items, int n_col_items, const DevPair *pairs,
                                double *img, float *out, const double2 *tab, hipStream_t s);
hipError_t launch_warp_partials(const TileItem *tiles, int n_tiles, const double2 *u,
                                const int4 *tile_nodes, const int2 *tile_pbc,
                                const uint8_t *tile_loc, const float *coef, const float *re,
                                float *warped, double *partials, unsigned *flags,
                                hipStream_t s);
hipError_t launch_msd_finish(const DevPair *pairs, int n_pairs, const double *partials,
                             double *msd, hipStream_t s);
// Algorithm 1 as printed (explicit update, umbrella smoothing), natural node order.
hipError_t launch_explicit_smooth(const NodeItem *items, int n_items, const DevPair *pairs,
                                  int n_pairs, const double2 *u0, double2 *u,
                                  const int32_t *r_ptr, const int32_t *r_idx, double lambda,
                                  bool smooth, bool sample, const int2 *xy, const float *coef,
                                  const float *rho, NodeRec *rec, unsigned *flags,
                                  const double *partials, double *finish_msd, hipStream_t s);
hipError_t launch_explicit_update(const NodeItem *items, int n_items, const DevPair *pairs,
                                  const double2 *u, const NodeRec *rec, const int4 *tri,
                                  const int32_t *o_ptr, const int2 *o_jk, double tau,
                                  double2 *u0, unsigned *flags, const TileItem *tiles, int n_tiles,
                                  const int4 *tile_nodes, const int2 *tile_pbc,
                                  const uint8_t *tile_loc, const float *coef, const float *re,
                                  double *partials, hipStream_t s);
// Per-pair activity flags (1 active, 0 retired) into every work descriptor.
hipError_t launch_set_active(const int32_t *flags, DevPair *pairs, int n_pairs, DevBlock *blocks,
                             const int32_t *block_pair, int n_blocks, NodeItem *items,
                             int n_items, TileItem *tiles, int n_tiles, ApexFwdItem *af, int n_af,
                             ApexBwdItem *ab, int n_ab, hipStream_t s);
hipError_t launch_to_solve_order(int n, const double2 *src, const int32_t *iperm, double2 *x,
                                 hipStream_t s);
hipError_t launch_from_solve_order(int n, const double2 *x, const int32_t *iperm, double2 *dst,
                                   hipStream_t s);
hipError_t launch_h_from_solve_order(int n, const float2 *hs, const int32_t *iperm, float2 *h,
                                     hipStream_t s);

}  // namespace mr
