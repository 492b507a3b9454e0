/*
 * meshreg.h -- C ABI of the MI355X (gfx950) mesh-based image registration library.
 *
 * The library implements the per-iteration hot path of triangular-mesh image
 * registration (Baghaie, Yu, D'souza, "Fast Mesh-Based Medical Image
 * Registration", arXiv:1411.2141).  The objective is eq. 1,
 *     E[u] = D[Re, Te o u] + alpha S[u],
 * with the nodal SSD data term of eq. 4 (template sampled at the displaced
 * nodes, eq. 3) and the P1 diffusion energy S[u] = 1/2 sum_c u_c^T K u_c as the
 * regulariser (the mesh Laplacian of Section 2.3 in symmetric form).  One
 * iteration follows Algorithm 1 (update, then smoothing) in semi-implicit form:
 *
 *   t_i, g_i = s_Te(V_i - 1/2 + u_i), grad s_Te(...)      cubic B-spline (abstract)
 *   r_i = t_i - s_Re(V_i - 1/2),  h_i = r_i g_i          eq. 4, eq. 6
 *   f = (M h) / m                                        eq. 10 applied to the P1 load
 *   b = u - tau f                                        eq. 5
 *   (I + tau alpha K) u+ = b  for x and y                eq. 7-8 made implicit; solved
 *                                                        directly (abstract) with a
 *                                                        sparse Cholesky factor
 *
 * and the result is judged by the MSD of the piecewise-linearly warped template
 * against Re (Section 1; Fig. 3; Table 1).  mesh_reg_run repeats the iteration
 * until a relative-MSD stopping rule retires each pair (Algorithm 1's loop "to
 * convergence"); mesh_reg_step_explicit runs Algorithm 1 exactly as printed
 * (explicit update with the eq. 9-10 mesh gradient on the deformed mesh, then
 * the eq. 14 umbrella smoothing) on the same context.
 *
 * Conventions
 *   - Pixel (row i, col j) is the unit square [j, j+1) x [i, i+1); the mesh covers
 *     [0, W] x [0, H] (Section 2.1); nodes sit on integer pixel corners (x, y).
 *   - Spline coordinate = image coordinate - 1/2, so sample [i][j] sits at (j, i).
 *     Boundary: half-sample symmetric.  Coefficients are FP32.
 *   - Displacements u are FP64, packed pair-major in the order of the pairs given
 *     to mesh_reg_init; within a pair node-major with (x, y) interleaved:
 *     u[2 * (node_offset(p) + i) + c].
 *   - Images and image gradients are FP32, packed pair-major, each pair row-major.
 *   - Every call enqueues work on the given HIP stream (NULL = default stream) and
 *     returns without synchronising; outputs land in device memory.
 *
 * Ownership
 *   - The caller owns every DEVICE buffer passed in; the library never frees them.
 *   - mesh_reg_init copies the mesh and builds its own coefficient images, so te/re
 *     may be released after init returns (init synchronises its stream).
 *   - The context owns its tables, factor, schedules and scratch; mesh_reg_destroy
 *     frees them.  A context must not be used from two threads at once, and its
 *     calls must not overlap on different streams (they share its scratch).
 *
 * Errors
 *   - Every call returns an MR_* status; nothing is thrown across the ABI.
 *   - On error mesh_reg_init sets *out = NULL; other calls leave the state as it was
 *     before the call when they fail during validation.
 *   - mesh_reg_last_error() returns a thread-local message for the last failure.
 *   - Non-finite displacements met by a kernel raise a sticky device flag that the
 *     next call reports as MR_ENONFINITE (the offending coordinates are clamped
 *     so no access leaves the images).
 */
#ifndef MESHREG_H
#define MESHREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mr_ctx mr_ctx;

enum {
  MR_OK = 0,
  MR_EINVAL = -1,      /* invalid argument or mesh */
  MR_ENOMEM = -2,      /* host or device allocation failed */
  MR_EHIP = -3,        /* a HIP runtime call failed */
  MR_ENOTSPD = -4,     /* (I + tau alpha K) not positive definite (non-positive pivot) */
  MR_ESTATE = -5,      /* call not valid in the context's state (e.g. host-only) */
  MR_ENONFINITE = -6   /* a kernel met a non-finite displacement */
};

enum { MR_FORCE_P1 = 0, MR_FORCE_NODAL = 1 };

enum {
  MR_FLAG_HOST_ONLY = 1, /* build tables, operators and the factor only; no device work */
  MR_FLAG_NO_TUNE = 4,   /* skip the solve-schedule autotuning at init (fixed 256-thread
                            workgroups) */
  MR_FLAG_SEPARATE_ASSEMBLY = 8, /* the force assembly of an iteration runs in a launch of its
                            own (otherwise the autotuner chooses between that and assembling
                            inside the first forward solve launch; untuned: inside) */
  MR_FLAG_GRAPH = 2      /* mesh_reg_step (and each chunk of mesh_reg_run) captures its
                            launches in a HIP graph once per (u, n_iter, msd_trace, stream)
                            and replays it on later calls with the same arguments (a NULL
                            stream runs eagerly) */
};

/* One registration pair (Algorithm 1, "Inputs"; Section 2.1 for (V, T)). */
typedef struct {
  int32_t height, width;       /* image rows, columns (1 .. 65535; at most 2^31 - 1 pixels) */
  int32_t n_nodes, n_tris;     /* >= 3 and >= 1 */
  const int32_t *node_xy;      /* HOST [n_nodes][2] integer corners (x, y) in [0,W]x[0,H]; copied */
  const int32_t *tris;         /* HOST [n_tris][3] node indices, positive signed area
                                  (b - a) x (c - a) > 0 in (x, y); copied */
  const float *te;             /* DEVICE [H][W] template; read during init only */
  const float *re;             /* DEVICE [H][W] reference; read during init only */
  double alpha;                /* regularisation weight of eq. 1, >= 0 */
} mr_pair;

typedef struct {
  double tau;                  /* step size of eq. 5, > 0 */
  int32_t force_mode;          /* MR_FORCE_P1 (default) or MR_FORCE_NODAL (f = h, eq. 6 literally) */
  int32_t flags;               /* MR_FLAG_* */
  int32_t apex_rows;           /* solve schedule: most rows per pair in the apex (the top levels
                                  of the block tree, solved with the explicit inverse of their
                                  factor block); 0 = automatic (several pairs: a level joins
                                  while the inverse entries it adds stay within
                                  max(2^21 / n_pairs, 2^18), up to 1024 rows per pair; one pair:
                                  up to 16384 rows), -1 = none */
  int32_t bwd_split_rows;      /* solve schedule: panel rows per backward workgroup; 0 = automatic
                                  (128 for one pair, unsplit for a batch) */
  int32_t solve_kernel;        /* solve schedule: 0 = autotuned per level; 1 = wavefront per
                                  block with the block's factor data copied straight into LDS
                                  (blocks <= 64 rows, <= 64 KB); 8 or 16 = wavefront per block
                                  with 8 or 16 loads per lane in flight (blocks <= 64 rows);
                                  32, 33 or 34 = half wavefront per block (blocks <= 32 rows)
                                  with 8, 16 or 4 loads per lane in flight; these five
                                  need unsplit backward blocks; 64, 128, 256, 512 or 1024 =
                                  workgroup per block of that size; levels where the choice is not admissible
                                  take the smallest admissible workgroup size.  MR_FLAG_NO_TUNE
                                  with 0 means 256 everywhere. */
} mr_params;

/* Pre-computation (Algorithm 1): validates every mesh, builds tables T1-T6
 * (node->triangle slots, 1-ring, operator pattern, doubled areas, lumped-mass
 * weights, pixel->triangle map), the P1 stiffness and mass, a nested-dissection
 * ordering, the FP64 Cholesky factor of (I + tau alpha K) per pair and its block
 * solve schedule, then (unless MR_FLAG_HOST_ONLY) uploads everything, computes
 * the B-spline coefficients of te and re and the reference samples at the
 * undisplaced nodes on the device, and (unless MR_FLAG_NO_TUNE) times the
 * admissible workgroup sizes of every solve level on this data and keeps the
 * fastest.  Synchronises `stream` before returning.
 * Errors: MR_EINVAL (bad argument or mesh: index out of range, non-positive area,
 * unreferenced node, node outside the image, uncovered pixel, tau <= 0, alpha < 0,
 * NaN), MR_ENOTSPD, MR_ENOMEM, MR_EHIP. */
int mesh_reg_init(const mr_pair *pairs, int32_t n_pairs, const mr_params *params,
                  void *stream, mr_ctx **out);

/* n_iter >= 0 iterations of Algorithm 1 (semi-implicit) on every pair, in place.
 * u: DEVICE [sum n][2] FP64, in/out.  msd_trace: DEVICE [n_iter][n_pairs] FP64 or
 * NULL; when given, MSD(u^{k+1}) of every pair is written after iteration k (the
 * full-pixel warp runs every iteration).  Errors: MR_EINVAL, MR_ESTATE, MR_EHIP,
 * MR_ENONFINITE (reported by the call after the one that met it). */
int mesh_reg_step(mr_ctx *ctx, double *u, int32_t n_iter, double *msd_trace, void *stream);

/* Algorithm 1's loop run to convergence (the paper gives no criterion; this is a
 * relative-MSD rule), pair by pair: after every check_every (>= 1) iterations each
 * pair still running compares its MSD m_now with m_prev, the MSD check_every
 * iterations earlier (MSD(u0) at first), and retires when m_prev <= 0 or
 * m_prev - m_now < rel_tol * m_prev (an increase retires too), or when max_iter
 * (>= 0) iterations are done.  A retired pair's work items skip every later
 * launch, so its u stays as it was at its retirement while the others go on.
 * u: DEVICE [sum n][2] FP64, in/out.  iters_out: HOST [n_pairs], the iterations
 * each pair ran (a multiple of check_every, or max_iter).  msd_out: DEVICE
 * [n_pairs] FP64, each pair's MSD at its final u.  rel_tol: finite, >= 0.
 * The full-pixel warp runs only at the check points.  Synchronises `stream` after
 * every chunk (the decision is taken on the host); every pair is active again on
 * return.  Calls on one context must not overlap.  Errors as mesh_reg_step. */
int mesh_reg_run(mr_ctx *ctx, double *u, int32_t max_iter, int32_t check_every, double rel_tol,
                 int32_t *iters_out, double *msd_out, void *stream);

/* n_iter >= 0 iterations of Algorithm 1 as printed (explicit, Section 2) on every
 * pair, in place: with u = u_1^k,
 *   t_i = s_Te(V_i - 1/2 + u_i), r_i = t_i - s_Re(V_i - 1/2)         eq. 3-4
 *   g_i = sum_j A_j grad t_Tj / sum_j A_j over i's triangles          eq. 9-10
 *         (grad t_Tj the linear gradient of t on the triangle's deformed corners
 *         V + u, A_j its unsigned deformed area; zero-area triangles add nothing)
 *   u_0 = u - tau r g                                                 eq. 5-6
 *   u_1^{k+1} = (1 - lambda) u_0 + lambda A^Lap u_0                   eq. 11-14
 *         (A^Lap: 1/m_i on the m_i nodes of i's 1-ring)
 * tau: finite, >= 0 (the paper's 0.005 is for 0-255 intensities: 0.005 * 255^2 on
 * [0, 1] images); lambda: 0 .. 1 (the paper's 0.8).  The context's own tau, alpha
 * and factor are not used.  u: DEVICE [sum n][2] FP64, natural node order, in/out.
 * msd_trace: DEVICE [n_iter][n_pairs] FP64 or NULL (MSD(u_1^{k+1}) after
 * iteration k).  Graph replay as mesh_reg_step.  Timing families: smoothing and
 * sampling count as "sample", the update as "assemble".  The first call builds
 * the variant's tables on the device (synchronising `stream`).  Errors as
 * mesh_reg_step. */
int mesh_reg_step_explicit(mr_ctx *ctx, double *u, int32_t n_iter, double tau, double lambda,
                           double *msd_trace, void *stream);

/* Warp and MSD (Section 1; Fig. 3): every pixel takes the piecewise-linear
 * displacement of its triangle (T6), the template spline is sampled at the
 * displaced pixel centre and msd[p] = mean over pixels of (W - Re)^2 (FP64,
 * deterministic order).  u: DEVICE [sum n][2]; msd: DEVICE [n_pairs];
 * warped: DEVICE [sum H*W] FP32 or NULL. */
int mesh_reg_warp_msd(mr_ctx *ctx, const double *u, double *msd, float *warped, void *stream);

/* mesh_reg_warp_msd for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and results, with the per-tile partial sums in a static device
 * array of the library (2^19 tiles of 16 x 16 pixels, 4 MiB per GPU, held until
 * the process ends) instead of the context's buffer; the call allocates nothing.
 * Calls on one GPU share that array, so calls that overlap on one GPU race.
 * Errors: as mesh_reg_warp_msd, plus MR_EINVAL when the context has more pixel
 * tiles than the array holds, MR_ESTATE when mesh_reg_init did not run on this
 * GPU. */
int mesh_reg_warp_msd_noalloc(mr_ctx *ctx, const double *u, double *msd, float *warped,
                              void *stream);

/* The force of one iteration (eq. 4-6 and eq. 10) for the given u:
 * h: DEVICE [sum n][2] FP32 or NULL (h_i = r_i g_i); b: DEVICE [sum n][2] FP64 or
 * NULL (b = u - tau f, natural node order). */
int mesh_reg_force(mr_ctx *ctx, const double *u, float *h, double *b, void *stream);

/* x = (I + tau alpha K)^-1 b per pair and component, by the FP64 triangular
 * solves of the Cholesky factor.  b, x: DEVICE [sum n][2]; may alias. */
int mesh_reg_solve(mr_ctx *ctx, const double *b, double *x, void *stream);

/* Reverse mode of the objective of eq. 1 as unrolled by Algorithm 1 (n_iter
 * semi-implicit iterations from u0, eq. 3-8, then the warp + MSD of Section 1):
 * with L = sum_p g_msd[p] * MSD_p(u^N), writes dL/du0 (DEVICE [sum n][2] FP64 or
 * NULL), dL/dalpha_p (DEVICE [n_pairs] FP64 or NULL), dL/dTe (DEVICE [sum H*W]
 * FP32 or NULL) and the forward MSDs (DEVICE [n_pairs] FP64 or NULL).
 * Iterates u^k are recomputed from checkpoints every ckpt_every (>= 1) iterations;
 * the adjoint solves reuse each pair's factor.  g_msd: DEVICE [n_pairs] FP64. */
int mesh_reg_backward(mr_ctx *ctx, const double *u0, int32_t n_iter, int32_t ckpt_every,
                      const double *g_msd, double *g_u0, double *g_alpha, float *g_te,
                      double *msd, void *stream);

/* The forward pass of the objective of eq. 1 as unrolled by Algorithm 1, keeping
 * what mesh_reg_backward_ckpt needs: n_iter (>= 0) iterations in place on u
 * (DEVICE [sum n][2] FP64, in u^0, out u^N) that also write the checkpoints
 * ckpt[q] = u^{q ckpt_every} for q < n_seg and ckpt[n_seg] = u^N, with
 * n_seg = ceil(n_iter / ckpt_every) (ckpt: DEVICE [n_seg + 1][sum n][2] FP64,
 * caller-owned, 16-byte aligned), and the MSD of u^N (msd: DEVICE [n_pairs] FP64
 * or NULL; Section 1).  The iterates are those of mesh_reg_step bit for bit.
 * Errors: MR_EINVAL (null or misaligned u or ckpt, n_iter < 0, ckpt_every < 1),
 * MR_ESTATE, MR_EHIP, MR_ENONFINITE. */
int mesh_reg_forward_ckpt(mr_ctx *ctx, double *u, int32_t n_iter, int32_t ckpt_every,
                          double *ckpt, double *msd, void *stream);

/* Reverse mode as mesh_reg_backward, from the checkpoints a mesh_reg_forward_ckpt
 * call with the same n_iter and ckpt_every wrote (read only; the forward pass is
 * not run again, only the iterates between checkpoints are recomputed).  The
 * context's alpha, template and tau must be those of that forward call.
 * Errors: MR_EINVAL (null or misaligned ckpt or g_u0, null g_msd, n_iter < 0,
 * ckpt_every < 1), MR_ESTATE, MR_EHIP, MR_ENONFINITE. */
int mesh_reg_backward_ckpt(mr_ctx *ctx, const double *ckpt, int32_t n_iter, int32_t ckpt_every,
                           const double *g_msd, double *g_u0, double *g_alpha, float *g_te,
                           double *msd, void *stream);

/* Replace pair `pair`'s alpha, the regularisation weight of eq. 1 (alpha S[u]):
 * numeric re-factorisation of (I + tau alpha K) with the symbolic analysis
 * reused, then upload.  Synchronises `stream`.  Errors: MR_EINVAL (pair out of
 * range, alpha negative or not finite), MR_ENOTSPD (a pivot overflows or is not
 * positive), MR_EHIP; on MR_EINVAL and MR_ENOTSPD the pair keeps its old alpha
 * and factor. */
int mesh_reg_set_alpha(mr_ctx *ctx, int32_t pair, double alpha, void *stream);

/* Replace pair `pair`'s template (DEVICE [H][W] FP32): recomputes its spline
 * coefficients.  Enqueued on `stream`. */
int mesh_reg_set_template(mr_ctx *ctx, int32_t pair, const float *te, void *stream);

/* Table export for tests.  Copies table `table_id` (MR_TAB_*) of `pair` into
 * host_out (if not NULL) and writes its element count to *len.  Element types:
 * int64 for every table except MR_TAB_T6 (int32 [H][W]) and MR_TAB_PERM (int32). */
enum {
  MR_TAB_T1_PTR = 10, MR_TAB_T1_SLOT = 11,   /* slot = 3 * triangle + corner */
  MR_TAB_T2_PTR = 20, MR_TAB_T2_IDX = 21,
  MR_TAB_T3_PTR = 30, MR_TAB_T3_IDX = 31,
  MR_TAB_T4 = 40, MR_TAB_T5 = 50, MR_TAB_T6 = 60,
  MR_TAB_PERM = 70                           /* elimination order: perm[k] = node */
};
int mesh_reg_get_tables(mr_ctx *ctx, int32_t pair, int32_t table_id, void *host_out,
                        int64_t *len);

/* Scalar facts about a pair or the context (MR_INFO_*), written to *value. */
enum {
  MR_INFO_N_NODES = 1, MR_INFO_N_TRIS = 2, MR_INFO_NNZ_L = 3, MR_INFO_N_BLOCKS = 4,
  MR_INFO_FWD_LEVELS = 5, MR_INFO_BWD_LEVELS = 6, MR_INFO_NODE_OFFSET = 7,
  MR_INFO_PIXEL_OFFSET = 8, MR_INFO_N_PAIRS = 9, MR_INFO_DEVICE_BYTES = 10,
  MR_INFO_SOLVE_OFFBLOCK = 11,  /* off-block factor entries per direction */
  MR_INFO_SOLVE_DENSE = 12,     /* packed dense-inverse entries per direction */
  MR_INFO_MASS_NNZ = 13,        /* entries of the force operator rows */
  MR_INFO_APEX_ROWS = 14,       /* rows of the apex of the solve (0: none) */
  MR_INFO_SOLVE_BYTES = 15,     /* algorithmic bytes of one solve call (both triangular passes) */
  MR_INFO_FUSED_ASSEMBLY = 16,  /* context: 1 if an iteration assembles the right-hand side inside
                                   the first forward solve launch, 0 if in a launch of its own
                                   (chosen by the autotuner) */
  MR_INFO_TILE_ENTRIES = 17     /* distinct triangles of T6 summed over the pair's 16 x 16 pixel
                                   tiles (the warp's per-tile triangle lists) */
};
int mesh_reg_get_info(mr_ctx *ctx, int32_t pair, int32_t key, int64_t *value);

/* Per-kernel timing: when enabled, every kernel launch carries a start/stop
 * event pair attached to its dispatch (hipExtLaunchKernel), so host gaps are
 * not counted; mesh_reg_kernel_times returns,
 * per family (MR_KF_*), the summed milliseconds and the launch count, and resets
 * them.  Synchronises the stream of the last launch. */
enum { MR_KF_SAMPLE = 0, MR_KF_ASSEMBLE = 1, MR_KF_SOLVE = 2, MR_KF_WARP = 3, MR_KF_COUNT = 4 };
int mesh_reg_enable_timing(mr_ctx *ctx, int32_t enable);
int mesh_reg_kernel_times(mr_ctx *ctx, double *ms, int64_t *launches);

/* Switches the graph replay of mesh_reg_step (MR_FLAG_GRAPH) on or off for
 * later calls; switching it off drops the cached graph.  While timing is
 * enabled mesh_reg_step always runs eagerly. */
int mesh_reg_set_graph(mr_ctx *ctx, int32_t enable);

void mesh_reg_destroy(mr_ctx *ctx);

/* Thread-local text of the last failure on this thread; valid until the next
 * call on that thread. */
const char *mesh_reg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MESHREG_H */
