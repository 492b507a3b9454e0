// The library context: host pre-computation of every pair plus the packed
// device arrays the kernels read.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/meshreg.h"
#include "device.h"
#include "host.h"
#include "launch.h"

namespace mr {

template <typename T>
struct DevArray {
  T *ptr = nullptr;
  size_t count = 0;
  DevArray() = default;
  DevArray(const DevArray &) = delete;
  DevArray &operator=(const DevArray &) = delete;
  ~DevArray() { release(); }
  hipError_t alloc(size_t n) {
    release();
    count = n;
    if (n == 0) return hipSuccess;
    return hipMalloc((void **)&ptr, n * sizeof(T));
  }
  void release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    count = 0;
  }
  size_t bytes() const { return count * sizeof(T); }
};

}  // namespace mr

struct mr_ctx {
  int device = 0;
  mr_params params{};
  int32_t n_pairs = 0;
  bool host_only = false;
  std::vector<mr::PairHost> host;
  std::vector<mr::DevPair> dpairs;
  int64_t n_nodes = 0, n_tris = 0, n_pix = 0, nnz_factor = 0;
  int n_node_items = 0, n_tiles = 0;
  // per pair offsets into the packed factor arrays (for re-factorisation)
  std::vector<int64_t> dense_off, panel_off;

  mr::DevArray<mr::DevPair> d_pairs;
  mr::DevArray<mr::NodeItem> d_node_items;
  mr::DevArray<mr::TileItem> d_tiles;
  mr::DevArray<int2> d_xy, d_xy_s;             // node corners, natural and solve order
  mr::DevArray<int32_t> d_block_pair, d_active;   // pair of each block; per-pair activity
  mr::DevArray<double> d_run_trace;               // mesh_reg_run: MSD at a check point
  mr::DevArray<int4> d_tri;                     // triangle corners, natural order
  mr::DevArray<int32_t> d_t6, d_iperm, d_perm;
  // per pixel-tile triangle entry (TileItem): corner nodes in natural and in
  // solve order, each with the packed first corner, and the other corners
  mr::DevArray<int4> d_tile_nodes, d_tile_nodes_s;
  mr::DevArray<int2> d_tile_pbc;
  mr::DevArray<uint8_t> d_tile_loc;             // per tile pixel: its entry in the tile's list
  mr::DevArray<int32_t> d_lam_ptr, d_lam_idx;   // per node its (tile entry, corner) slots
                                                // 3 entry + corner, ascending
  mr::DevArray<float> d_coef, d_re, d_rho, d_rho_s;   // rho natural and solve order
  mr::DevArray<int32_t> d_mptr;                 // force operator rows (bit 31: two-word entries)
  mr::DevArray<uint32_t> d_ment;                // its entries (column offset | numerator)
  mr::DevArray<float> d_minv;                   // per row 1 / (4 * 6 m_i)
  mr::DevArray<float2> d_h;
  mr::DevArray<double2> d_x;
  mr::DevArray<mr::DevBlock> d_blocks;
  mr::DevArray<int2> d_fwd_items, d_bwd_items;   // (block, slice) per level
  std::vector<int32_t> fwd_ptr, bwd_ptr;     // level -> range of the item lists (host)
  std::vector<int32_t> fwd_lds, bwd_lds;     // level -> dynamic LDS bytes without the
                                             // per-thread part (16 B per thread added at launch)
  std::vector<int32_t> fwd_nt, bwd_nt;       // level -> workgroup size (autotuned)
  std::vector<int32_t> fwd_bp, bwd_bp;       // level -> smallest allowed workgroup size
  mr::DevArray<double2> d_partials2;         // backward slice partial sums
  // apex (top of every pair's block tree, explicit inverse by subtree structure)
  mr::DevArray<double> d_pcol;                  // panels, column-major copy (forward wave kernel)
  mr::DevArray<double2> d_ybuf;                 // forward solve result y (solve order)
  std::vector<uint8_t> bwd_split;               // per backward level: has split blocks
  std::vector<int32_t> fwd_direct, bwd_direct;  // per level: LDS of the direct-staged kernels
  std::vector<int32_t> fwd_maxb, bwd_maxb;      // per level: rows of its largest block
  mr::DevArray<double2> d_thomas;                // prefilter tables of every image side
  std::map<int32_t, int64_t> thomas_off;         // side -> offset into d_thomas
  mr::DevArray<mr::PrefItem> d_pref_rows, d_pref_cols;  // batched prefilter work items
  mr::DevArray<double> d_prefilter_tmp;          // prefilter scratch (largest pair)
  mr::DevArray<int32_t> d_upper_rows;           // solve rows outside the first forward level
  int64_t n_apex_rows = 0;
  int32_t apex_bwd_lds = 16;                    // dynamic LDS of the apex backward launch
  mr::DevArray<int32_t> d_apex_rows, d_apex_cidx;
  mr::DevArray<int64_t> d_apex_cptr;
  mr::DevArray<mr::ApexFwdItem> d_apex_fitems;
  mr::DevArray<mr::ApexBwdItem> d_apex_bitems;
  mr::DevArray<int2> d_apex_rng;
  mr::DevArray<mr::ApexRow> d_apex_arow;
  mr::DevArray<double> d_apex_xf, d_apex_xb;
  mr::DevArray<double2> d_apex_part, d_apex_y;
  std::vector<int64_t> apex_xf_base, apex_xb_base;   // per pair offsets into d_apex_xf / d_apex_xb
  mr::DevArray<double2> d_apex_t;
  int32_t bwd_split_rows = 128;              // panel rows per backward workgroup
  mr::DevArray<unsigned> d_blk_counters;
  mr::DevArray<int64_t> d_cptr;
  mr::DevArray<int32_t> d_cidx, d_below;
  mr::DevArray<double> d_dcol, d_drow, d_prow;
  mr::DevArray<double2> d_upd;
  mr::DevArray<double> d_partials, d_msd_tmp;
  mr::DevArray<unsigned> d_flags;
  unsigned *host_flags = nullptr;            // pinned copy of d_flags

  // adjoint (allocated by the first backward call)
  mr::DevArray<double2> d_ck, d_seg, d_lam, d_lam_s, d_mu;  // d_lam_s: lambda in solve order
  mr::DevArray<double2> d_lam_part;             // lambda^N per (tile entry, corner)
  mr::DevArray<double> d_cbar, d_alpha_part, d_kval, d_mwt_t;
  mr::DevArray<int32_t> d_kptr, d_kcol;

  // explicit variant (allocated by its first call): each node's triangles as
  // their other two corners and the 1-ring, as CSR with global ids, u_0 and
  // the node records
  mr::DevArray<int32_t> d_x_sptr, d_x_rptr, d_x_ridx;
  mr::DevArray<int2> d_x_opp;
  mr::DevArray<double2> d_x_u0;
  mr::DevArray<mr::NodeRec> d_x_rec;

  // cached HIP graph of one mesh_reg_step (or mesh_reg_step_explicit) call
  hipGraphExec_t graph_exec = nullptr;
  const void *graph_u = nullptr, *graph_trace = nullptr;
  int32_t graph_iters = -1;
  hipStream_t graph_stream = nullptr;
  int graph_mode = -1;                       // 0 semi-implicit, 1 explicit variant
  double graph_tau = 0.0, graph_lam = 0.0;   // the explicit variant's step parameters

  bool timing = false;
  bool fuse_first = true;   // the first forward level assembles b (else a separate launch)
  std::vector<mr::TimedLaunch> pending;
  mr::LaunchTimer timer;

  ~mr_ctx();
  int upload_all(hipStream_t s);
  int upload_factor(int pair, hipStream_t s);
  int upload_prefilter_tables(hipStream_t s);
  int prefilter_any(int p, const float *img_f, const double *img_d, float *coef_out,
                    hipStream_t s);
  int prefilter_pair(int p, const float *img, float *coef_out, hipStream_t s);
  int prefilter_pair_d(int p, const double *img, float *coef_out, hipStream_t s);
  int upload_adjoint_operators(hipStream_t s);
  hipError_t sample(bool with_warp, hipStream_t s);
  hipError_t set_active(const std::vector<int32_t> &flags, hipStream_t s);
  hipError_t assemble(double *finish_msd, hipStream_t s);
  hipError_t force(const double2 *u, hipStream_t s);
  hipError_t solve(double2 *x, double2 *out, hipStream_t s, const mr::AssembleArgs *fuse);
  hipError_t iterate(double2 *u, double *msd_out, double **pending, bool x_holds_u,
                     bool write_u, hipStream_t s);
  hipError_t finish_pending(const double2 *u, double **pending, hipStream_t s);
  hipError_t warp(const double2 *u, double *msd, float *warped, hipStream_t s);
  int check_flags();
  int tune(hipStream_t s);
  bool admissible(bool fwd, size_t lev, int nt) const;
  void force_solve_kernel(int nt);
  hipError_t solve_level(bool fwd, int lev, double2 *x, double2 *out, hipStream_t s,
                         const mr::AssembleArgs *fuse);
  int step(double2 *u, int32_t n_iter, double *msd_trace, hipStream_t s);
  int upload_explicit_tables(hipStream_t s);
  int step_explicit(double2 *u, int32_t n_iter, double tau, double lam, double *msd_trace,
                    hipStream_t s);
  void post_flags(hipStream_t s);
  void timed_begin(int family, hipStream_t s);
  void timed_end(hipStream_t s);
  int64_t device_bytes() const;
  int backward(const double *u0, int32_t n_iter, int32_t ckpt_every, const double *g_msd,
               double *g_u0, double *g_alpha, float *g_te, double *msd, hipStream_t s);
  int forward_with_ckpt(double *u, int32_t n_iter, int32_t ckpt_every, double *ckpt, double *msd,
                        hipStream_t s);
  int backward_from_ckpt(const double *ckpt, int32_t n_iter, int32_t ckpt_every,
                         const double *g_msd, double *g_u0, double *g_alpha, float *g_te,
                         double *msd, hipStream_t s);
  int reserve_adjoint(int32_t n_iter, int32_t ckpt_every, hipStream_t s);
  hipError_t forward_ckpt(double2 *ck, int32_t n_iter, int32_t ckpt_every, hipStream_t s);
  int reverse(const double2 *ck, int32_t n_iter, int32_t ckpt_every, const double *g_msd,
              double *g_u0, double *g_alpha, float *g_te, double *msd, hipStream_t s);
};

namespace mr {
using Ctx = ::mr_ctx;
}

// Records the thread-local last-error text; returns `code`.
int mr_set_error(int code, const std::string &msg);
