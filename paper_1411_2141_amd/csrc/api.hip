// C ABI of the registration library: context set-up (Algorithm 1's
// pre-computation), the iteration loop, warp + MSD, and table export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/meshreg.h"
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "ctx.h"

using namespace mr;

static thread_local std::string g_last_error;

int mr_set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

static int fail(int code, const std::string &msg) { return mr_set_error(code, msg); }

// A roctx range around an entry point (named after it), so that profiler
// traces group each call's kernel launches; a no-op without a profiler.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// Static device scratch of mesh_reg_warp_msd_noalloc: the per-tile FP64
// partial sums of the warp + MSD, 2^19 tiles of 16 x 16 pixels (4 MiB, images
// of up to 2^27 pixels in all).  Each GPU the library runs on holds its own
// copy until the process ends; its device address is looked up once per
// device by mesh_reg_init (hipGetSymbolAddress with that device current) and
// only that address is used on the host (the array's name is a host-side
// stand-in).  Calls on one GPU share it: overlapping calls race.
constexpr size_t kScratchDoubles = size_t(1) << 19;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

static int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(MR_EINVAL, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return MR_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MR_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double *>(ptr);
  return MR_OK;
}

static double *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(MR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

namespace mr {

template <typename T>
static hipError_t upload(DevArray<T> &dst, const std::vector<T> &src, hipStream_t s) {
  hipError_t e = dst.alloc(src.size());
  if (e != hipSuccess || src.empty()) return e;
  return hipMemcpyAsync(dst.ptr, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Thomas elimination of the B-spline interpolation system of length N
// (diagonal 4/6, 5/6 at both ends for the half-sample-symmetric boundary,
// off-diagonal 1/6): per k, (cp_k, 1 / pivot_k) with pivot_0 = 5/6,
// pivot_k = diag_k - cp_{k-1} / 6 and cp_k = (1/6) / pivot_k.
static std::vector<double2> thomas_table(int N) {
  std::vector<double2> t(std::max(N, 1), make_double2(0.0, 0.0));
  if (N <= 1) return t;
  const double off = 1.0 / 6.0;
  double cp_prev = 0.0;
  for (int k = 0; k < N; ++k) {
    const double diag = (k == 0 || k == N - 1) ? 5.0 / 6.0 : 4.0 / 6.0;
    const double piv = k == 0 ? diag : diag - off * cp_prev;
    const double cp = off / piv;
    t[k] = make_double2(cp, 1.0 / piv);
    cp_prev = cp;
  }
  return t;
}

}  // namespace mr

// Per-launch timing: between timed_begin and timed_end every launch of the
// calling thread records dispatch-attached events under `fam`.
void mr_ctx::timed_begin(int fam, hipStream_t) {
  if (!timing) return;
  timer.family = fam;
  timer.out = &pending;
  mr::tl_launch_timer = &timer;
}

void mr_ctx::timed_end(hipStream_t) { mr::tl_launch_timer = nullptr; }

// Launches the two triangular solves on x (solve order, in place).  When `out`
// is given, the backward pass also scatters the result to natural order there.
hipError_t mr_ctx::solve_level(bool fwd, int lev, double2 *x, double2 *out, hipStream_t s,
                               const AssembleArgs *fuse) {
  if (fwd) {
    const int cnt = fwd_ptr[lev + 1] - fwd_ptr[lev];
    if (!cnt && !fuse) return hipSuccess;
    const int nt = fwd_nt[lev];
    return launch_solve_fwd_level(d_blocks.ptr, d_fwd_items.ptr + fwd_ptr[lev], cnt,
                                  nt == 1 ? fwd_direct[lev] : fwd_lds[lev] + 16 * nt, nt,
                                  d_cptr.ptr, d_cidx.ptr, d_dcol.ptr,
                                  d_prow.ptr, d_pcol.ptr, x, d_ybuf.ptr, d_upd.ptr, fuse, s);
  }
  const int cnt = bwd_ptr[lev + 1] - bwd_ptr[lev];
  if (!cnt) return hipSuccess;
  const int nt = bwd_nt[lev];
  return launch_solve_bwd_level(d_blocks.ptr, d_bwd_items.ptr + bwd_ptr[lev], cnt,
                                nt == 1 ? bwd_direct[lev] : bwd_lds[lev] + 16 * nt, nt,
                                d_below.ptr, d_drow.ptr, d_prow.ptr,
                                x, d_ybuf.ptr, d_perm.ptr, out, d_partials2.ptr,
                                d_blk_counters.ptr, s);
}

// With `fuse`, the right-hand side is assembled by the first forward level's
// launch (AssembleArgs) instead of being read from x.
hipError_t mr_ctx::solve(double2 *x, double2 *out, hipStream_t s, const AssembleArgs *fuse) {
  hipError_t e = hipSuccess;
  const int n_fl = (int)fwd_ptr.size() - 1;
  for (int lev = 0; lev < std::max(n_fl, fuse ? 1 : 0); ++lev) {
    const AssembleArgs *f = lev == 0 ? fuse : nullptr;
    if (!f && fwd_ptr[lev + 1] == fwd_ptr[lev]) continue;
    timed_begin(MR_KF_SOLVE, s);
    e = solve_level(true, lev, x, out, s, f);
    timed_end(s);
    if (e != hipSuccess) return e;
  }
  if (n_apex_rows) {
    timed_begin(MR_KF_SOLVE, s);
    e = launch_apex_solve((int)n_apex_rows, d_apex_rows.ptr, d_apex_cptr.ptr, d_apex_cidx.ptr,
                          d_upd.ptr, x, d_apex_t.ptr, d_apex_fitems.ptr,
                          (int)d_apex_fitems.count, d_apex_xf.ptr, d_apex_part.ptr,
                          d_apex_arow.ptr, d_apex_y.ptr, d_apex_bitems.ptr,
                          (int)d_apex_bitems.count, d_apex_rng.ptr, apex_bwd_lds, d_apex_xb.ptr,
                          d_perm.ptr, out, s);
    timed_end(s);
    if (e != hipSuccess) return e;
  }
  for (int lev = 0; lev < (int)bwd_ptr.size() - 1; ++lev) {
    if (bwd_ptr[lev + 1] == bwd_ptr[lev]) continue;
    timed_begin(MR_KF_SOLVE, s);
    e = solve_level(false, lev, x, out, s, nullptr);
    timed_end(s);
    if (e != hipSuccess) return e;
  }
  return e;
}

// Autotuner: for every solve level, times each admissible kernel on the
// context's own data (first each level alone, then each level inside the
// whole solve) and keeps the fastest: the half-wavefront-per-block kernels
// (blocks of at most 32 rows; 8 or 16 loads per lane in flight), the wavefront-per-block kernels with
// direct LDS staging (blocks of at most 64 rows whose factor data fits 64 KB)
// or with register batches (blocks of at most 64 rows) (backward: no split
// blocks), and the workgroup-per-block
// kernels with 64, 128, 256, 512 or 1024 threads (at least the level's
// largest block rounded up to a power of two).  The level kernels only read and write the
// solve scratch vectors, so running them on whatever those hold is harmless.
bool mr_ctx::admissible(bool fwd, size_t lev, int nt) const {
  const std::vector<int32_t> &minnt = fwd ? fwd_bp : bwd_bp;
  if (nt == 1)
    return minnt[lev] <= 64 && (fwd ? fwd_direct[lev] : bwd_direct[lev]) <= 64 * 1024 &&
           (fwd || !bwd_split[lev]);
  if (nt == 32 || nt == 33 || nt == 34)
    return (fwd ? fwd_maxb[lev] : bwd_maxb[lev]) <= 32 && (fwd || !bwd_split[lev]);
  if (nt < 64) return minnt[lev] <= 64 && (fwd || !bwd_split[lev]);
  return nt >= minnt[lev];
}

// Every level takes `nt` where admissible, else the smallest admissible
// workgroup size.
void mr_ctx::force_solve_kernel(int nt) {
  for (int dir = 0; dir < 2; ++dir) {
    const bool fwd = dir == 0;
    std::vector<int32_t> &choice = fwd ? fwd_nt : bwd_nt;
    for (size_t lev = 0; lev < choice.size(); ++lev) {
      int pick = 256;
      if (admissible(fwd, lev, nt)) {
        pick = nt;
      } else {
        for (int w : {64, 128, 256})
          if (admissible(fwd, lev, w)) {
            pick = w;
            break;
          }
      }
      choice[lev] = pick;
    }
  }
}

int mr_ctx::tune(hipStream_t s) {
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  int rc = MR_OK;
  // the first forward level runs fused with the force assembly in the
  // iteration, so it is timed that way (on scratch data: u = x)
  const AssembleArgs fuse{d_mptr.ptr, d_ment.ptr, d_minv.ptr, d_h.ptr, d_x.ptr,
                          d_upper_rows.ptr, (int32_t)d_upper_rows.count, n_pairs, params.tau,
                          d_pairs.ptr, d_partials.ptr, nullptr, d_active.ptr};
  // best of the second and third of three runs, in ms (negative on error)
  auto time_it = [&](auto &&run) -> float {
    float t_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      hipError_t e = hipEventRecord(a, s);
      if (e == hipSuccess) e = run();
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) {
        rc = fail(MR_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        return -1.0f;
      }
      if (rep > 0) t_min = std::min(t_min, ms);
    }
    return t_min;
  };
  static const int kCandidates[] = {1, 8, 16, 32, 33, 34, 64, 128, 256, 512, 1024};
  // The first forward level either assembles the right-hand side itself
  // (fused) or follows a separate assembly launch; both are candidates unless
  // the separate launch is requested.
  const bool separate = (params.flags & MR_FLAG_SEPARATE_ASSEMBLY) != 0;
  auto first_level = [&](bool fused) -> hipError_t {
    if (fused) return solve_level(true, 0, d_x.ptr, nullptr, s, &fuse);
    hipError_t e = assemble(nullptr, s);
    return e == hipSuccess ? solve_level(true, 0, d_x.ptr, nullptr, s, nullptr) : e;
  };
  // pass 1: every level on its own
  for (int dir = 0; dir < 2 && rc == MR_OK; ++dir) {
    const bool fwd = dir == 0;
    std::vector<int32_t> &choice = fwd ? fwd_nt : bwd_nt;
    for (size_t lev = 0; lev < choice.size() && rc == MR_OK; ++lev) {
      float best = 1e30f;
      int best_nt = choice[lev];
      bool best_fused = !separate;
      for (int nt : kCandidates) {
        if (!admissible(fwd, lev, nt)) continue;
        choice[lev] = nt;
        for (int f = fwd && lev == 0 && separate ? 0 : 1; f >= (fwd && lev == 0 ? 0 : 1); --f) {
          const float t = time_it([&] {
            return fwd && lev == 0 ? first_level(f != 0)
                                   : solve_level(fwd, (int)lev, d_x.ptr, nullptr, s, nullptr);
          });
          if (t < 0.0f) break;
          if (t < best) {
            best = t;
            best_nt = nt;
            best_fused = f != 0;
          }
        }
        if (rc != MR_OK) break;
      }
      choice[lev] = best_nt;
      if (fwd && lev == 0) fuse_first = best_fused;
    }
  }
  // pass 2: one level at a time inside the whole solve (the other levels and
  // the apex evict the caches as in an iteration), keeping a change only when
  // the whole solve gets faster
  auto whole = [&]() -> hipError_t {
    if (fuse_first) return solve(d_x.ptr, nullptr, s, &fuse);
    hipError_t e = assemble(nullptr, s);
    return e == hipSuccess ? solve(d_x.ptr, nullptr, s, nullptr) : e;
  };
  float cur = rc == MR_OK ? time_it(whole) : -1.0f;
  for (int dir = 0; dir < 2 && rc == MR_OK; ++dir) {
    const bool fwd = dir == 0;
    std::vector<int32_t> &choice = fwd ? fwd_nt : bwd_nt;
    const std::vector<int32_t> &ptr = fwd ? fwd_ptr : bwd_ptr;
    for (size_t lev = 0; lev < choice.size() && rc == MR_OK; ++lev) {
      if (ptr[lev + 1] == ptr[lev] && !(fwd && lev == 0)) continue;
      const int kept = choice[lev];
      const bool kept_fused = fuse_first;
      int best_nt = kept;
      bool best_fused = kept_fused;
      for (int nt : kCandidates) {
        if (!admissible(fwd, lev, nt)) continue;
        for (int f = fwd && lev == 0 && separate ? 0 : 1; f >= (fwd && lev == 0 ? 0 : 1); --f) {
          if (nt == kept && (f != 0) == kept_fused) continue;
          choice[lev] = nt;
          if (fwd && lev == 0) fuse_first = f != 0;
          const float t = time_it(whole);
          if (t < 0.0f) break;
          if (t < cur) {
            cur = t;
            best_nt = nt;
            best_fused = f != 0;
          }
        }
        if (rc != MR_OK) break;
      }
      choice[lev] = best_nt;
      fuse_first = fwd && lev == 0 ? best_fused : fuse_first;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return rc;
}

// Sample launch at the node displacements in x (solve order; h in solve
// order); with `with_warp` it also writes the warp partials of the same
// displacements (triangle corners in solve order).
hipError_t mr_ctx::sample(bool with_warp, hipStream_t s) {
  timed_begin(MR_KF_SAMPLE, s);
  hipError_t e = launch_sample(d_node_items.ptr, n_node_items, d_pairs.ptr, d_x.ptr, d_xy_s.ptr,
                               d_coef.ptr, d_rho_s.ptr, d_h.ptr, d_flags.ptr, d_tiles.ptr,
                               with_warp ? n_tiles : 0, d_x.ptr, d_tile_nodes_s.ptr,
                               d_tile_pbc.ptr, d_tile_loc.ptr, d_re.ptr, d_partials.ptr, s);
  timed_end(s);
  return e;
}

// Force assembly into x (solve order), in place: u is read from x.
hipError_t mr_ctx::assemble(double *finish_msd, hipStream_t s) {
  timed_begin(MR_KF_ASSEMBLE, s);
  hipError_t e = launch_assemble((int)n_nodes, d_mptr.ptr, d_ment.ptr, d_minv.ptr, d_h.ptr, d_x.ptr,
                                 d_x.ptr, params.tau, d_pairs.ptr, n_pairs, d_partials.ptr,
                                 finish_msd, d_active.ptr, s);
  timed_end(s);
  return e;
}

// h (solve order) and b (solve order, in x) at u (natural order).
hipError_t mr_ctx::force(const double2 *u, hipStream_t s) {
  hipError_t e = launch_to_solve_order((int)n_nodes, u, d_iperm.ptr, d_x.ptr, s);
  if (e == hipSuccess) e = sample(false, s);
  return e == hipSuccess ? assemble(nullptr, s) : e;
}

// One iteration u <- S^-1 (u - tau f(u)).  Sampling, assembly and the warp
// read the displacements in solve order from x, which the previous
// iteration's backward solve left there; with `x_holds_u` false (the first
// iteration of a run) u is permuted into x first.  The new displacements go to
// x and, with `write_u`, also to u (natural order).  `*pending`, when set, is
// the MSD output for the current displacements: its warp shares the sample
// launch and its final sum the assembly.  On return `*pending` is `msd_out`
// (the MSD of the new u, to be produced by the next iteration or by
// finish_pending, which needs u written).
hipError_t mr_ctx::iterate(double2 *u, double *msd_out, double **pending, bool x_holds_u,
                           bool write_u, hipStream_t s) {
  double *msd_now = *pending;
  *pending = nullptr;
  hipError_t e = hipSuccess;
  if (!x_holds_u) e = launch_to_solve_order((int)n_nodes, u, d_iperm.ptr, d_x.ptr, s);
  if (e == hipSuccess) e = sample(msd_now != nullptr, s);
  const AssembleArgs fuse{d_mptr.ptr, d_ment.ptr, d_minv.ptr,    d_h.ptr,
                          d_x.ptr,    d_upper_rows.ptr, (int32_t)d_upper_rows.count, n_pairs,
                          params.tau, d_pairs.ptr, d_partials.ptr, msd_now, d_active.ptr};
  if (e == hipSuccess && !fuse_first) e = assemble(msd_now, s);
  if (e == hipSuccess) e = solve(d_x.ptr, write_u ? u : nullptr, s, fuse_first ? &fuse : nullptr);
  if (e == hipSuccess) *pending = msd_out;
  return e;
}

hipError_t mr_ctx::finish_pending(const double2 *u, double **pending, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (*pending) e = warp(u, *pending, nullptr, s);
  *pending = nullptr;
  return e;
}

hipError_t mr_ctx::warp(const double2 *u, double *msd, float *warped, hipStream_t s) {
  timed_begin(MR_KF_WARP, s);
  hipError_t e = launch_warp_partials(d_tiles.ptr, n_tiles, u, d_tile_nodes.ptr,
                                      d_tile_pbc.ptr, d_tile_loc.ptr, d_coef.ptr,
                                      d_re.ptr, warped, d_partials.ptr, d_flags.ptr, s);
  if (e == hipSuccess) e = launch_msd_finish(d_pairs.ptr, n_pairs, d_partials.ptr, msd, s);
  timed_end(s);
  return e;
}

int mr_ctx::check_flags() {
  if (host_flags && *host_flags) {
    const unsigned f = *host_flags;
    *host_flags = 0;
    hipMemsetAsync(d_flags.ptr, 0, sizeof(unsigned), nullptr);
    return fail(MR_ENONFINITE, f & kFlagNonFiniteNode
                                   ? "a non-finite or out-of-range node displacement was met"
                                   : "a non-finite or out-of-range pixel displacement was met");
  }
  return MR_OK;
}

void mr_ctx::post_flags(hipStream_t s) {
  if (host_flags) hipMemcpyAsync(host_flags, d_flags.ptr, sizeof(unsigned), hipMemcpyDeviceToHost, s);
}

mr_ctx::~mr_ctx() {
  if (graph_exec) hipGraphExecDestroy(graph_exec);
  for (auto &p : pending) {
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  if (host_flags) hipHostFree(host_flags);
}

// Column-major copies of the row-major block panels (same offsets): entry
// (k, j) of block B's m x b panel moves from poff + k b + j to poff + j m + k.
static void transpose_panels(const std::vector<DevBlock> &blocks, const std::vector<double> &prow,
                             std::vector<double> &pcol) {
  for (const DevBlock &B : blocks) {
    const int64_t b = B.r1 - B.r0, m = B.m;
    for (int64_t k = 0; k < m; ++k)
      for (int64_t j = 0; j < b; ++j) pcol[B.poff + j * m + k] = prow[B.poff + k * b + j];
  }
}

// Uploads tables, operators and the factor of every pair into packed device
// arrays, and builds the work lists.
int mr_ctx::upload_all(hipStream_t s) {
  n_nodes = n_tris = n_pix = 0;
  dpairs.resize(n_pairs);
  std::vector<NodeItem> items;
  std::vector<TileItem> tiles;
  std::vector<int32_t> tile_tri;
  std::vector<uint8_t> tile_loc;
  for (int p = 0; p < n_pairs; ++p) {
    const PairHost &h = host[p];
    DevPair &d = dpairs[p];
    d.height = h.height;
    d.width = h.width;
    d.pix_off = n_pix;
    d.node_off = (int32_t)n_nodes;
    d.n = h.n;
    d.tri_off = (int32_t)n_tris;
    d.nt = h.nt;
    d.tile_off = (int32_t)tiles.size();
    d.tiles_x = (h.width + kTile - 1) / kTile;
    const int ty = (h.height + kTile - 1) / kTile;
    d.n_tiles = d.tiles_x * ty;
    d.active = 1;
    for (int y = 0; y < ty; ++y)
      for (int x = 0; x < d.tiles_x; ++x) {
        // the tile's distinct triangles (T6 over its pixels inside the image),
        // ascending, and each pixel's position among them
        const int y0 = y * kTile, x0 = x * kTile;
        int32_t ids[kTile * kTile];
        int n_ids = 0;
        for (int r = y0; r < std::min(h.height, y0 + kTile); ++r)
          for (int c = x0; c < std::min(h.width, x0 + kTile); ++c)
            ids[n_ids++] = h.tab.t6[(size_t)r * h.width + c];
        std::sort(ids, ids + n_ids);
        const int n_ent = (int)(std::unique(ids, ids + n_ids) - ids);
        if ((int64_t)tile_tri.size() + n_ent >= (int64_t)INT32_MAX)
          return fail(MR_EINVAL, "too many pixel-tile triangle entries");
        tiles.push_back({p, y0, x0, 1, (int32_t)tile_tri.size(), n_ent, h.height, h.width,
                         d.pix_off});
        tile_tri.insert(tile_tri.end(), ids, ids + n_ent);
        const size_t lo = tile_loc.size();
        tile_loc.resize(lo + kTile * kTile, 0);
        for (int r = y0; r < std::min(h.height, y0 + kTile); ++r)
          for (int c = x0; c < std::min(h.width, x0 + kTile); ++c) {
            const int32_t t = h.tab.t6[(size_t)r * h.width + c];
            tile_loc[lo + (r - y0) * kTile + (c - x0)] =
                (uint8_t)(std::lower_bound(ids, ids + n_ent, t) - ids);
          }
      }
    d.item_off = (int32_t)items.size();
    for (int b = 0; b < h.n; b += kNodeChunk)
      items.push_back({p, d.node_off + b, d.node_off + std::min(h.n, b + kNodeChunk), 1});
    d.n_items = (int32_t)items.size() - d.item_off;
    n_nodes += h.n;
    n_tris += h.nt;
    n_pix += (int64_t)h.height * h.width;
  }
  if (n_nodes >= INT32_MAX / 2 || n_tris >= INT32_MAX / 2)
    return fail(MR_EINVAL, "too many nodes or triangles in one context");
  n_node_items = (int)items.size();
  n_tiles = (int)tiles.size();
  // packed node and triangle data
  std::vector<int2> xy(n_nodes);
  std::vector<int4> tri(n_tris);
  std::vector<int32_t> t6(n_pix), iperm(n_nodes), perm(n_nodes);
  std::vector<int32_t> mptr(n_nodes + 1, 0);
  std::vector<uint32_t> ment;
  std::vector<float> minv(n_nodes);
  std::vector<DevBlock> blocks;
  std::vector<int32_t> block_pair;              // pair of each block
  std::vector<int64_t> cptr(n_nodes + 1, 0);
  std::vector<int32_t> cidx, below;
  std::vector<double> dcol, drow, prow;
  int max_fl = 0, max_bl = 0;
  for (int p = 0; p < n_pairs; ++p) {
    max_fl = std::max(max_fl, host[p].plan.apex_level);
    max_bl = std::max(max_bl, host[p].plan.apex_level);
  }
  std::vector<int32_t> apex_rows_g;
  std::vector<int64_t> apex_cptr_g(1, 0);
  std::vector<int32_t> apex_cidx_g;
  std::vector<ApexFwdItem> apex_fitems;
  std::vector<ApexBwdItem> apex_bitems;
  std::vector<int2> apex_rng;
  std::vector<ApexRow> apex_arow;
  int64_t apex_xf_total = 0, apex_xb_total = 0, apex_part_total = 0;
  int32_t apex_path_max = 0;
  std::vector<int32_t> upper_rows;              // solve rows outside the first forward level
  apex_xf_base.assign(n_pairs, 0);
  apex_xb_base.assign(n_pairs, 0);
  std::vector<std::vector<int2>> fwd_lv(max_fl), bwd_lv(max_bl);
  std::vector<int32_t> fwd_lds_v(max_fl, 0), bwd_lds_v(max_bl, 0);
  std::vector<int32_t> fwd_bp_v(max_fl, 64), bwd_bp_v(max_bl, 64);
  std::vector<uint8_t> bwd_split_v(max_bl, 0);
  std::vector<int32_t> fwd_direct_v(max_fl, 0), bwd_direct_v(max_bl, 0);
  std::vector<int32_t> fwd_maxb_v(max_fl, 0), bwd_maxb_v(max_bl, 0);
  int32_t n_partials = 0, n_counters = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const PairHost &h = host[p];
    const DevPair &d = dpairs[p];
    const int32_t no = d.node_off;
    for (int i = 0; i < h.n; ++i) xy[no + i] = make_int2(h.xy[2 * i], h.xy[2 * i + 1]);
    for (int t = 0; t < h.nt; ++t)
      tri[d.tri_off + t] = make_int4(no + h.tri[3 * t], no + h.tri[3 * t + 1], no + h.tri[3 * t + 2], 0);
    std::copy(h.tab.t6.begin(), h.tab.t6.end(), t6.begin() + d.pix_off);
    for (int i = 0; i < h.n; ++i) {
      iperm[no + i] = no + h.iperm[i];
      perm[no + i] = no + h.perm[i];
    }
    // force operator rows and columns in solve order (row k is node perm[k];
    // h is sampled in solve order): f_i = sum_j (24 M_ij) h_j / (4 * 6 m_i),
    // i.e. the mass row divided by the lumped mass, with 6 m_i = t5_i; the
    // columns keep the row order of the natural pattern.  An entry is one
    // word, the column's offset from the row (16 bits, signed) above the
    // integer numerator 24 M_ij (16 bits); a row with an entry outside those
    // ranges (a separator node far from a neighbour in solve order) stores
    // each entry as two words, the column and the numerator as FP32, and is
    // flagged by bit 31 of its mptr.
    std::vector<std::pair<int32_t, int64_t>> ent;     // one row's (column, numerator)
    for (int k = 0; k < h.n; ++k) {
      const int i = h.perm[k];
      const int32_t row = no + k;
      ent.clear();
      double den = 1.0;
      if (params.force_mode == MR_FORCE_NODAL) {
        ent.push_back({row, 1});
      } else {
        den = 4.0 * (double)h.tab.t5[i];
        for (int64_t q = h.tab.t3_ptr[i]; q < h.tab.t3_ptr[i + 1]; ++q)
          ent.push_back({no + h.iperm[h.tab.t3_idx[q]], h.mval[q]});
      }
      minv[row] = (float)(1.0 / den);
      bool narrow = true;
      for (const auto &e : ent)
        narrow = narrow && std::abs(e.first - row) <= 32767 && e.second >= 0 && e.second < 65536;
      if ((int64_t)ment.size() + 2 * (int64_t)ent.size() >= (int64_t)INT32_MAX)
        return fail(MR_EINVAL, "force operator too large");
      mptr[row] = (int32_t)ment.size() | (narrow ? 0 : (int32_t)0x80000000u);
      for (const auto &e : ent) {
        if (narrow) {
          ment.push_back(((uint32_t)(uint16_t)(int16_t)(e.first - row) << 16) | (uint32_t)e.second);
        } else {
          const float num = (float)e.second;
          uint32_t bits;
          std::memcpy(&bits, &num, sizeof bits);
          ment.push_back((uint32_t)e.first);
          ment.push_back(bits);
        }
      }
    }
    mptr[no + h.n] = (int32_t)ment.size();
    // solve plan, shifted to global rows
    const SolvePlan &pl = h.plan;
    const int64_t doff = (int64_t)dcol.size();
    const int64_t poff = (int64_t)prow.size();
    const int64_t uoff = (int64_t)below.size();
    dense_off.push_back(doff);
    panel_off.push_back(poff);
    const int32_t boff = (int32_t)blocks.size();
    for (size_t k = 0; k < pl.blocks.size(); ++k) {
      const SolveBlock &B = pl.blocks[k];
      const int32_t m = (int32_t)(pl.below_ptr[k + 1] - pl.below_ptr[k]);
      const int32_t b = B.r1 - B.r0;
      if (b > kBlockMax) return fail(MR_EINVAL, "solve block larger than the kernel limit");
      // panel rows per forward slice / backward chunk
      const int64_t nd = (int64_t)b * (b + 1) / 2;
      const int32_t rs = 64;
      const int32_t ns = std::max<int32_t>(1, (m + rs - 1) / rs);
      const int32_t bs = std::max<int32_t>(1, (m + bwd_split_rows - 1) / bwd_split_rows);
      DevBlock db{no + B.r0, no + B.r1, m, B.fwd_group, doff + pl.dense_off[k],
                  poff + pl.panel_off[k], uoff + pl.below_ptr[k], ns, rs, bs, 0, 0, 1};
      block_pair.push_back(p);
      if (bs > 1) {
        db.part_off = n_partials;
        db.cnt_idx = n_counters++;
        n_partials += bs * b;
      }
      const int32_t kn = std::min(rs, m);
      const int64_t lf = solve_fwd_lds_bytes(b, kn, 0), lb = solve_bwd_lds_bytes(b, kn, 0);
      if (lf + 16 * 256 > kSolveLdsBudget || lb + 16 * 256 > kSolveLdsBudget)
        return fail(MR_EINVAL, "solve block does not fit the LDS budget");
      int32_t bp = 64;
      while (bp < b) bp <<= 1;
      const int32_t id = boff + (int32_t)k;
      if (pl.is_apex[k] || B.fwd_level != 0)
        for (int32_t r = B.r0; r < B.r1; ++r) upper_rows.push_back(no + r);
      if (!pl.is_apex[k]) {
        // backward levels: the forward levels below the apex, top first
        // (a parent's forward level is higher than its children's)
        const int32_t bl = max_fl - 1 - B.fwd_level;
        for (int32_t q = 0; q < ns; ++q) fwd_lv[B.fwd_level].push_back(make_int2(id, q));
        for (int32_t q = 0; q < bs; ++q) bwd_lv[bl].push_back(make_int2(id, q));
        fwd_lds_v[B.fwd_level] = std::max<int32_t>(fwd_lds_v[B.fwd_level], (int32_t)lf);
        bwd_lds_v[bl] = std::max<int32_t>(bwd_lds_v[bl], (int32_t)lb);
        fwd_bp_v[B.fwd_level] = std::max(fwd_bp_v[B.fwd_level], bp);
        bwd_bp_v[bl] = std::max(bwd_bp_v[bl], bp);
        if (bs > 1) bwd_split_v[bl] = 1;
        fwd_maxb_v[B.fwd_level] = std::max(fwd_maxb_v[B.fwd_level], b);
        bwd_maxb_v[bl] = std::max(bwd_maxb_v[bl], b);
        // LDS of the direct-staged kernels: the whole dense inverse and panel,
        // each rounded up to 16 bytes (the copies move whole 16-byte chunks)
        const int32_t direct = (int32_t)std::min<int64_t>(
            INT32_MAX, 8 * ((nd + 1) / 2 * 2 + ((int64_t)m * b + 1) / 2 * 2));
        fwd_direct_v[B.fwd_level] = std::max(fwd_direct_v[B.fwd_level], direct);
        bwd_direct_v[bl] = std::max(bwd_direct_v[bl], direct);
      }
      blocks.push_back(db);
    }
    dcol.insert(dcol.end(), pl.dinv_col.begin(), pl.dinv_col.end());
    drow.insert(drow.end(), pl.dinv_row.begin(), pl.dinv_row.end());
    prow.insert(prow.end(), pl.panel_row.begin(), pl.panel_row.end());
    for (int32_t r : pl.below_idx) below.push_back(no + r);
    // apex of this pair, in the shared numbering of apex positions
    {
      const int32_t A0 = (int32_t)apex_rows_g.size();
      const int32_t na = (int32_t)pl.apex_rows.size();
      apex_xf_base[p] = apex_xf_total;
      apex_xb_base[p] = apex_xb_total;
      for (int32_t i = 0; i < na; ++i) {
        apex_rows_g.push_back(no + pl.apex_rows[i]);
        for (int64_t q = pl.apex_cptr[i]; q < pl.apex_cptr[i + 1]; ++q)
          apex_cidx_g.push_back((int32_t)(uoff + pl.apex_cidx[q]));
        apex_cptr_g.push_back((int64_t)apex_cidx_g.size());
      }
      apex_xf_total += na ? pl.apex_xf_off[na] : 0;
      apex_xb_total += na ? pl.apex_xb_off[na] : 0;
      for (const ApexBlock &A : pl.apex_blocks) {
        const int32_t nr = A.a1 - A.a0;
        const int32_t nseg = (A.a1 - A.c0 + kApexSeg - 1) / kApexSeg;
        if (apex_part_total + (int64_t)nr * nseg >= INT32_MAX) return fail(MR_EINVAL, "apex too large");
        const int32_t pbase = (int32_t)apex_part_total;
        apex_part_total += (int64_t)nr * nseg;
        for (int32_t i = A.a0; i < A.a1; ++i)
          apex_arow.push_back({pbase + (i - A.a0), nr, (i - A.c0) / kApexSeg + 1,
                               no + pl.apex_rows[i]});
        for (int32_t q = 0; q < nseg; ++q) {
          const int32_t k0 = A.c0 + q * kApexSeg, k1 = std::min(A.a1, k0 + kApexSeg);
          for (int32_t g = A.a0; g < A.a1; g += kApexRowsPerItem) {
            const int32_t g1 = std::min(A.a1, g + kApexRowsPerItem);
            if (g1 - 1 < k0) continue;          // no row of the group reaches the segment
            apex_fitems.push_back({A0 + g, A0 + g1, A0 + k0, A0 + k1, A0 + A.c0,
                                   pbase + q * nr + (g - A.a0), p, 1,
                                   apex_xf_base[p] + pl.apex_xf_off[g]});
          }
        }
        // ancestor ranges, adjacent ones merged
        const int32_t roff = (int32_t)apex_rng.size();
        for (int32_t k = A.anc_off; k < A.anc_off + A.n_anc; ++k) {
          const ApexBlock &G = pl.apex_blocks[pl.apex_anc[k]];
          if ((int32_t)apex_rng.size() > roff && apex_rng.back().y == A0 + G.a0)
            apex_rng.back().y = A0 + G.a1;
          else
            apex_rng.push_back(make_int2(A0 + G.a0, A0 + G.a1));
        }
        const int32_t nrng = (int32_t)apex_rng.size() - roff;
        if (nrng > kApexMaxRanges) return fail(MR_EINVAL, "apex block with too many ancestor ranges");
        for (int32_t g = A.a0; g < A.a1; g += kApexRowsPerItem) {
          const int32_t g1 = std::min(A.a1, g + kApexRowsPerItem);
          const int32_t len = (A.a1 - g) + A.anc_rows;
          if (len > kApexPath) return fail(MR_EINVAL, "apex path longer than the LDS limit");
          apex_path_max = std::max(apex_path_max, len);
          apex_bitems.push_back({A0 + g, A0 + g1, A0 + A.a1, roff, nrng, len, p, 1,
                                 apex_xb_base[p] + pl.apex_xb_off[g]});
        }
      }
    }
    const int64_t co = (int64_t)cidx.size();
    for (int r = 0; r < h.n; ++r) cptr[no + r + 1] = co + pl.cptr[r + 1];
    for (int32_t k : pl.cidx) cidx.push_back((int32_t)(uoff + k));
  }
  std::vector<int2> fwd_items, bwd_items;
  fwd_ptr.assign(1, 0);
  bwd_ptr.assign(1, 0);
  for (auto &lv : fwd_lv) {
    fwd_items.insert(fwd_items.end(), lv.begin(), lv.end());
    fwd_ptr.push_back((int32_t)fwd_items.size());
  }
  for (auto &lv : bwd_lv) {
    bwd_items.insert(bwd_items.end(), lv.begin(), lv.end());
    bwd_ptr.push_back((int32_t)bwd_items.size());
  }
  fwd_lds = fwd_lds_v;
  bwd_lds = bwd_lds_v;
  fwd_bp = fwd_bp_v;
  bwd_bp = bwd_bp_v;
  bwd_split = bwd_split_v;
  fwd_direct = fwd_direct_v;
  bwd_direct = bwd_direct_v;
  fwd_maxb = fwd_maxb_v;
  bwd_maxb = bwd_maxb_v;
  fwd_nt.assign(fwd_bp.size(), 256);
  bwd_nt.assign(bwd_bp.size(), 256);
  if (below.size() >= (size_t)INT32_MAX) return fail(MR_EINVAL, "solve update buffer too large");
  nnz_factor = (int64_t)prow.size() + (int64_t)dcol.size();
  HIP_TRY(upload(d_pairs, dpairs, s));
  HIP_TRY(upload(d_node_items, items, s));
  HIP_TRY(upload(d_tiles, tiles, s));
  HIP_TRY(upload(d_tile_loc, tile_loc, s));
  HIP_TRY(upload(d_xy, xy, s));
  {
    std::vector<int2> xy_s(n_nodes);            // node corners in solve order
    for (int64_t k = 0; k < n_nodes; ++k) xy_s[k] = xy[perm[k]];
    HIP_TRY(upload(d_xy_s, xy_s, s));
  }
  HIP_TRY(upload(d_tri, tri, s));
  {
    // per pixel-tile triangle entry: the corner nodes (natural and solve
    // order) with the first corner's coordinates, and the other two corners'
    // coordinates, packed as x | y << 16 (image sides below 65536)
    auto pk = [&](int node) { return (int)((uint32_t)xy[node].x | ((uint32_t)xy[node].y << 16)); };
    std::vector<int4> tn(tile_tri.size()), tns(tile_tri.size());
    std::vector<int2> tpbc(tile_tri.size());
    for (const TileItem &ti : tiles)
      for (int32_t k = ti.ent_off; k < ti.ent_off + ti.n_ent; ++k) {
        const int4 c = tri[dpairs[ti.pair].tri_off + tile_tri[k]];
        tn[k] = make_int4(c.x, c.y, c.z, pk(c.x));
        tns[k] = make_int4(iperm[c.x], iperm[c.y], iperm[c.z], pk(c.x));
        tpbc[k] = make_int2(pk(c.y), pk(c.z));
      }
    HIP_TRY(upload(d_tile_nodes, tn, s));
    HIP_TRY(upload(d_tile_nodes_s, tns, s));
    HIP_TRY(upload(d_tile_pbc, tpbc, s));
    // per node, the slots 3 k + corner of the tile entries k it is a corner
    // of, ascending (the warp adjoint sums lambda^N in this order)
    if (3 * (int64_t)tn.size() >= (int64_t)INT32_MAX) return fail(MR_EINVAL, "too many tile entries");
    std::vector<int32_t> lptr(n_nodes + 1, 0), lidx(3 * tn.size());
    for (const int4 &t : tn) {
      ++lptr[t.x + 1];
      ++lptr[t.y + 1];
      ++lptr[t.z + 1];
    }
    for (int64_t v = 0; v < n_nodes; ++v) lptr[v + 1] += lptr[v];
    {
      std::vector<int32_t> cur(lptr.begin(), lptr.end() - 1);
      for (size_t k = 0; k < tn.size(); ++k) {
        lidx[cur[tn[k].x]++] = (int32_t)(3 * k);
        lidx[cur[tn[k].y]++] = (int32_t)(3 * k + 1);
        lidx[cur[tn[k].z]++] = (int32_t)(3 * k + 2);
      }
    }
    HIP_TRY(upload(d_lam_ptr, lptr, s));
    HIP_TRY(upload(d_lam_idx, lidx, s));
  }
  HIP_TRY(upload(d_t6, t6, s));
  HIP_TRY(upload(d_iperm, iperm, s));
  HIP_TRY(upload(d_perm, perm, s));
  HIP_TRY(upload(d_mptr, mptr, s));
  HIP_TRY(upload(d_ment, ment, s));
  HIP_TRY(upload(d_minv, minv, s));
  HIP_TRY(upload(d_blocks, blocks, s));
  HIP_TRY(upload(d_block_pair, block_pair, s));
  {
    // every pair active; the last entry flags that some pair is retired
    std::vector<int32_t> act(n_pairs + 1, 1);
    act[n_pairs] = 0;
    HIP_TRY(upload(d_active, act, s));
  }
  n_apex_rows = (int64_t)apex_rows_g.size();
  HIP_TRY(upload(d_upper_rows, upper_rows, s));
  HIP_TRY(upload(d_apex_rows, apex_rows_g, s));
  HIP_TRY(upload(d_apex_cptr, apex_cptr_g, s));
  HIP_TRY(upload(d_apex_cidx, apex_cidx_g, s));
  HIP_TRY(upload(d_apex_fitems, apex_fitems, s));
  HIP_TRY(upload(d_apex_bitems, apex_bitems, s));
  HIP_TRY(upload(d_apex_rng, apex_rng, s));
  HIP_TRY(upload(d_apex_arow, apex_arow, s));
  HIP_TRY(d_apex_y.alloc(std::max<int64_t>(n_apex_rows, 1)));
  apex_bwd_lds = 16 * std::max(apex_path_max, 1);
  HIP_TRY(d_apex_xf.alloc(std::max<int64_t>(apex_xf_total, 1)));
  HIP_TRY(d_apex_xb.alloc(std::max<int64_t>(apex_xb_total, 1)));
  HIP_TRY(d_apex_part.alloc(std::max<int64_t>(apex_part_total, 1)));
  HIP_TRY(d_apex_t.alloc(std::max<int64_t>(n_apex_rows, 1)));
  for (int p = 0; p < n_pairs; ++p) {
    const SolvePlan &pl = host[p].plan;
    if (!pl.apex_xf.empty())
      HIP_TRY(hipMemcpyAsync(d_apex_xf.ptr + apex_xf_base[p], pl.apex_xf.data(),
                             pl.apex_xf.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (!pl.apex_xb.empty())
      HIP_TRY(hipMemcpyAsync(d_apex_xb.ptr + apex_xb_base[p], pl.apex_xb.data(),
                             pl.apex_xb.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(upload(d_fwd_items, fwd_items, s));
  HIP_TRY(upload(d_bwd_items, bwd_items, s));
  HIP_TRY(d_partials2.alloc(std::max(n_partials, 1)));
  HIP_TRY(d_blk_counters.alloc(std::max(n_counters, 1)));
  HIP_TRY(hipMemsetAsync(d_blk_counters.ptr, 0, sizeof(unsigned) * std::max(n_counters, 1), s));
  HIP_TRY(upload(d_cptr, cptr, s));
  HIP_TRY(upload(d_cidx, cidx, s));
  HIP_TRY(upload(d_below, below, s));
  HIP_TRY(upload(d_prow, prow, s));
  {
    std::vector<double> pcol(prow.size());
    transpose_panels(blocks, prow, pcol);
    HIP_TRY(upload(d_pcol, pcol, s));
  }
  HIP_TRY(d_ybuf.alloc(n_nodes));
  HIP_TRY(d_upd.alloc(std::max<size_t>(below.size(), 1)));
  HIP_TRY(upload(d_dcol, dcol, s));
  HIP_TRY(upload(d_drow, drow, s));
  HIP_TRY(d_coef.alloc(n_pix));
  HIP_TRY(d_re.alloc(n_pix));
  HIP_TRY(d_rho.alloc(n_nodes));
  HIP_TRY(d_rho_s.alloc(n_nodes));
  HIP_TRY(d_h.alloc(n_nodes));
  HIP_TRY(d_x.alloc(n_nodes));
  HIP_TRY(d_partials.alloc(std::max(n_tiles, 1)));
  HIP_TRY(d_flags.alloc(1));
  HIP_TRY(d_msd_tmp.alloc(n_pairs));
  HIP_TRY(hipMemsetAsync(d_flags.ptr, 0, sizeof(unsigned), s));
  HIP_TRY(hipHostMalloc((void **)&host_flags, sizeof(unsigned), hipHostMallocDefault));
  *host_flags = 0;
  return MR_OK;
}

// Re-uploads the numeric values of one pair's factor (same structure).
int mr_ctx::upload_factor(int p, hipStream_t s) {
  const SolvePlan &pl = host[p].plan;
  auto put = [&](double *dst, const std::vector<double> &v) {
    return v.empty() ? hipSuccess
                     : hipMemcpyAsync(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s);
  };
  HIP_TRY(put(d_prow.ptr + panel_off[p], pl.panel_row));
  {
    // column-major copy of this pair's panels (blocks are stored per pair in order)
    std::vector<double> pcol(pl.panel_row.size());
    std::vector<DevBlock> bl(pl.blocks.size());
    for (size_t k = 0; k < pl.blocks.size(); ++k) {
      bl[k].r0 = pl.blocks[k].r0;
      bl[k].r1 = pl.blocks[k].r1;
      bl[k].m = (int32_t)(pl.below_ptr[k + 1] - pl.below_ptr[k]);
      bl[k].poff = pl.panel_off[k];
    }
    transpose_panels(bl, pl.panel_row, pcol);
    HIP_TRY(put(d_pcol.ptr + panel_off[p], pcol));
  }
  HIP_TRY(put(d_apex_xf.ptr + apex_xf_base[p], pl.apex_xf));
  HIP_TRY(put(d_apex_xb.ptr + apex_xb_base[p], pl.apex_xb));
  HIP_TRY(put(d_dcol.ptr + dense_off[p], pl.dinv_col));
  HIP_TRY(put(d_drow.ptr + dense_off[p], pl.dinv_row));
  HIP_TRY(hipStreamSynchronize(s));
  return MR_OK;
}

int64_t mr_ctx::device_bytes() const {
  return (int64_t)(d_pairs.bytes() + d_node_items.bytes() + d_tiles.bytes() + d_xy.bytes() +
                   d_tri.bytes() + d_t6.bytes() + d_tile_nodes.bytes() +
                   d_tile_nodes_s.bytes() + d_tile_pbc.bytes() + d_tile_loc.bytes() + d_lam_ptr.bytes() +
                   d_lam_idx.bytes() + d_iperm.bytes() + d_perm.bytes() +
                   d_coef.bytes() + d_re.bytes() + d_rho.bytes() + d_rho_s.bytes() +
                   d_x_sptr.bytes() + d_x_opp.bytes() + d_x_rptr.bytes() + d_x_ridx.bytes() +
                   d_x_u0.bytes() + d_x_rec.bytes() +
                   d_xy_s.bytes() + d_mptr.bytes() +
                   d_ment.bytes() + d_minv.bytes() + d_h.bytes() + d_x.bytes() +
                   d_blocks.bytes() + d_fwd_items.bytes() + d_bwd_items.bytes() + d_cptr.bytes() +
                   d_cidx.bytes() + d_below.bytes() + d_partials2.bytes() + d_prow.bytes() +
                   d_upd.bytes() + d_dcol.bytes() + d_drow.bytes() + d_partials.bytes() +
                   d_pcol.bytes() + d_ybuf.bytes() +
                   d_apex_xf.bytes() + d_apex_xb.bytes() + d_apex_part.bytes() +
                   d_apex_cidx.bytes() + d_apex_arow.bytes() + d_apex_fitems.bytes() +
                   d_apex_bitems.bytes() +
                   d_msd_tmp.bytes() + d_flags.bytes());
}

// B-spline coefficients (B^-1 along rows, then columns) of one pair's FP32 or
// FP64 image; B is symmetric, so the same map is its own adjoint.
// Thomas tables of every image side of the context, back to back, and a
// scratch image of the largest pair (built once; the prefilter launches of
// all pairs share them in stream order).
int mr_ctx::upload_prefilter_tables(hipStream_t s) {
  std::vector<double2> all;
  int64_t max_pix = 1;
  for (const DevPair &d : dpairs) {
    for (int N : {d.height, d.width})
      if (!thomas_off.count(N)) {
        thomas_off[N] = (int64_t)all.size();
        const std::vector<double2> t = thomas_table(N);
        all.insert(all.end(), t.begin(), t.end());
      }
    max_pix = std::max<int64_t>(max_pix, (int64_t)d.height * d.width);
  }
  HIP_TRY(upload(d_thomas, all, s));
  HIP_TRY(d_prefilter_tmp.alloc(max_pix));
  // work items of the batched passes: 64 rows / columns of one pair each
  std::vector<PrefItem> rows, cols;
  for (int p = 0; p < n_pairs; ++p) {
    const DevPair &d = dpairs[p];
    const int32_t tw = (int32_t)thomas_off.at(d.width), th = (int32_t)thomas_off.at(d.height);
    for (int32_t r = 0; r < d.height; r += 64) rows.push_back(PrefItem{p, r, tw, th});
    for (int32_t c = 0; c < d.width; c += 64) cols.push_back(PrefItem{p, c, tw, th});
  }
  HIP_TRY(upload(d_pref_rows, rows, s));
  HIP_TRY(upload(d_pref_cols, cols, s));
  HIP_TRY(hipStreamSynchronize(s));            // the host vectors go out of scope
  return MR_OK;
}

int mr_ctx::prefilter_any(int p, const float *img_f, const double *img_d, float *coef_out,
                          hipStream_t s) {
  const DevPair &d = dpairs[p];
  HIP_TRY(launch_prefilter(img_f, img_d, d_prefilter_tmp.ptr, coef_out, d.height, d.width,
                           d_thomas.ptr + thomas_off.at(d.width),
                           d_thomas.ptr + thomas_off.at(d.height), s));
  return MR_OK;
}

int mr_ctx::prefilter_pair(int p, const float *img, float *coef_out, hipStream_t s) {
  return prefilter_any(p, img, nullptr, coef_out, s);
}

int mr_ctx::prefilter_pair_d(int p, const double *img, float *coef_out, hipStream_t s) {
  return prefilter_any(p, nullptr, img, coef_out, s);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" const char *mesh_reg_last_error(void) { return g_last_error.c_str(); }

static int check_ctx(mr_ctx *c, bool need_device) {
  if (!c) return fail(MR_EINVAL, "null context");
  if (need_device && c->host_only) return fail(MR_ESTATE, "context was built host-only");
  return MR_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Entries of X one level may add to the apex, per pair: moving a level into
// the apex saves two launches of the whole batch (a fixed latency) and costs
// streaming its entries of X for every pair, so the budget shrinks with the
// number of pairs, down to 2^18 (measured on a 256-pair batch: the top levels
// of the block tree are worth an apex of 1-2 thousand rows per pair).
static int64_t apex_level_budget(int32_t n_pairs) {
  return std::max<int64_t>(int64_t(1) << 18, (int64_t(1) << 21) / std::max(1, n_pairs));
}

extern "C" int mesh_reg_init(const mr_pair *pairs, int32_t n_pairs, const mr_params *params,
                             void *stream, mr_ctx **out) {
  const TraceRange range_("mesh_reg_init");
  if (!out) return fail(MR_EINVAL, "out is null");
  *out = nullptr;
  if (!pairs || n_pairs < 1 || !params) return fail(MR_EINVAL, "need pairs, n_pairs >= 1 and params");
  if (!(params->tau > 0.0) || !std::isfinite(params->tau)) return fail(MR_EINVAL, "tau must be finite and > 0");
  if (params->force_mode != MR_FORCE_P1 && params->force_mode != MR_FORCE_NODAL)
    return fail(MR_EINVAL, "unknown force_mode");
  {
    const int32_t k = params->solve_kernel;
    if (k != 0 && k != 1 && k != 8 && k != 16 && k != 32 && k != 33 && k != 34 && k != 64 &&
        k != 128 && k != 256 && k != 512 && k != 1024)
      return fail(MR_EINVAL,
                  "solve_kernel must be 0, 1, 8, 16, 32, 33, 34, 64, 128, 256, 512 or 1024");
  }
  const bool host_only = (params->flags & MR_FLAG_HOST_ONLY) != 0;
  for (int p = 0; p < n_pairs; ++p) {
    const mr_pair &q = pairs[p];
    if (!(q.alpha >= 0.0) || !std::isfinite(q.alpha))
      return fail(MR_EINVAL, "pair " + std::to_string(p) + ": alpha must be finite and >= 0");
    if (!q.node_xy || !q.tris) return fail(MR_EINVAL, "pair " + std::to_string(p) + ": null mesh");
    if (q.n_nodes < 3 || q.n_tris < 1 || q.height < 1 || q.width < 1)
      return fail(MR_EINVAL, "pair " + std::to_string(p) + ": empty mesh or image");
    if (q.height > 65535 || q.width > 65535)
      return fail(MR_EINVAL, "pair " + std::to_string(p) + ": image sides must be below 65536");
    if ((int64_t)q.height * q.width > INT32_MAX)
      return fail(MR_EINVAL, "pair " + std::to_string(p) + ": more than 2^31 - 1 pixels");
    if (!host_only && (!q.te || !q.re))
      return fail(MR_EINVAL, "pair " + std::to_string(p) + ": null te/re");
  }
  mr_ctx *c = new (std::nothrow) mr_ctx();
  if (!c) return fail(MR_ENOMEM, "context allocation failed");
  c->params = *params;
  c->n_pairs = n_pairs;
  c->host_only = host_only;
  c->host.resize(n_pairs);
  OrderOptions opt;
  // automatic apex: at most 1024 rows per pair in a batch, a level joining
  // while the inverse entries it adds stay within the per-level budget
  // (measured on a 256-pair batch); a single pair leaves the GPU idle on its
  // small top levels, so there the apex takes up to 16384 rows whatever their
  // entries (on the 2048^2 pair 15,951 rows against 6,722 under the budget:
  // 0.36 -> 0.30 ms per iteration; smaller pairs reach the tree's second
  // level first)
  opt.apex_max = params->apex_rows > 0 ? params->apex_rows
                 : params->apex_rows < 0 ? 0
                 : n_pairs > 1           ? 1024
                                         : 16384;
  opt.apex_level_entries = (params->apex_rows > 0 || n_pairs == 1) ? (int64_t(1) << 40)
                                                                   : apex_level_budget(n_pairs);
  // splitting a backward panel over workgroups costs a device-scope fence per
  // workgroup; it only pays when a single pair leaves most of the GPU idle
  c->bwd_split_rows = params->bwd_split_rows > 0 ? std::max(8, params->bwd_split_rows)
                      : n_pairs == 1 ? 128 : (1 << 30);
  for (int p = 0; p < n_pairs; ++p) {
    const mr_pair &q = pairs[p];
    PairHost &h = c->host[p];
    h.height = q.height;
    h.width = q.width;
    h.n = q.n_nodes;
    h.nt = q.n_tris;
    h.alpha = q.alpha;
    h.xy.assign(q.node_xy, q.node_xy + 2 * (size_t)q.n_nodes);
    h.tri.assign(q.tris, q.tris + 3 * (size_t)q.n_tris);
  }
  // pairs are prepared independently, on up to 32 host threads
  std::vector<std::string> errs(n_pairs);
  std::vector<char> not_spd(n_pairs, 0);
  {
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int p = next++; p < n_pairs; p = next++) {
        bool ns = false;
        errs[p] = prepare_pair(c->host[p], params->tau, opt, &ns);
        not_spd[p] = ns;
      }
    };
    const int nt = std::max(1, std::min<int>({n_pairs, 32, (int)std::thread::hardware_concurrency()}));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
  }
  for (int p = 0; p < n_pairs; ++p)
    if (!errs[p].empty()) {
      delete c;
      return fail(not_spd[p] ? MR_ENOTSPD : MR_EINVAL, "pair " + std::to_string(p) + ": " + errs[p]);
    }
  if (host_only) {
    *out = c;
    return MR_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(MR_EHIP, "no HIP device available");
  }
  if ((rc = resolve_scratch(c->device)) != MR_OK) {
    delete c;
    return rc;
  }
  if ((rc = c->upload_all(s)) != MR_OK || (rc = c->upload_prefilter_tables(s)) != MR_OK) {
    delete c;
    return rc;
  }
  for (int p = 0; p < n_pairs; ++p) {
    const DevPair &d = c->dpairs[p];
    float *coef_re = c->d_re.ptr + d.pix_off;  // temporarily holds Re's coefficients
    if ((rc = c->prefilter_pair(p, pairs[p].te, c->d_coef.ptr + d.pix_off, s)) != MR_OK ||
        (rc = c->prefilter_pair(p, pairs[p].re, coef_re, s)) != MR_OK) {
      delete c;
      return rc;
    }
  }
  hipError_t e = launch_sample_rho(c->d_node_items.ptr, c->n_node_items, c->d_pairs.ptr,
                                   c->d_xy.ptr, c->d_re.ptr, c->d_rho.ptr, s);
  if (e == hipSuccess)                   // the same samples in solve order
    e = launch_sample_rho(c->d_node_items.ptr, c->n_node_items, c->d_pairs.ptr, c->d_xy_s.ptr,
                          c->d_re.ptr, c->d_rho_s.ptr, s);
  // the reference pixels themselves replace its coefficients
  for (int p = 0; p < n_pairs && e == hipSuccess; ++p) {
    const DevPair &d = c->dpairs[p];
    e = hipMemcpyAsync(c->d_re.ptr + d.pix_off, pairs[p].re,
                       sizeof(float) * (size_t)d.height * d.width, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete c;
    return fail(MR_EHIP, std::string("init: ") + hipGetErrorString(e));
  }
  c->fuse_first = !(params->flags & MR_FLAG_SEPARATE_ASSEMBLY);
  if (params->solve_kernel != 0) {
    c->force_solve_kernel(params->solve_kernel);
  } else if (!(params->flags & MR_FLAG_NO_TUNE) && (rc = c->tune(s)) != MR_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MR_OK;
}

// The launches of n_iter iterations (no host synchronisation, no memsets, so
// the sequence can be captured in a graph).
int mr_ctx::step(double2 *u, int32_t n_iter, double *msd_trace, hipStream_t s) {
  double *pending = nullptr;
  for (int k = 0; k < n_iter; ++k)
    HIP_TRY(iterate(u, msd_trace ? msd_trace + (size_t)k * n_pairs : nullptr, &pending, k > 0,
                    k + 1 == n_iter, s));
  HIP_TRY(finish_pending(u, &pending, s));
  return MR_OK;
}

// Enqueues `enqueue(s)` eagerly, or replays the cached graph of it when
// MR_FLAG_GRAPH is set (captured on first use for this key: the variant, its
// step parameters and the arguments).
template <typename F>
static int replay(mr_ctx *c, int mode, double tau, double lam, const void *u, int32_t n_iter,
                  const double *msd_trace, hipStream_t s, F &&enqueue) {
  // graphs cannot be captured on the legacy default stream
  const bool use_graph = (c->params.flags & MR_FLAG_GRAPH) && !c->timing && n_iter > 0 && s;
  if (!use_graph) return enqueue(s);
  if (!c->graph_exec || c->graph_u != u || c->graph_trace != msd_trace ||
      c->graph_iters != n_iter || c->graph_stream != s || c->graph_mode != mode ||
      c->graph_tau != tau || c->graph_lam != lam) {
    if (c->graph_exec) {
      hipGraphExecDestroy(c->graph_exec);
      c->graph_exec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    HIP_TRY(e);
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIP_TRY(e);
    c->graph_u = u;
    c->graph_trace = msd_trace;
    c->graph_iters = n_iter;
    c->graph_stream = s;
    c->graph_mode = mode;
    c->graph_tau = tau;
    c->graph_lam = lam;
  }
  HIP_TRY(hipGraphLaunch(c->graph_exec, s));
  return MR_OK;
}

// n_iter iterations of the semi-implicit scheme, eagerly or from the graph.
static int run_iterations(mr_ctx *c, double *u, int32_t n_iter, double *msd_trace, hipStream_t s) {
  double2 *u2 = reinterpret_cast<double2 *>(u);
  return replay(c, 0, 0.0, 0.0, u, n_iter, msd_trace, s,
                [&](hipStream_t st) { return c->step(u2, n_iter, msd_trace, st); });
}

extern "C" int mesh_reg_step(mr_ctx *c, double *u, int32_t n_iter, double *msd_trace,
                             void *stream) {
  const TraceRange range_("mesh_reg_step");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || n_iter < 0) return fail(MR_EINVAL, "u must be a 16-byte aligned device pointer; n_iter >= 0");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = run_iterations(c, u, n_iter, msd_trace, s))) return rc;
  c->post_flags(s);
  return MR_OK;
}

// Per-pair activity (1 active, 0 retired; one more entry, nonzero when some
// pair is retired) into d_active and every work descriptor.
hipError_t mr_ctx::set_active(const std::vector<int32_t> &flags, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d_active.ptr, flags.data(), sizeof(int32_t) * flags.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = launch_set_active(d_active.ptr, d_pairs.ptr, n_pairs, d_blocks.ptr, d_block_pair.ptr,
                        (int)d_blocks.count, d_node_items.ptr, n_node_items, d_tiles.ptr, n_tiles,
                        d_apex_fitems.ptr, (int)d_apex_fitems.count, d_apex_bitems.ptr,
                        (int)d_apex_bitems.count, s);
  // the flags were read from pageable host memory: finish before it goes away
  return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

// Each node's triangles (table T1: slot 3 t + corner) as their other two
// corners in cyclic order, and each node's 1-ring (table T2), for every pair
// with global ids, for the explicit variant.
int mr_ctx::upload_explicit_tables(hipStream_t s) {
  std::vector<int32_t> sptr(n_nodes + 1, 0), rptr(n_nodes + 1, 0), ridx;
  std::vector<int2> opp;
  for (int p = 0; p < n_pairs; ++p) {
    const PairHost &h = host[p];
    const int64_t no = dpairs[p].node_off;
    if ((int64_t)opp.size() + (int64_t)h.tab.t1_slot.size() > INT32_MAX ||
        (int64_t)ridx.size() + (int64_t)h.tab.t2_idx.size() > INT32_MAX)
      return fail(MR_EINVAL, "explicit variant: more than 2^31 - 1 table entries");
    for (int i = 0; i < h.n; ++i) {
      for (int64_t q = h.tab.t1_ptr[i]; q < h.tab.t1_ptr[i + 1]; ++q) {
        const int64_t t = h.tab.t1_slot[q] / 3, a = h.tab.t1_slot[q] % 3;
        const int32_t *c = &h.tri[3 * t];
        opp.push_back(make_int2((int32_t)(no + c[(a + 1) % 3]), (int32_t)(no + c[(a + 2) % 3])));
      }
      for (int64_t q = h.tab.t2_ptr[i]; q < h.tab.t2_ptr[i + 1]; ++q)
        ridx.push_back((int32_t)(no + h.tab.t2_idx[q]));
      sptr[no + i + 1] = (int32_t)opp.size();
      rptr[no + i + 1] = (int32_t)ridx.size();
    }
  }
  HIP_TRY(upload(d_x_sptr, sptr, s));
  HIP_TRY(upload(d_x_opp, opp, s));
  HIP_TRY(upload(d_x_rptr, rptr, s));
  HIP_TRY(upload(d_x_ridx, ridx, s));
  HIP_TRY(d_x_u0.alloc(n_nodes));
  HIP_TRY(d_x_rec.alloc(n_nodes));
  HIP_TRY(hipStreamSynchronize(s));
  return MR_OK;
}

// n_iter iterations of Algorithm 1 as printed, in place on u (natural order).
// Iteration k: smooth u_0 into u (not at k = 0) and sample t at u; then the
// update u_0 = u - tau r g.  After the last iteration one more smoothing
// leaves u_1^N in u.  MSD(u_1^k) (trace row k - 1) is warped by the update
// launch of iteration k and finished by the next smoothing launch; the last
// one by a warp of its own.
int mr_ctx::step_explicit(double2 *u, int32_t n_iter, double tau, double lam, double *msd_trace,
                          hipStream_t s) {
  if (n_iter == 0) return MR_OK;
  double2 *u0 = d_x_u0.ptr;
  NodeRec *rec = d_x_rec.ptr;
  for (int k = 0; k <= n_iter; ++k) {
    // rows of the trace finished here (from the previous update's tiles)
    double *fin = (msd_trace && k >= 2) ? msd_trace + (size_t)(k - 2) * n_pairs : nullptr;
    timed_begin(MR_KF_SAMPLE, s);
    const hipError_t es = launch_explicit_smooth(
        d_node_items.ptr, n_node_items, d_pairs.ptr, n_pairs, u0, u, d_x_rptr.ptr, d_x_ridx.ptr,
        lam, k > 0, k < n_iter, d_xy.ptr, d_coef.ptr, d_rho.ptr, rec, d_flags.ptr, d_partials.ptr,
        fin, s);
    timed_end(s);          // before any return, so no timer stays attached to the thread
    HIP_TRY(es);
    if (k == n_iter) break;
    const int tiles = (msd_trace && k > 0) ? n_tiles : 0;
    timed_begin(MR_KF_ASSEMBLE, s);
    const hipError_t eu = launch_explicit_update(
        d_node_items.ptr, n_node_items, d_pairs.ptr, u, rec, d_tri.ptr, d_x_sptr.ptr, d_x_opp.ptr,
        tau, u0, d_flags.ptr, d_tiles.ptr, tiles, d_tile_nodes.ptr, d_tile_pbc.ptr, d_tile_loc.ptr,
        d_coef.ptr, d_re.ptr, d_partials.ptr, s);
    timed_end(s);
    HIP_TRY(eu);
  }
  if (msd_trace) HIP_TRY(warp(u, msd_trace + (size_t)(n_iter - 1) * n_pairs, nullptr, s));
  return MR_OK;
}

extern "C" int mesh_reg_step_explicit(mr_ctx *c, double *u, int32_t n_iter, double tau,
                                      double lambda, double *msd_trace, void *stream) {
  const TraceRange range_("mesh_reg_step_explicit");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || n_iter < 0 || !std::isfinite(tau) || !(tau >= 0.0) ||
      !(lambda >= 0.0 && lambda <= 1.0))
    return fail(MR_EINVAL, "explicit: need aligned u, n_iter >= 0, finite tau >= 0 and "
                           "0 <= lambda <= 1");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  // the record array is allocated last: present only after a complete upload
  if (!c->d_x_rec.ptr && (rc = c->upload_explicit_tables(s))) return rc;
  double2 *u2 = reinterpret_cast<double2 *>(u);
  if ((rc = replay(c, 1, tau, lambda, u, n_iter, msd_trace, s, [&](hipStream_t st) {
         return c->step_explicit(u2, n_iter, tau, lambda, msd_trace, st);
       })))
    return rc;
  c->post_flags(s);
  return MR_OK;
}

extern "C" int mesh_reg_run(mr_ctx *c, double *u, int32_t max_iter, int32_t check_every,
                            double rel_tol, int32_t *iters_out, double *msd_out, void *stream) {
  const TraceRange range_("mesh_reg_run");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || max_iter < 0 || check_every < 1 || !iters_out || !msd_out ||
      !(rel_tol >= 0.0) || !std::isfinite(rel_tol))
    return fail(MR_EINVAL, "need aligned u, max_iter >= 0, check_every >= 1, finite rel_tol >= 0, "
                           "iters_out and msd_out");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int np = c->n_pairs;
  if ((int64_t)c->d_run_trace.count < np) HIP_TRY(c->d_run_trace.alloc(np));
  // MSD of the starting displacements
  std::vector<double> prev(np), now(np), final_msd(np);
  HIP_TRY(c->warp(reinterpret_cast<const double2 *>(u), c->d_run_trace.ptr, nullptr, s));
  HIP_TRY(hipMemcpyAsync(prev.data(), c->d_run_trace.ptr, sizeof(double) * np,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> active(np, 1);
  int32_t done = 0, n_active = np;
  for (int p = 0; p < np; ++p) {
    final_msd[p] = prev[p];
    iters_out[p] = 0;
  }
  while (done < max_iter && n_active > 0) {
    const int32_t chunk = std::min(check_every, max_iter - done);
    // the chunk's iterations without the per-iteration warp, then the MSD of
    // the pairs still running
    if ((rc = run_iterations(c, u, chunk, nullptr, s))) break;
    hipError_t e = c->warp(reinterpret_cast<const double2 *>(u), c->d_run_trace.ptr, nullptr, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(now.data(), c->d_run_trace.ptr, sizeof(double) * np,
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = fail(MR_EHIP, std::string("run: ") + hipGetErrorString(e));
      break;
    }
    done += chunk;
    bool retired = false;
    for (int p = 0; p < np; ++p) {
      if (!active[p]) continue;
      iters_out[p] = done;
      final_msd[p] = now[p];
      // relative decrease of the MSD over the chunk below the tolerance
      // (an increase counts as converged)
      if (!(prev[p] > 0.0) || (prev[p] - now[p]) < rel_tol * prev[p]) {
        active[p] = 0;
        --n_active;
        retired = true;
      }
      prev[p] = now[p];
    }
    if (retired && n_active > 0 && done < max_iter) {
      std::vector<int32_t> flags(active);
      flags.push_back(1);                     // some pair is retired
      e = c->set_active(flags, s);
      if (e != hipSuccess) {
        rc = fail(MR_EHIP, std::string("run: ") + hipGetErrorString(e));
        break;
      }
    }
  }
  // every pair active again for later calls
  std::vector<int32_t> all(np + 1, 1);
  all[np] = 0;
  const hipError_t e = c->set_active(all, s);
  if (rc) return rc;
  if (e != hipSuccess) return fail(MR_EHIP, std::string("run: ") + hipGetErrorString(e));
  HIP_TRY(hipMemcpyAsync(msd_out, final_msd.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->post_flags(s);
  return MR_OK;
}

extern "C" int mesh_reg_warp_msd(mr_ctx *c, const double *u, double *msd, float *warped,
                                 void *stream) {
  const TraceRange range_("mesh_reg_warp_msd");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || !msd) return fail(MR_EINVAL, "need aligned u and msd");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(c->warp(reinterpret_cast<const double2 *>(u), msd, warped, s));
  c->post_flags(s);
  return MR_OK;
}

extern "C" int mesh_reg_warp_msd_noalloc(mr_ctx *c, const double *u, double *msd, float *warped,
                                         void *stream) {
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || !msd) return fail(MR_EINVAL, "need aligned u and msd");
  if ((int64_t)c->n_tiles > (int64_t)kScratchDoubles)
    return fail(MR_EINVAL, "warp_msd_noalloc: " + std::to_string(c->n_tiles) +
                               " pixel tiles exceed the static scratch of " +
                               std::to_string(kScratchDoubles) + " tiles (" +
                               std::to_string(kScratchDoubles * kTile * kTile) + " pixels)");
  double *partials = scratch_ptr(c->device);
  if (!partials) return fail(MR_ESTATE, "warp_msd_noalloc: no scratch address for this device");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  // every tile of an active pair writes its own partial before the finish
  // reads it (all pairs are active outside mesh_reg_run), so nothing needs
  // clearing; no kernel timing here (it would create events)
  hipError_t e = launch_warp_partials(c->d_tiles.ptr, c->n_tiles,
                                      reinterpret_cast<const double2 *>(u), c->d_tile_nodes.ptr,
                                      c->d_tile_pbc.ptr, c->d_tile_loc.ptr,
                                      c->d_coef.ptr, c->d_re.ptr, warped, partials,
                                      c->d_flags.ptr, s);
  if (e == hipSuccess) e = launch_msd_finish(c->d_pairs.ptr, c->n_pairs, partials, msd, s);
  HIP_TRY(e);
  c->post_flags(s);
  return MR_OK;
}

extern "C" int mesh_reg_force(mr_ctx *c, const double *u, float *h, double *b, void *stream) {
  const TraceRange range_("mesh_reg_force");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!u || !aligned16(u) || (b && !aligned16(b)) || (h && ((uintptr_t)h & 7u)))
    return fail(MR_EINVAL, "need aligned u (and h, b)");
  if ((rc = c->check_flags())) return rc;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(c->force(reinterpret_cast<const double2 *>(u), s));
  if (h) HIP_TRY(launch_h_from_solve_order((int)c->n_nodes, c->d_h.ptr, c->d_iperm.ptr,
                                           reinterpret_cast<float2 *>(h), s));
  if (b) HIP_TRY(launch_from_solve_order((int)c->n_nodes, c->d_x.ptr, c->d_iperm.ptr,
                                         reinterpret_cast<double2 *>(b), s));
  c->post_flags(s);
  return MR_OK;
}

extern "C" int mesh_reg_solve(mr_ctx *c, const double *b, double *x, void *stream) {
  const TraceRange range_("mesh_reg_solve");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!b || !x || !aligned16(b) || !aligned16(x)) return fail(MR_EINVAL, "need aligned b and x");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_to_solve_order((int)c->n_nodes, reinterpret_cast<const double2 *>(b),
                                c->d_iperm.ptr, c->d_x.ptr, s));
  HIP_TRY(c->solve(c->d_x.ptr, reinterpret_cast<double2 *>(x), s, nullptr));
  return MR_OK;
}

extern "C" int mesh_reg_set_alpha(mr_ctx *c, int32_t pair, double alpha, void *stream) {
  const TraceRange range_("mesh_reg_set_alpha");
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (pair < 0 || pair >= c->n_pairs) return fail(MR_EINVAL, "pair out of range");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MR_EINVAL, "alpha must be finite and >= 0");
  PairHost &h = c->host[pair];
  const double old = h.alpha;
  // on any failure the host factor goes back to the old alpha (the device
  // copy was never touched), so the context stays as it was
  auto restore = [&]() {
    h.alpha = old;
    bool dummy;
    refactor(h, c->params.tau, &dummy);
    fill_dense_inverses(h);
    fill_panels(h);
    fill_apex_inverse(h);
  };
  h.alpha = alpha;
  bool not_spd = false;
  std::string e = refactor(h, c->params.tau, &not_spd);
  if (!e.empty()) {
    restore();
    return fail(not_spd ? MR_ENOTSPD : MR_EINVAL, e);
  }
  fill_dense_inverses(h);
  fill_panels(h);
  e = fill_apex_inverse(h);
  if (!e.empty()) {
    restore();
    return fail(MR_EINVAL, e);
  }
  if (c->host_only) return MR_OK;
  hipStream_t s = (hipStream_t)stream;
  return c->upload_factor(pair, s);
}

extern "C" int mesh_reg_set_template(mr_ctx *c, int32_t pair, const float *te, void *stream) {
  const TraceRange range_("mesh_reg_set_template");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (pair < 0 || pair >= c->n_pairs || !te) return fail(MR_EINVAL, "bad pair or null te");
  hipStream_t s = (hipStream_t)stream;
  return c->prefilter_pair(pair, te, c->d_coef.ptr + c->dpairs[pair].pix_off, s);
}

extern "C" int mesh_reg_get_tables(mr_ctx *c, int32_t pair, int32_t table_id, void *host_out,
                                   int64_t *len) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (pair < 0 || pair >= c->n_pairs || !len) return fail(MR_EINVAL, "bad pair or null len");
  const PairHost &h = c->host[pair];
  const std::vector<int64_t> *v64 = nullptr;
  const std::vector<int32_t> *v32 = nullptr;
  switch (table_id) {
    case MR_TAB_T1_PTR: v64 = &h.tab.t1_ptr; break;
    case MR_TAB_T1_SLOT: v64 = &h.tab.t1_slot; break;
    case MR_TAB_T2_PTR: v64 = &h.tab.t2_ptr; break;
    case MR_TAB_T2_IDX: v64 = &h.tab.t2_idx; break;
    case MR_TAB_T3_PTR: v64 = &h.tab.t3_ptr; break;
    case MR_TAB_T3_IDX: v64 = &h.tab.t3_idx; break;
    case MR_TAB_T4: v64 = &h.tab.t4; break;
    case MR_TAB_T5: v64 = &h.tab.t5; break;
    case MR_TAB_T6: v32 = &h.tab.t6; break;
    case MR_TAB_PERM: v32 = &h.perm; break;
    default: return fail(MR_EINVAL, "unknown table id");
  }
  if (v64) {
    *len = (int64_t)v64->size();
    if (host_out) std::memcpy(host_out, v64->data(), v64->size() * sizeof(int64_t));
  } else {
    *len = (int64_t)v32->size();
    if (host_out) std::memcpy(host_out, v32->data(), v32->size() * sizeof(int32_t));
  }
  return MR_OK;
}

// Algorithmic bytes of one solve call of a pair, each datum counted once per
// pass that needs it: the dense inverses (forward and backward copies) and
// panels (read by both passes) of the blocks below the apex, the apex's X by
// rows and by columns, the update buffer (written and read) with its index
// lists, the right-hand side, the intermediate and final vectors, and the
// result scattered to natural order.
static int64_t solve_bytes(const PairHost &h) {
  const SolvePlan &pl = h.plan;
  int64_t b = 0;
  for (size_t s = 0; s < pl.blocks.size(); ++s) {
    if (pl.is_apex[s]) continue;
    const int64_t r = pl.blocks[s].r1 - pl.blocks[s].r0;
    const int64_t m = pl.below_ptr[s + 1] - pl.below_ptr[s];
    b += 2 * 8 * (r * (r + 1) / 2) + 2 * 8 * (m * r);   // dense inverses, panel twice
    b += 16 * m + 16 * m + 4 * m;                        // updates written and read, below index
  }
  b += 4 * (int64_t)pl.cidx.size();                      // contribution lists
  const int64_t na = (int64_t)pl.apex_rows.size();
  if (na) b += 8 * (pl.apex_xf_off[na] + pl.apex_xb_off[na]) + 16 * na;   // X twice, t
  b += (int64_t)h.n * (16 + 16 + 16 + 16 + 16 + 4);     // b in, y out, y in, z out, out, perm
  return b;
}

// Distinct triangles of T6 summed over the pair's kTile x kTile pixel tiles.
static int64_t tile_entries(const PairHost &h) {
  int64_t total = 0;
  int32_t ids[kTile * kTile];
  for (int y0 = 0; y0 < h.height; y0 += kTile)
    for (int x0 = 0; x0 < h.width; x0 += kTile) {
      int n = 0;
      for (int r = y0; r < std::min(h.height, y0 + kTile); ++r)
        for (int c = x0; c < std::min(h.width, x0 + kTile); ++c)
          ids[n++] = h.tab.t6[(size_t)r * h.width + c];
      std::sort(ids, ids + n);
      total += std::unique(ids, ids + n) - ids;
    }
  return total;
}

extern "C" int mesh_reg_get_info(mr_ctx *c, int32_t pair, int32_t key, int64_t *value) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (!value) return fail(MR_EINVAL, "null value");
  if (key == MR_INFO_N_PAIRS) {
    *value = c->n_pairs;
    return MR_OK;
  }
  if (key == MR_INFO_DEVICE_BYTES) {
    *value = c->device_bytes();
    return MR_OK;
  }
  if (key == MR_INFO_FUSED_ASSEMBLY) {
    *value = c->fuse_first ? 1 : 0;
    return MR_OK;
  }
  if (pair < 0 || pair >= c->n_pairs) return fail(MR_EINVAL, "pair out of range");
  const PairHost &h = c->host[pair];
  switch (key) {
    case MR_INFO_N_NODES: *value = h.n; break;
    case MR_INFO_N_TRIS: *value = h.nt; break;
    case MR_INFO_NNZ_L: *value = h.L.colptr.empty() ? 0 : h.L.colptr[h.n]; break;
    case MR_INFO_N_BLOCKS: *value = (int64_t)h.plan.blocks.size(); break;
    case MR_INFO_SOLVE_OFFBLOCK: *value = (int64_t)h.plan.panel_row.size(); break;
    case MR_INFO_SOLVE_DENSE: *value = (int64_t)h.plan.dinv_col.size(); break;
    case MR_INFO_MASS_NNZ:
      *value = c->params.force_mode == MR_FORCE_NODAL ? h.n : (int64_t)h.tab.t3_idx.size();
      break;
    case MR_INFO_APEX_ROWS: *value = (int64_t)h.plan.apex_rows.size(); break;
    case MR_INFO_SOLVE_BYTES: *value = solve_bytes(h); break;
    case MR_INFO_TILE_ENTRIES: *value = tile_entries(h); break;
    case MR_INFO_FWD_LEVELS: *value = h.plan.n_fwd_levels; break;
    case MR_INFO_BWD_LEVELS: *value = h.plan.n_bwd_levels; break;
    case MR_INFO_NODE_OFFSET: {
      int64_t o = 0;
      for (int p = 0; p < pair; ++p) o += c->host[p].n;
      *value = o;
      break;
    }
    case MR_INFO_PIXEL_OFFSET: {
      int64_t o = 0;
      for (int p = 0; p < pair; ++p) o += (int64_t)c->host[p].height * c->host[p].width;
      *value = o;
      break;
    }
    default: return fail(MR_EINVAL, "unknown info key");
  }
  return MR_OK;
}

extern "C" int mesh_reg_enable_timing(mr_ctx *c, int32_t enable) {
  int rc = check_ctx(c, true);
  if (rc) return rc;
  c->timing = enable != 0;
  return MR_OK;
}

extern "C" int mesh_reg_set_graph(mr_ctx *c, int32_t enable) {
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (enable) {
    c->params.flags |= MR_FLAG_GRAPH;
  } else {
    c->params.flags &= ~MR_FLAG_GRAPH;
    if (c->graph_exec) {
      HIP_TRY(hipGraphExecDestroy(c->graph_exec));
      c->graph_exec = nullptr;
    }
  }
  return MR_OK;
}

extern "C" int mesh_reg_kernel_times(mr_ctx *c, double *ms, int64_t *launches) {
  int rc = check_ctx(c, true);
  if (rc) return rc;
  if (!ms || !launches) return fail(MR_EINVAL, "null output");
  for (int f = 0; f < MR_KF_COUNT; ++f) {
    ms[f] = 0.0;
    launches[f] = 0;
  }
  for (auto &p : c->pending) {
    HIP_TRY(hipEventSynchronize(p.stop));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, p.start, p.stop));
    ms[p.family] += t;
    launches[p.family] += 1;
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  c->pending.clear();
  return MR_OK;
}

extern "C" void mesh_reg_destroy(mr_ctx *c) { delete c; }

extern "C" int mesh_reg_forward_ckpt(mr_ctx *c, double *u, int32_t n_iter, int32_t ckpt_every,
                                     double *ckpt, double *msd, void *stream) {
  const TraceRange range_("mesh_reg_forward_ckpt");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  return c->forward_with_ckpt(u, n_iter, ckpt_every, ckpt, msd, (hipStream_t)stream);
}

extern "C" int mesh_reg_backward_ckpt(mr_ctx *c, const double *ckpt, int32_t n_iter,
                                      int32_t ckpt_every, const double *g_msd, double *g_u0,
                                      double *g_alpha, float *g_te, double *msd, void *stream) {
  const TraceRange range_("mesh_reg_backward_ckpt");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  return c->backward_from_ckpt(ckpt, n_iter, ckpt_every, g_msd, g_u0, g_alpha, g_te, msd,
                               (hipStream_t)stream);
}

extern "C" int mesh_reg_backward(mr_ctx *c, const double *u0, int32_t n_iter, int32_t ckpt_every,
                                 const double *g_msd, double *g_u0, double *g_alpha, float *g_te,
                                 double *msd, void *stream) {
  const TraceRange range_("mesh_reg_backward");
  int rc = check_ctx(c, true);
  if (rc) return rc;
  return c->backward(u0, n_iter, ckpt_every, g_msd, g_u0, g_alpha, g_te, msd, (hipStream_t)stream);
}
