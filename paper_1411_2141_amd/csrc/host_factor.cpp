// Ordering, FP64 sparse Cholesky factorisation of S = I + tau alpha K and the
// block schedule of its triangular solves.
//
// The paper solves its sparse mesh system directly (abstract; Section 3.3);
// here the system is the implicit diffusion step (eq. 7-8 taken implicitly
// with the symmetric P1 stiffness).  The factor is computed once per mesh and
// alpha on the host; the GPU only runs the two triangular solves per iteration.
//
// Ordering: geometric nested dissection on the node coordinates.  A node set is
// split by a straight cut across one axis, chosen among the positions that
// leave each side at least 30 % of the set for the smallest separator per
// pair of halves (not at the median: on adaptive meshes a cut through coarse
// cells crosses few nodes); the separator is the smaller of the two one-sided
// boundary sets; the halves are ordered first, the separator last.  Small sets become leaf blocks, separators become one or
// more chained blocks.  Every block is a contiguous row range of P S P^T and
// the block tree contains the elimination tree, which is what lets the solve
// run block-parallel level by level.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <thread>

#include "host.h"

namespace mr {

namespace {

struct NDState {
  const PairHost &p;
  const OrderOptions &opt;
  std::vector<int32_t> order;
  std::vector<std::pair<int32_t, int32_t>> ranges;
  std::vector<int32_t> parent;
  std::vector<int8_t> side;   // -1 outside the current set, 0 left, 1 right
  NDState(const PairHost &pp, const OrderOptions &o) : p(pp), opt(o), side(pp.n, -1) {}

  int32_t emit(const std::vector<int32_t> &nodes) {
    const int32_t r0 = (int32_t)order.size();
    order.insert(order.end(), nodes.begin(), nodes.end());
    ranges.emplace_back(r0, (int32_t)order.size());
    parent.push_back(-1);
    return (int32_t)ranges.size() - 1;
  }

  struct Cut {
    int axis;        // coordinate axis (0: x, 1: y)
    int32_t value;   // nodes whose coordinate is < value go left
  };

  // The cut of S.  Candidates: for each coordinate axis, every position c
  // whose two sides each hold at least a fraction `nd_balance` of S.  Each
  // is scored by the size of the smaller one-sided boundary set it leaves
  // (the separator it would give), divided by the product of the two side
  // sizes (nd_score 1: small separators between large halves) or alone
  // (nd_score 0), computed for all c at once from per-node intervals: a node
  // v left of c is on the left boundary iff c <= (largest coordinate among
  // its neighbours in S), a node right of c is on the right boundary iff
  // c > (smallest coordinate among its neighbours in S).  The best score
  // wins, ties going to the more balanced cut, then to axis 0.  On adaptive
  // meshes the cut moves off the median into coarse regions, where few
  // nodes lie along it.
  Cut best_cut(const std::vector<int32_t> &S) {
    for (int32_t v : S) side[v] = 0;                  // membership of S
    const auto &ptr = p.tab.t2_ptr;
    const auto &idx = p.tab.t2_idx;
    const int64_t ns = (int64_t)S.size();
    Cut best{0, 0};
    int64_t best_sep = INT64_MAX, best_imb = INT64_MAX;
    for (int axis = 0; axis < 2; ++axis) {
      int32_t lo = INT32_MAX, hi = INT32_MIN;
      for (int32_t v : S) {
        lo = std::min(lo, p.xy[2 * v + axis]);
        hi = std::max(hi, p.xy[2 * v + axis]);
      }
      if (hi == lo) continue;
      const int32_t len = hi - lo + 2;
      std::vector<int64_t> below(len + 1, 0), dl(len + 1, 0), dr(len + 1, 0);
      for (int32_t v : S) {
        const int32_t cv = p.xy[2 * v + axis] - lo;
        int32_t mx = cv, mn = cv;
        for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) {
          const int32_t w = (int32_t)idx[k];
          if (side[w] < 0) continue;
          const int32_t cw = p.xy[2 * w + axis] - lo;
          mx = std::max(mx, cw);
          mn = std::min(mn, cw);
        }
        below[cv + 1] += 1;               // nodes with coordinate < c, counted from c = cv + 1 on
        if (mx > cv) {                    // left boundary for cv < c <= mx
          dl[cv + 1] += 1;
          dl[mx + 1] -= 1;
        }
        if (mn < cv) {                    // right boundary for mn < c <= cv
          dr[mn + 1] += 1;
          dr[cv + 1] -= 1;
        }
      }
      int64_t nb = 0, sl = 0, sr = 0;
      for (int32_t c = 0; c <= len; ++c) {
        nb += below[c];
        sl += dl[c];
        sr += dr[c];
        if (c == 0 || c > hi - lo) continue;
        const int64_t left = nb, right = ns - nb;
        if ((double)std::min(left, right) < opt.nd_balance * (double)ns) continue;
        int64_t sep = std::min(sl, sr);
        const int64_t imb = std::abs(left - right);
        if (opt.nd_score == 1)
          sep = (int64_t)(1e12 * (double)(sep + 1) / ((double)left * (double)right));
        if (sep < best_sep || (sep == best_sep && imb < best_imb)) {
          best_sep = sep;
          best_imb = imb;
          best = Cut{axis, lo + c};
        }
      }
    }
    if (best_sep == INT64_MAX) {
      // no admissible cut (tiny or degenerate sets): the median of the wider axis
      int32_t lo[2] = {INT32_MAX, INT32_MAX}, hi[2] = {INT32_MIN, INT32_MIN};
      for (int32_t v : S)
        for (int a = 0; a < 2; ++a) {
          lo[a] = std::min(lo[a], p.xy[2 * v + a]);
          hi[a] = std::max(hi[a], p.xy[2 * v + a]);
        }
      int axis = (hi[0] - lo[0] >= hi[1] - lo[1]) ? 0 : 1;
      if (hi[axis] == lo[axis]) axis ^= 1;
      std::vector<int32_t> tmp;
      for (int32_t v : S) tmp.push_back(p.xy[2 * v + axis]);
      std::nth_element(tmp.begin(), tmp.begin() + tmp.size() / 2, tmp.end());
      int32_t c = tmp[tmp.size() / 2];
      if (c == lo[axis]) {
        int32_t nxt = INT32_MAX;
        for (int32_t v : tmp)
          if (v > lo[axis]) nxt = std::min(nxt, v);
        c = nxt;
      }
      best = Cut{axis, c};
    }
    for (int32_t v : S) side[v] = -1;
    return best;
  }

  // Orders `S` (consumed) and returns the block id of its subtree root.
  int32_t run(std::vector<int32_t> S) {
    if ((int32_t)S.size() <= opt.leaf_max) {
      std::sort(S.begin(), S.end());
      return emit(S);
    }
    const Cut cut = best_cut(S);
    for (int32_t v : S) side[v] = p.xy[2 * v + cut.axis] < cut.value ? 0 : 1;
    std::vector<int32_t> sepL, sepR;
    const auto &ptr = p.tab.t2_ptr;
    const auto &idx = p.tab.t2_idx;
    for (int32_t v : S) {
      const int8_t sv = side[v];
      for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) {
        const int8_t sw = side[idx[k]];
        if (sw >= 0 && sw != sv) {
          (sv == 0 ? sepL : sepR).push_back(v);
          break;
        }
      }
    }
    const bool useR = sepR.size() <= sepL.size();
    std::vector<int32_t> &sep = useR ? sepR : sepL;
    for (int32_t v : sep) side[v] = 2;
    std::vector<int32_t> A, B;
    for (int32_t v : S) {
      if (side[v] == 0) A.push_back(v);
      else if (side[v] == 1) B.push_back(v);
    }
    for (int32_t v : S) side[v] = -1;
    std::vector<int32_t>().swap(S);
    const int32_t a = A.empty() ? -1 : run(std::move(A));
    const int32_t b = B.empty() ? -1 : run(std::move(B));
    // separator nodes along the cut, then chunked into chained blocks
    const int other = cut.axis ^ 1;
    std::sort(sep.begin(), sep.end(), [&](int32_t u, int32_t v) {
      const int32_t cu = p.xy[2 * u + other], cv = p.xy[2 * v + other];
      return cu != cv ? cu < cv : u < v;
    });
    const int32_t ns = (int32_t)sep.size();
    const int32_t nchunk = std::max<int32_t>(1, (ns + opt.block_max - 1) / opt.block_max);
    int32_t prev = -1, first = -1;
    for (int32_t q = 0; q < nchunk; ++q) {
      const int32_t s0 = (int32_t)((int64_t)ns * q / nchunk), s1 = (int32_t)((int64_t)ns * (q + 1) / nchunk);
      std::vector<int32_t> part(sep.begin() + s0, sep.begin() + s1);
      const int32_t id = emit(part);
      if (prev >= 0) parent[prev] = id;
      if (first < 0) first = id;
      prev = id;
    }
    if (a >= 0) parent[a] = first;
    if (b >= 0) parent[b] = first;
    return prev;
  }
};

inline int32_t next_pow2_clamped(double x, int32_t lo, int32_t hi) {
  int32_t g = lo;
  while (g < hi && g < x) g *= 2;
  return g;
}

}  // namespace

std::string nested_dissection(PairHost &p, const OrderOptions &opt,
                              std::vector<std::pair<int32_t, int32_t>> &ranges,
                              std::vector<int32_t> &range_parent) {
  NDState st(p, opt);
  std::vector<int32_t> all(p.n);
  for (int32_t i = 0; i < p.n; ++i) all[i] = i;
  st.run(std::move(all));
  if ((int32_t)st.order.size() != p.n) return "nested dissection lost nodes";
  p.perm = st.order;
  p.iperm.assign(p.n, -1);
  for (int32_t k = 0; k < p.n; ++k) p.iperm[p.perm[k]] = k;
  for (int32_t i = 0; i < p.n; ++i)
    if (p.iperm[i] < 0) return "nested dissection produced a non-permutation";
  ranges = std::move(st.ranges);
  range_parent = std::move(st.parent);
  return "";
}

// Permuted matrix A = P S P^T: row k holds entries (iperm[j], S[perm[k], j]).
static void permuted_rows(const PairHost &p, double tau,
                          std::vector<std::vector<std::pair<int32_t, double>>> &rows) {
  rows.assign(p.n, {});
  const auto &ptr = p.tab.t3_ptr;
  const auto &idx = p.tab.t3_idx;
  const double ta = tau * p.alpha;
  for (int32_t k = 0; k < p.n; ++k) {
    const int32_t v = p.perm[k];
    for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q) {
      const int32_t j = (int32_t)idx[q];
      const double s = (j == v ? 1.0 : 0.0) + ta * p.kval[q];
      rows[k].emplace_back(p.iperm[j], s);
    }
    std::sort(rows[k].begin(), rows[k].end());
  }
}

// Up-looking numeric factorisation over the stored row patterns.
static std::string numeric(PairHost &p, double tau, bool *not_spd) {
  Factor &L = p.L;
  const int32_t n = L.n;
  std::vector<std::vector<std::pair<int32_t, double>>> A;
  permuted_rows(p, tau, A);
  std::vector<double> x(n, 0.0);
  std::vector<int64_t> next(n);
  for (int32_t j = 0; j < n; ++j) next[j] = L.colptr[j] + 1;
  for (int32_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (auto &e : A[i]) {
      if (e.first < i) x[e.first] = e.second;
      else if (e.first == i) d = e.second;
    }
    for (int64_t q = p.L_rowptr[i]; q < p.L_rowptr[i + 1]; ++q) {
      const int32_t j = p.L_rowcol[q];
      const double lij = x[j] / L.val[L.colptr[j]];
      x[j] = 0.0;
      for (int64_t r = L.colptr[j] + 1; r < next[j]; ++r) x[L.rowidx[r]] -= L.val[r] * lij;
      d -= lij * lij;
      L.rowidx[next[j]] = i;
      L.val[next[j]] = lij;
      ++next[j];
    }
    if (!(d > 0.0) || !std::isfinite(d)) {
      *not_spd = true;
      char buf[128];
      std::snprintf(buf, sizeof buf, "non-positive pivot %.3e at elimination step %d", d, i);
      return buf;
    }
    L.rowidx[L.colptr[i]] = i;
    L.val[L.colptr[i]] = std::sqrt(d);
  }
  for (int32_t j = 0; j < n; ++j)
    if (next[j] != L.colptr[j + 1]) return "factor structure mismatch";
  return "";
}

std::string cholesky(PairHost &p, double tau, bool *not_spd) {
  *not_spd = false;
  const int32_t n = p.n;
  Factor &L = p.L;
  L.n = n;
  // permuted lower pattern
  std::vector<std::vector<std::pair<int32_t, double>>> A;
  permuted_rows(p, tau, A);
  // elimination tree (with path-compressed ancestors)
  L.parent.assign(n, -1);
  std::vector<int32_t> anc(n, -1);
  for (int32_t i = 0; i < n; ++i)
    for (auto &e : A[i]) {
      int32_t k = e.first;
      if (k >= i) continue;
      while (k != -1 && k != i) {
        const int32_t nk = anc[k];
        anc[k] = i;
        if (nk == -1) L.parent[k] = i;
        k = nk;
      }
    }
  // row patterns: walk up the tree from each entry of row i until a marked node
  std::vector<int32_t> mark(n, -1), count(n, 1);
  p.L_rowptr.assign(n + 1, 0);
  p.L_rowcol.clear();
  std::vector<int32_t> rowbuf;
  for (int32_t i = 0; i < n; ++i) {
    rowbuf.clear();
    mark[i] = i;
    for (auto &e : A[i]) {
      int32_t k = e.first;
      if (k >= i) continue;
      while (k != -1 && mark[k] != i) {
        mark[k] = i;
        rowbuf.push_back(k);
        k = L.parent[k];
      }
    }
    std::sort(rowbuf.begin(), rowbuf.end());
    for (int32_t j : rowbuf) ++count[j];
    p.L_rowcol.insert(p.L_rowcol.end(), rowbuf.begin(), rowbuf.end());
    p.L_rowptr[i + 1] = (int64_t)p.L_rowcol.size();
  }
  L.colptr.assign(n + 1, 0);
  for (int32_t j = 0; j < n; ++j) L.colptr[j + 1] = L.colptr[j] + count[j];
  L.rowidx.assign(L.colptr[n], 0);
  L.val.assign(L.colptr[n], 0.0);
  return numeric(p, tau, not_spd);
}

std::string refactor(PairHost &p, double tau, bool *not_spd) {
  *not_spd = false;
  return numeric(p, tau, not_spd);
}

void fill_dense_inverses(PairHost &p) {
  SolvePlan &pl = p.plan;
  const Factor &L = p.L;
  std::vector<double> D, X;
  for (size_t s = 0; s < pl.blocks.size(); ++s) {
    const int32_t r0 = pl.blocks[s].r0, r1 = pl.blocks[s].r1, b = r1 - r0;
    if (b == 0) continue;
    D.assign((size_t)b * b, 0.0);
    X.assign((size_t)b * b, 0.0);
    for (int32_t j = r0; j < r1; ++j)
      for (int64_t q = L.colptr[j]; q < L.colptr[j + 1]; ++q) {
        const int32_t i = L.rowidx[q];
        if (i >= r1) break;
        D[(size_t)(i - r0) * b + (j - r0)] = L.val[q];
      }
    // X = D^-1 (lower triangular), column by column
    for (int32_t c = 0; c < b; ++c) {
      X[(size_t)c * b + c] = 1.0 / D[(size_t)c * b + c];
      for (int32_t i = c + 1; i < b; ++i) {
        double acc = 0.0;
        for (int32_t k = c; k < i; ++k) acc += D[(size_t)i * b + k] * X[(size_t)k * b + c];
        X[(size_t)i * b + c] = -acc / D[(size_t)i * b + i];
      }
    }
    const int64_t off = pl.dense_off[s];
    for (int32_t j = 0; j < b; ++j) {
      const int64_t oc = off + (int64_t)j * b - (int64_t)j * (j - 1) / 2;
      for (int32_t i = j; i < b; ++i) pl.dinv_col[oc + (i - j)] = X[(size_t)i * b + j];
    }
    for (int32_t i = 0; i < b; ++i) {
      const int64_t orow = off + (int64_t)i * (i + 1) / 2;
      for (int32_t j = 0; j <= i; ++j) pl.dinv_row[orow + j] = X[(size_t)i * b + j];
    }
  }
}

void fill_panels(PairHost &p) {
  SolvePlan &pl = p.plan;
  const Factor &L = p.L;
  std::vector<int32_t> pos(L.n, -1);
  for (size_t s = 0; s < pl.blocks.size(); ++s) {
    const int32_t r0 = pl.blocks[s].r0, r1 = pl.blocks[s].r1, b = r1 - r0;
    const int64_t k0 = pl.below_ptr[s], m = pl.below_ptr[s + 1] - k0;
    for (int64_t k = 0; k < m; ++k) pos[pl.below_idx[k0 + k]] = (int32_t)k;
    const int64_t off = pl.panel_off[s];
    std::fill(pl.panel_row.begin() + off, pl.panel_row.begin() + off + m * b, 0.0);
    for (int32_t j = r0; j < r1; ++j)
      for (int64_t q = L.colptr[j] + 1; q < L.colptr[j + 1]; ++q) {
        const int32_t r = L.rowidx[q];
        if (r < r1) continue;
        const int64_t k = pos[r];
        pl.panel_row[off + k * b + (j - r0)] = L.val[q];
      }
    for (int64_t k = 0; k < m; ++k) pos[pl.below_idx[k0 + k]] = -1;
  }
}

std::string build_solve_plan(PairHost &p, const std::vector<std::pair<int32_t, int32_t>> &ranges,
                             const std::vector<int32_t> &range_parent, const OrderOptions &opt) {
  SolvePlan &pl = p.plan;
  const Factor &L = p.L;
  const int32_t n = L.n;
  const int32_t nb = (int32_t)ranges.size();
  pl.blocks.assign(nb, SolveBlock{});
  std::vector<int32_t> blk_of(n, -1);
  for (int32_t s = 0; s < nb; ++s) {
    SolveBlock &B = pl.blocks[s];
    B.r0 = ranges[s].first;
    B.r1 = ranges[s].second;
    B.parent = range_parent[s];
    if (B.r1 - B.r0 > opt.block_max) return "block larger than block_max";
    if (B.parent >= 0 && B.parent <= s) return "block tree not in postorder";
    for (int32_t r = B.r0; r < B.r1; ++r) blk_of[r] = s;
  }
  for (int32_t r = 0; r < n; ++r)
    if (blk_of[r] < 0) return "row not covered by a block";
  // descendants of block s are the contiguous ids [desc_lo[s], s] (postorder)
  std::vector<int32_t> desc_lo(nb);
  for (int32_t s = 0; s < nb; ++s) desc_lo[s] = s;
  for (int32_t s = 0; s < nb; ++s)
    if (pl.blocks[s].parent >= 0)
      desc_lo[pl.blocks[s].parent] = std::min(desc_lo[pl.blocks[s].parent], desc_lo[s]);
  // every factor entry must couple a block to itself or to an ancestor
  for (int32_t k = 0; k < n; ++k)
    for (int64_t q = L.colptr[k] + 1; q < L.colptr[k + 1]; ++q) {
      const int32_t bi = blk_of[L.rowidx[q]], bk = blk_of[k];
      if (bk < desc_lo[bi] || bk > bi) return "factor entry outside the block tree";
    }
  // levels
  for (int32_t s = 0; s < nb; ++s) pl.blocks[s].fwd_level = 0;
  for (int32_t s = 0; s < nb; ++s) {
    const int32_t par = pl.blocks[s].parent;
    if (par >= 0) pl.blocks[par].fwd_level = std::max(pl.blocks[par].fwd_level, pl.blocks[s].fwd_level + 1);
  }
  for (int32_t s = nb - 1; s >= 0; --s) {
    const int32_t par = pl.blocks[s].parent;
    pl.blocks[s].bwd_level = par >= 0 ? pl.blocks[par].bwd_level + 1 : 0;
  }
  pl.n_fwd_levels = pl.n_bwd_levels = 0;
  for (auto &B : pl.blocks) {
    pl.n_fwd_levels = std::max(pl.n_fwd_levels, B.fwd_level + 1);
    pl.n_bwd_levels = std::max(pl.n_bwd_levels, B.bwd_level + 1);
  }
  // blocks in forward-level order: dense inverses, panels and update entries
  // of one level are stored contiguously
  std::vector<int32_t> lorder(nb);
  for (int32_t s = 0; s < nb; ++s) lorder[s] = s;
  std::stable_sort(lorder.begin(), lorder.end(), [&](int32_t a, int32_t b) {
    return pl.blocks[a].fwd_level < pl.blocks[b].fwd_level;
  });
  // every block's entries start on a 16-byte boundary (sizes rounded up to an
  // even number of doubles) so the device can stage them with 16-byte loads
  pl.dense_off.assign(nb, 0);
  int64_t tot = 0;
  for (int32_t s : lorder) {
    const int64_t b = pl.blocks[s].r1 - pl.blocks[s].r0;
    pl.dense_off[s] = tot;
    tot += (b * (b + 1) / 2 + 1) / 2 * 2;
  }
  pl.dinv_col.assign(tot, 0.0);
  pl.dinv_row.assign(tot, 0.0);
  // below-sets (union of the column structures under each block)
  pl.below_ptr.assign(nb + 1, 0);
  pl.below_idx.clear();
  std::vector<int32_t> mark(n, -1), rows;
  for (int32_t s = 0; s < nb; ++s) {
    const SolveBlock &B = pl.blocks[s];
    rows.clear();
    for (int32_t j = B.r0; j < B.r1; ++j)
      for (int64_t q = L.colptr[j] + 1; q < L.colptr[j + 1]; ++q) {
        const int32_t r = L.rowidx[q];
        if (r >= B.r1 && mark[r] != s) {
          mark[r] = s;
          rows.push_back(r);
        }
      }
    std::sort(rows.begin(), rows.end());
    pl.below_idx.insert(pl.below_idx.end(), rows.begin(), rows.end());
    pl.below_ptr[s + 1] = (int64_t)pl.below_idx.size();
  }
  if (pl.below_idx.size() >= (size_t)INT32_MAX) return "update buffer too large";
  pl.max_below = 0;
  pl.panel_off.assign(nb, 0);
  int64_t ptot = 0;
  for (int32_t s : lorder) {
    const int64_t m = pl.below_ptr[s + 1] - pl.below_ptr[s];
    pl.max_below = std::max<int32_t>(pl.max_below, (int32_t)m);
    pl.panel_off[s] = ptot;
    ptot += (m * (pl.blocks[s].r1 - pl.blocks[s].r0) + 1) / 2 * 2;
  }
  pl.panel_row.assign(ptot, 0.0);
  // contributors of each row, in increasing block order
  pl.cptr.assign(n + 1, 0);
  for (int32_t r : pl.below_idx) pl.cptr[r + 1]++;
  for (int32_t r = 0; r < n; ++r) pl.cptr[r + 1] += pl.cptr[r];
  pl.cidx.assign(pl.cptr[n], 0);
  {
    std::vector<int64_t> next(pl.cptr.begin(), pl.cptr.end() - 1);
    for (int32_t s = 0; s < nb; ++s)
      for (int64_t k = pl.below_ptr[s]; k < pl.below_ptr[s + 1]; ++k)
        pl.cidx[next[pl.below_idx[k]]++] = (int32_t)k;
  }
  // lanes per row of the forward contributor gathers
  for (auto &B : pl.blocks) {
    const int32_t b = B.r1 - B.r0;
    int64_t cnt = 0;
    for (int32_t r = B.r0; r < B.r1; ++r) cnt += pl.cptr[r + 1] - pl.cptr[r];
    B.fwd_group = next_pow2_clamped(b ? (double)cnt / b : 0.0, 1, 64);
  }
  fill_dense_inverses(p);
  fill_panels(p);
  return "";
}

std::string build_apex(PairHost &p, const OrderOptions &opt) {
  SolvePlan &pl = p.plan;
  const int32_t nb = (int32_t)pl.blocks.size();
  // rows per forward level, and per block the rows of all its ancestors
  std::vector<int64_t> rows_at(pl.n_fwd_levels, 0);
  for (auto &B : pl.blocks) rows_at[B.fwd_level] += B.r1 - B.r0;
  std::vector<int64_t> anc_rows(nb, 0);
  std::vector<int32_t> by_level(nb);
  for (int32_t s = 0; s < nb; ++s) by_level[s] = s;
  std::stable_sort(by_level.begin(), by_level.end(), [&](int32_t x, int32_t y) {
    return pl.blocks[x].fwd_level > pl.blocks[y].fwd_level;
  });
  for (int32_t s : by_level) {
    const int32_t q = pl.blocks[s].parent;
    if (q >= 0) anc_rows[s] = anc_rows[q] + (pl.blocks[q].r1 - pl.blocks[q].r0);
  }
  std::vector<int64_t> path_at(pl.n_fwd_levels, 0);     // longest path of a block at a level
  for (int32_t s = 0; s < nb; ++s)
    path_at[pl.blocks[s].fwd_level] = std::max<int64_t>(
        path_at[pl.blocks[s].fwd_level], anc_rows[s] + pl.blocks[s].r1 - pl.blocks[s].r0);
  // entries a level adds to X: each block's own triangle and its rows
  // against every ancestor block's rows
  std::vector<int64_t> ent_at(pl.n_fwd_levels, 0);
  for (int32_t s = 0; s < nb; ++s) {
    const int64_t b = pl.blocks[s].r1 - pl.blocks[s].r0;
    ent_at[pl.blocks[s].fwd_level] += b * (b + 1) / 2 + b * anc_rows[s];
  }
  // the apex is the highest run of levels within the limits
  int32_t cut = pl.n_fwd_levels;
  int64_t acc = 0;
  for (int32_t l = pl.n_fwd_levels - 1; l >= 1 && opt.apex_max > 0; --l) {
    if (acc + rows_at[l] > opt.apex_max || path_at[l] > kApexPathMax ||
        ent_at[l] > opt.apex_level_entries)
      break;
    acc += rows_at[l];
    cut = l;
  }
  if (cut > pl.n_fwd_levels - 2) cut = pl.n_fwd_levels;   // fewer than two levels: no apex
  pl.apex_level = cut;
  pl.is_apex.assign(nb, 0);
  pl.apex_rows.clear();
  pl.apex_blocks.clear();
  pl.apex_anc.clear();
  pl.apex_c0.clear();
  pl.apex_blk.clear();
  std::vector<int32_t> ablocks;                // apex block -> block id, ascending rows
  for (int32_t s = 0; s < nb; ++s)
    if (pl.blocks[s].fwd_level >= cut) {
      pl.is_apex[s] = 1;
      ablocks.push_back(s);
    }
  std::sort(ablocks.begin(), ablocks.end(),
            [&](int32_t x, int32_t y) { return pl.blocks[x].r0 < pl.blocks[y].r0; });
  std::vector<int32_t> apex_id(nb, -1);
  for (size_t k = 0; k < ablocks.size(); ++k) {
    const SolveBlock &B = pl.blocks[ablocks[k]];
    apex_id[ablocks[k]] = (int32_t)k;
    ApexBlock A{(int32_t)pl.apex_rows.size(), 0, 0, 0, 0, 0};
    for (int32_t r = B.r0; r < B.r1; ++r) pl.apex_rows.push_back(r);
    A.a1 = (int32_t)pl.apex_rows.size();
    A.c0 = A.a0;
    pl.apex_blocks.push_back(A);
  }
  // subtree start: children come before their parent in row order
  for (size_t k = 0; k < ablocks.size(); ++k) {
    const int32_t q = pl.blocks[ablocks[k]].parent;
    if (q >= 0 && apex_id[q] >= 0) {
      ApexBlock &P = pl.apex_blocks[apex_id[q]];
      P.c0 = std::min(P.c0, pl.apex_blocks[k].c0);
    }
  }
  for (size_t k = 0; k < ablocks.size(); ++k) {
    ApexBlock &A = pl.apex_blocks[k];
    A.anc_off = (int32_t)pl.apex_anc.size();
    for (int32_t q = pl.blocks[ablocks[k]].parent; q >= 0; q = pl.blocks[q].parent) {
      if (apex_id[q] < 0) return "apex block with a non-apex ancestor";
      pl.apex_anc.push_back(apex_id[q]);
      A.anc_rows += pl.apex_blocks[apex_id[q]].a1 - pl.apex_blocks[apex_id[q]].a0;
    }
    A.n_anc = (int32_t)pl.apex_anc.size() - A.anc_off;
    if (A.a1 - A.a0 + A.anc_rows > kApexPathMax) return "apex path longer than the limit";
    for (int32_t i = A.a0; i < A.a1; ++i) {
      pl.apex_c0.push_back(A.c0);
      pl.apex_blk.push_back((int32_t)k);
    }
  }
  // storage offsets of X by rows (forward) and by columns (backward)
  const int32_t na = (int32_t)pl.apex_rows.size();
  pl.apex_xf_off.assign(na + 1, 0);
  pl.apex_xb_off.assign(na + 1, 0);
  for (int32_t i = 0; i < na; ++i) {
    const ApexBlock &A = pl.apex_blocks[pl.apex_blk[i]];
    pl.apex_xf_off[i + 1] = pl.apex_xf_off[i] + (i - pl.apex_c0[i] + 1);
    pl.apex_xb_off[i + 1] = pl.apex_xb_off[i] + (A.a1 - i) + A.anc_rows;
  }
  // contributions to apex rows from non-apex blocks only
  std::vector<int32_t> blk_of_upd(pl.below_idx.size());
  for (int32_t s = 0; s < nb; ++s)
    for (int64_t k = pl.below_ptr[s]; k < pl.below_ptr[s + 1]; ++k) blk_of_upd[k] = s;
  pl.apex_cptr.assign(pl.apex_rows.size() + 1, 0);
  pl.apex_cidx.clear();
  for (size_t i = 0; i < pl.apex_rows.size(); ++i) {
    const int32_t r = pl.apex_rows[i];
    for (int64_t q = pl.cptr[r]; q < pl.cptr[r + 1]; ++q)
      if (!pl.is_apex[blk_of_upd[pl.cidx[q]]]) pl.apex_cidx.push_back(pl.cidx[q]);
    pl.apex_cptr[i + 1] = (int64_t)pl.apex_cidx.size();
  }
  return fill_apex_inverse(p);
}

std::string fill_apex_inverse(PairHost &p) {
  SolvePlan &pl = p.plan;
  const Factor &L = p.L;
  const int32_t na = (int32_t)pl.apex_rows.size();
  pl.apex_xf.assign(pl.apex_xf_off[na], 0.0);
  pl.apex_xb.assign(pl.apex_xb_off[na], 0.0);
  if (na == 0) return "";
  // sparse L(apex, apex) by columns, in apex positions
  std::vector<int32_t> pos(L.n, -1);
  for (int32_t i = 0; i < na; ++i) pos[pl.apex_rows[i]] = i;
  std::vector<std::vector<std::pair<int32_t, double>>> col(na);
  std::vector<double> diag(na);
  for (int32_t j = 0; j < na; ++j) {
    const int32_t c = pl.apex_rows[j];
    diag[j] = L.val[L.colptr[c]];
    for (int64_t q = L.colptr[c] + 1; q < L.colptr[c + 1]; ++q)
      if (pos[L.rowidx[q]] >= 0) col[j].emplace_back(pos[L.rowidx[q]], L.val[q]);
  }
  // column c of X: forward substitution of e_c (column-oriented, skipping
  // zeros); its entries are then read along c's path (c's block from c on,
  // then the ancestor blocks), and every entry off that path must be zero.
  // Columns are independent: large apexes split them over threads.
  auto columns = [&](int32_t c_begin, int32_t c_step, bool *bad) {
    std::vector<double> x(na, 0.0);
    for (int32_t c = c_begin; c < na; c += c_step) {
      x[c] = 1.0;
      for (int32_t j = c; j < na; ++j) {
        if (x[j] == 0.0) continue;
        x[j] /= diag[j];
        const double xj = x[j];
        for (auto &e : col[j]) x[e.first] -= e.second * xj;
      }
      const ApexBlock &A = pl.apex_blocks[pl.apex_blk[c]];
      int64_t kb = pl.apex_xb_off[c];
      auto take = [&](int32_t i) {
        pl.apex_xf[pl.apex_xf_off[i] + (c - pl.apex_c0[i])] = x[i];
        pl.apex_xb[kb++] = x[i];
        x[i] = 0.0;
      };
      for (int32_t i = c; i < A.a1; ++i) take(i);
      for (int32_t k = A.anc_off; k < A.anc_off + A.n_anc; ++k) {
        const ApexBlock &G = pl.apex_blocks[pl.apex_anc[k]];
        for (int32_t i = G.a0; i < G.a1; ++i) take(i);
      }
      for (int32_t i = c; i < na; ++i)
        if (x[i] != 0.0) {
          *bad = true;
          x[i] = 0.0;
        }
    }
  };
  const int32_t nthr =
      na >= 2048 ? (int32_t)std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1;
  std::vector<uint8_t> bad(nthr, 0);
  auto run = [&](int32_t t) {
    bool b = false;
    columns(t, nthr, &b);
    bad[t] = b;
  };
  if (nthr == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    for (int32_t t = 0; t < nthr; ++t) th.emplace_back(run, t);
    for (auto &t : th) t.join();
  }
  for (uint8_t b : bad)
    if (b) return "apex inverse has an entry outside the subtree structure";
  return "";
}

std::string prepare_pair(PairHost &p, double tau, const OrderOptions &opt, bool *not_spd) {
  *not_spd = false;
  std::string e = validate_mesh(p);
  if (!e.empty()) return e;
  e = build_tables(p);
  if (!e.empty()) return e;
  build_operators(p);
  std::vector<std::pair<int32_t, int32_t>> ranges;
  std::vector<int32_t> rparent;
  e = nested_dissection(p, opt, ranges, rparent);
  if (!e.empty()) return e;
  e = cholesky(p, tau, not_spd);
  if (!e.empty()) return e;
  e = build_solve_plan(p, ranges, rparent, opt);
  if (!e.empty()) return e;
  return build_apex(p, opt);
}

}  // namespace mr
