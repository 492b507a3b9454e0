// Host pre-computation check, built with g++ and the address and undefined-
// behaviour sanitizers by tests/test_host_sanitized.py.
//
// Reads one mesh, runs the library's host pipeline (validation, tables T1-T6,
// operators, nested dissection, Cholesky factor, block schedule, apex), then
// carries out the triangular solves the way the device schedule prescribes
// (forward levels below the apex pushing panel updates, the apex through its
// explicit inverse X, backward levels pulling the solved rows below each
// block) in plain sequential C++, and prints the residual of
// (I + tau alpha K) x = b for the stiffness the host built.  The same check
// is repeated after a numeric refactorisation with another alpha.
//
// Usage: plan_check MESH_FILE TAU ALPHA ALPHA2 APEX_MAX
// MESH_FILE: int32 height, width, n, nt, then n (x, y) pairs, then nt triples.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1411_2141_amd/csrc/host.h"

using namespace mr;

namespace {

bool read_mesh(const char *path, PairHost &p) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return false;
  int32_t hdr[4];
  bool ok = std::fread(hdr, sizeof(int32_t), 4, f) == 4;
  if (ok) {
    p.height = hdr[0];
    p.width = hdr[1];
    p.n = hdr[2];
    p.nt = hdr[3];
    p.xy.resize(2 * (size_t)p.n);
    p.tri.resize(3 * (size_t)p.nt);
    ok = std::fread(p.xy.data(), sizeof(int32_t), p.xy.size(), f) == p.xy.size() &&
         std::fread(p.tri.data(), sizeof(int32_t), p.tri.size(), f) == p.tri.size();
  }
  std::fclose(f);
  return ok;
}

// x = S^-1 b through the block schedule (rows in solve order inside).
std::vector<double> schedule_solve(const PairHost &p, const std::vector<double> &b) {
  const SolvePlan &pl = p.plan;
  const int n = p.n;
  std::vector<double> y(n), upd(pl.below_idx.size(), 0.0);
  for (int k = 0; k < n; ++k) y[k] = b[p.perm[k]];
  auto below_rows = [&](size_t s) { return pl.below_ptr[s + 1] - pl.below_ptr[s]; };
  // forward levels below the apex: t = b - pushed updates, y = D^-1 t, push P y
  for (int lev = 0; lev < pl.apex_level; ++lev)
    for (size_t s = 0; s < pl.blocks.size(); ++s) {
      const SolveBlock &B = pl.blocks[s];
      if (B.fwd_level != lev || pl.is_apex[s]) continue;
      const int bb = B.r1 - B.r0;
      std::vector<double> t(bb), yb(bb);
      for (int r = 0; r < bb; ++r) {
        double a = 0.0;
        for (int64_t q = pl.cptr[B.r0 + r]; q < pl.cptr[B.r0 + r + 1]; ++q) a += upd[pl.cidx[q]];
        t[r] = y[B.r0 + r] - a;
      }
      const int64_t off = pl.dense_off[s];
      for (int i = 0; i < bb; ++i) {
        double a = 0.0;
        for (int j = 0; j <= i; ++j)
          a += pl.dinv_col[off + (int64_t)j * bb - (int64_t)j * (j - 1) / 2 + (i - j)] * t[j];
        yb[i] = a;
        y[B.r0 + i] = a;
      }
      const int64_t k0 = pl.below_ptr[s], po = pl.panel_off[s];
      for (int64_t k = 0; k < below_rows(s); ++k) {
        double a = 0.0;
        for (int j = 0; j < bb; ++j) a += pl.panel_row[po + k * bb + j] * yb[j];
        upd[k0 + k] = a;
      }
    }
  // apex: t = b - updates of the blocks below, y = X t (row segments), then
  // z = X^T y (column paths)
  const int64_t na = (int64_t)pl.apex_rows.size();
  if (na > 0) {
    std::vector<double> t(na), ya(na);
    for (int64_t i = 0; i < na; ++i) {
      double a = 0.0;
      for (int64_t q = pl.apex_cptr[i]; q < pl.apex_cptr[i + 1]; ++q) a += upd[pl.apex_cidx[q]];
      t[i] = y[pl.apex_rows[i]] - a;
    }
    for (int64_t i = 0; i < na; ++i) {
      double a = 0.0;
      for (int64_t j = pl.apex_c0[i]; j <= i; ++j)
        a += pl.apex_xf[pl.apex_xf_off[i] + (j - pl.apex_c0[i])] * t[j];
      ya[i] = a;
    }
    for (int64_t j = 0; j < na; ++j) {
      const ApexBlock &A = pl.apex_blocks[pl.apex_blk[j]];
      int64_t k = pl.apex_xb_off[j];
      double a = 0.0;
      for (int64_t i = j; i < A.a1; ++i) a += pl.apex_xb[k++] * ya[i];
      for (int g = A.anc_off; g < A.anc_off + A.n_anc; ++g) {
        const ApexBlock &G = pl.apex_blocks[pl.apex_anc[g]];
        for (int64_t i = G.a0; i < G.a1; ++i) a += pl.apex_xb[k++] * ya[i];
      }
      if (k != pl.apex_xb_off[j + 1]) {
        std::printf("apex path length mismatch at %lld\n", (long long)j);
        std::exit(2);
      }
      y[pl.apex_rows[j]] = a;
    }
  }
  // backward levels below the apex, top first: t = y - P^T z(below), z = D^-T t
  for (int lev = pl.apex_level - 1; lev >= 0; --lev)
    for (size_t s = 0; s < pl.blocks.size(); ++s) {
      const SolveBlock &B = pl.blocks[s];
      if (B.fwd_level != lev || pl.is_apex[s]) continue;
      const int bb = B.r1 - B.r0;
      std::vector<double> t(bb);
      const int64_t k0 = pl.below_ptr[s], po = pl.panel_off[s];
      for (int j = 0; j < bb; ++j) {
        double a = 0.0;
        for (int64_t k = 0; k < below_rows(s); ++k)
          a += pl.panel_row[po + k * bb + j] * y[pl.below_idx[k0 + k]];
        t[j] = y[B.r0 + j] - a;
      }
      const int64_t off = pl.dense_off[s];
      for (int j = 0; j < bb; ++j) {
        double a = 0.0;
        for (int i = j; i < bb; ++i) a += pl.dinv_row[off + (int64_t)i * (i + 1) / 2 + j] * t[i];
        y[B.r0 + j] = a;
      }
    }
  std::vector<double> x(n);
  for (int k = 0; k < n; ++k) x[p.perm[k]] = y[k];
  return x;
}

// max |(I + tau alpha K) x - b| / max |b|, K on the T3 pattern.
double residual(const PairHost &p, double tau, const std::vector<double> &x,
                const std::vector<double> &b) {
  double rmax = 0.0, bmax = 0.0;
  for (int i = 0; i < p.n; ++i) {
    double a = x[i];
    for (int64_t q = p.tab.t3_ptr[i]; q < p.tab.t3_ptr[i + 1]; ++q)
      a += tau * p.alpha * p.kval[q] * x[p.tab.t3_idx[q]];
    rmax = std::fmax(rmax, std::fabs(a - b[i]));
    bmax = std::fmax(bmax, std::fabs(b[i]));
  }
  return rmax / bmax;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 6) {
    std::fprintf(stderr, "usage: plan_check MESH TAU ALPHA ALPHA2 APEX_MAX\n");
    return 2;
  }
  PairHost p;
  if (!read_mesh(argv[1], p)) {
    std::fprintf(stderr, "cannot read %s\n", argv[1]);
    return 2;
  }
  const double tau = std::atof(argv[2]);
  p.alpha = std::atof(argv[3]);
  const double alpha2 = std::atof(argv[4]);
  OrderOptions opt;
  opt.apex_max = std::atoi(argv[5]);
  bool not_spd = false;
  std::string e = prepare_pair(p, tau, opt, &not_spd);
  if (!e.empty()) {
    std::printf("prepare failed: %s\n", e.c_str());
    return 3;
  }
  std::vector<double> b(p.n);
  for (int i = 0; i < p.n; ++i) b[i] = std::sin(0.37 * i) + 1.5;
  const double r1 = residual(p, tau, schedule_solve(p, b), b);
  // numeric refactorisation with the structure kept (set_alpha's path)
  p.alpha = alpha2;
  e = refactor(p, tau, &not_spd);
  if (!e.empty()) {
    std::printf("refactor failed: %s\n", e.c_str());
    return 3;
  }
  fill_dense_inverses(p);
  fill_panels(p);
  e = fill_apex_inverse(p);
  if (!e.empty()) {
    std::printf("apex refill failed: %s\n", e.c_str());
    return 3;
  }
  const double r2 = residual(p, tau, schedule_solve(p, b), b);
  std::printf("n %d blocks %zu fwd_levels %d apex_rows %zu residual %.3e refactored %.3e\n", p.n,
              p.plan.blocks.size(), p.plan.n_fwd_levels, p.plan.apex_rows.size(), r1, r2);
  return 0;
}
