// Mesh validation, tables T1-T6 and the P1 operators of one pair.
//
// The mesh (V, T) is the paper's Section 2.1 input; the tables are the
// pre-computation of Algorithm 1 (1-ring N_1 and each node's neighbour
// triangles) plus the pixel->triangle map used to reconstruct the dense
// displacement (Section 1, Fig. 3).  The operators are the P1 stiffness K (the
// symmetric mesh Laplacian behind Section 2.3's diffusion smoothing) and the
// consistent mass M whose area weighting is eq. 10's triangle-to-node average.
#include <algorithm>
#include <cstdio>

#include "host.h"

namespace mr {

namespace {

inline int64_t cross2(int64_t ax, int64_t ay, int64_t bx, int64_t by) { return ax * by - ay * bx; }

}  // namespace

std::string validate_mesh(const PairHost &p) {
  char buf[256];
  if (p.height < 1 || p.width < 1) return "image sides must be >= 1";
  if (p.height > 32768 || p.width > 32768) return "image sides must be <= 32768";
  if (p.n < 3 || p.nt < 1) return "mesh needs >= 3 nodes and >= 1 triangle";
  for (int32_t i = 0; i < p.n; ++i) {
    const int32_t x = p.xy[2 * i], y = p.xy[2 * i + 1];
    if (x < 0 || x > p.width || y < 0 || y > p.height) {
      std::snprintf(buf, sizeof buf, "node %d at (%d, %d) outside [0,%d]x[0,%d]", i, x, y,
                    p.width, p.height);
      return buf;
    }
  }
  std::vector<uint8_t> used(p.n, 0);
  for (int32_t t = 0; t < p.nt; ++t) {
    for (int a = 0; a < 3; ++a) {
      const int32_t v = p.tri[3 * t + a];
      if (v < 0 || v >= p.n) {
        std::snprintf(buf, sizeof buf, "triangle %d corner %d: node index %d out of range", t, a, v);
        return buf;
      }
      used[v] = 1;
    }
    const int32_t *c = &p.tri[3 * t];
    const int64_t ax = p.xy[2 * c[0]], ay = p.xy[2 * c[0] + 1];
    const int64_t area2 = cross2(p.xy[2 * c[1]] - ax, p.xy[2 * c[1] + 1] - ay,
                                 p.xy[2 * c[2]] - ax, p.xy[2 * c[2] + 1] - ay);
    if (area2 <= 0) {
      std::snprintf(buf, sizeof buf, "triangle %d has non-positive signed area", t);
      return buf;
    }
  }
  for (int32_t i = 0; i < p.n; ++i)
    if (!used[i]) {
      std::snprintf(buf, sizeof buf, "node %d is not used by any triangle", i);
      return buf;
    }
  return "";
}

std::string build_tables(PairHost &p) {
  MeshTables &tb = p.tab;
  const int32_t n = p.n, nt = p.nt;
  // T4
  tb.t4.assign(nt, 0);
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t *c = &p.tri[3 * t];
    const int64_t ax = p.xy[2 * c[0]], ay = p.xy[2 * c[0] + 1];
    tb.t4[t] = cross2(p.xy[2 * c[1]] - ax, p.xy[2 * c[1] + 1] - ay, p.xy[2 * c[2]] - ax,
                      p.xy[2 * c[2] + 1] - ay);
  }
  // T1: counting sort of slots by node; triangles visited in id order keep each
  // node's slots sorted by triangle id.
  tb.t1_ptr.assign(n + 1, 0);
  for (int32_t s = 0; s < 3 * nt; ++s) tb.t1_ptr[p.tri[s] + 1]++;
  for (int32_t i = 0; i < n; ++i) tb.t1_ptr[i + 1] += tb.t1_ptr[i];
  tb.t1_slot.assign(3 * (size_t)nt, 0);
  {
    std::vector<int64_t> next(tb.t1_ptr.begin(), tb.t1_ptr.end() - 1);
    for (int32_t s = 0; s < 3 * nt; ++s) tb.t1_slot[next[p.tri[s]]++] = s;
  }
  // T5
  tb.t5.assign(n, 0);
  for (int32_t s = 0; s < 3 * nt; ++s) tb.t5[p.tri[s]] += tb.t4[s / 3];
  // T2 / T3: per node, the other corners of its triangles, sorted and unique
  tb.t2_ptr.assign(n + 1, 0);
  tb.t3_ptr.assign(n + 1, 0);
  tb.t2_idx.clear();
  tb.t3_idx.clear();
  std::vector<int64_t> row;
  for (int32_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t k = tb.t1_ptr[i]; k < tb.t1_ptr[i + 1]; ++k) {
      const int64_t s = tb.t1_slot[k];
      const int64_t t = s / 3, a = s % 3;
      row.push_back(p.tri[3 * t + (a + 1) % 3]);
      row.push_back(p.tri[3 * t + (a + 2) % 3]);
    }
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    for (int64_t j : row) tb.t2_idx.push_back(j);
    tb.t2_ptr[i + 1] = (int64_t)tb.t2_idx.size();
    auto pos = std::lower_bound(row.begin(), row.end(), (int64_t)i);
    row.insert(pos, (int64_t)i);
    for (int64_t j : row) tb.t3_idx.push_back(j);
    tb.t3_ptr[i + 1] = (int64_t)tb.t3_idx.size();
  }
  // T6: triangles in increasing id claim the unclaimed pixel centres they hold
  // (closed test in doubled integer coordinates), so ties go to the lowest id.
  const int32_t H = p.height, W = p.width;
  tb.t6.assign((size_t)H * W, -1);
  for (int32_t t = 0; t < nt; ++t) {
    int64_t P[3][2];
    int64_t xmin = INT64_MAX, xmax = INT64_MIN, ymin = INT64_MAX, ymax = INT64_MIN;
    for (int a = 0; a < 3; ++a) {
      P[a][0] = 2 * (int64_t)p.xy[2 * p.tri[3 * t + a]];
      P[a][1] = 2 * (int64_t)p.xy[2 * p.tri[3 * t + a] + 1];
      xmin = std::min(xmin, P[a][0]);
      xmax = std::max(xmax, P[a][0]);
      ymin = std::min(ymin, P[a][1]);
      ymax = std::max(ymax, P[a][1]);
    }
    // pixel j has doubled centre 2j+1: need xmin <= 2j+1 <= xmax
    const int64_t j0 = std::max<int64_t>(0, xmin / 2), j1 = std::min<int64_t>(W - 1, (xmax - 1) / 2);
    const int64_t i0 = std::max<int64_t>(0, ymin / 2), i1 = std::min<int64_t>(H - 1, (ymax - 1) / 2);
    for (int64_t i = i0; i <= i1; ++i) {
      const int64_t py = 2 * i + 1;
      for (int64_t j = j0; j <= j1; ++j) {
        int32_t &dst = tb.t6[(size_t)i * W + j];
        if (dst >= 0) continue;
        const int64_t px = 2 * j + 1;
        bool in = true;
        for (int a = 0; a < 3 && in; ++a) {
          const int b = (a + 1) % 3;
          in = cross2(P[b][0] - P[a][0], P[b][1] - P[a][1], px - P[a][0], py - P[a][1]) >= 0;
        }
        if (in) dst = t;
      }
    }
  }
  for (size_t q = 0; q < tb.t6.size(); ++q)
    if (tb.t6[q] < 0) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "pixel (%zu, %zu) is not covered by any triangle", q / W,
                    q % W);
      return buf;
    }
  return "";
}

void build_operators(PairHost &p) {
  const MeshTables &tb = p.tab;
  const size_t nnz = tb.t3_idx.size();
  p.kval.assign(nnz, 0.0);
  p.mval.assign(nnz, 0);
  auto find = [&](int32_t i, int32_t j) -> int64_t {
    auto b = tb.t3_idx.begin() + tb.t3_ptr[i], e = tb.t3_idx.begin() + tb.t3_ptr[i + 1];
    return std::lower_bound(b, e, (int64_t)j) - tb.t3_idx.begin();
  };
  for (int32_t t = 0; t < p.nt; ++t) {
    const int32_t *c = &p.tri[3 * t];
    int64_t e[3][2];  // edge opposite each corner: from the next to the one after
    for (int a = 0; a < 3; ++a) {
      const int32_t b = c[(a + 1) % 3], d = c[(a + 2) % 3];
      e[a][0] = (int64_t)p.xy[2 * d] - p.xy[2 * b];
      e[a][1] = (int64_t)p.xy[2 * d + 1] - p.xy[2 * b + 1];
    }
    const int64_t w = tb.t4[t];  // twice the area
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int64_t q = find(c[a], c[b]);
        // K_T[a][b] = e_a . e_b / (4 A) = e_a . e_b / (2 w)
        p.kval[q] += (double)(e[a][0] * e[b][0] + e[a][1] * e[b][1]) / (2.0 * (double)w);
        // 24 M_T[a][b] = 2 A (1 + delta_ab) = w (1 + delta_ab)
        p.mval[q] += w * (a == b ? 2 : 1);
      }
  }
}

}  // namespace mr
