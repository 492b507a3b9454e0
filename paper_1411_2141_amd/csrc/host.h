// Host-side (CPU) pre-computation of one registration pair: mesh tables,
// P1 operators, nested-dissection ordering, FP64 Cholesky factor and the
// block schedule of the triangular solves.  Plain C++17, no HIP: this part is
// built with g++ (and sanitizers) as well as hipcc.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mr {

// Tables T1-T6 of the pre-computation step of Algorithm 1.
struct MeshTables {
  std::vector<int64_t> t1_ptr, t1_slot;   // node -> slots 3*tri+corner, slots in triangle order
  std::vector<int64_t> t2_ptr, t2_idx;    // 1-ring, ascending
  std::vector<int64_t> t3_ptr, t3_idx;    // operator pattern = 1-ring + diagonal, ascending
  std::vector<int64_t> t4;                // twice the signed area per triangle
  std::vector<int64_t> t5;                // per node: sum of t4 over its triangles
  std::vector<int32_t> t6;                // per pixel: lowest-id triangle holding its centre
};

// Cholesky factor L of P S P^T stored by columns (CSC), rows ascending, with the
// diagonal first in every column.
struct Factor {
  int32_t n = 0;
  std::vector<int64_t> colptr;
  std::vector<int32_t> rowidx;
  std::vector<double> val;
  std::vector<int32_t> parent;            // elimination tree
};

// A block of consecutive rows [r0, r1) of the permuted system, solved as one
// unit (a supernode): its dense diagonal block of L is inverted, and the rows
// of L below it that its columns touch form a dense panel.
struct SolveBlock {
  int32_t r0, r1;
  int32_t parent;                          // block id, -1 for a root
  int32_t fwd_level, bwd_level;
  int32_t fwd_group;                       // lanes per row for the forward gathers
};

// One block of the apex in apex positions: rows [a0, a1); c0 = first apex
// position of its subtree; anc_off / n_anc index SolvePlan::apex_anc;
// anc_rows = rows of all its ancestors.
struct ApexBlock {
  int32_t a0, a1, c0, anc_off, n_anc, anc_rows;
};

struct SolvePlan {
  std::vector<SolveBlock> blocks;
  // dense inverses of the diagonal blocks, packed lower triangles:
  // column-major (forward) and row-major (backward), both b(b+1)/2 per block
  // (each block's entries start at an even offset, as do the panels')
  std::vector<int64_t> dense_off;          // per block, same offset in both arrays
  std::vector<double> dinv_col, dinv_row;
  // rows below each block touched by its columns, ascending; the positions
  // below_ptr[s] + k also index the forward update buffer
  std::vector<int64_t> below_ptr;          // nb + 1
  std::vector<int32_t> below_idx;
  // dense panels L(below(s), r0:r1): m x b, row-major, at panel_off[s]
  std::vector<int64_t> panel_off;
  std::vector<double> panel_row;
  // per row: update-buffer positions that contribute to it (ascending block)
  std::vector<int64_t> cptr;               // n + 1
  std::vector<int32_t> cidx;
  int32_t n_fwd_levels = 0, n_bwd_levels = 0;
  int32_t max_below = 0;
  // Apex: the top of the block tree (blocks with fwd_level >= apex_level),
  // solved with X = L(apex, apex)^-1 held explicitly.  X(i, j) can be nonzero
  // only when j's block lies in the subtree of i's block (the inverse of a
  // triangular factor keeps the elimination-tree ancestry), and in nested-
  // dissection order the apex rows of a subtree are one contiguous run of
  // apex positions.  So row i of X is kept from column apex_c0[i] to the
  // diagonal (forward), and column j of X over the rows of j's block from j on
  // followed by the rows of that block's ancestors (backward).
  int32_t apex_level = 0;                  // == n_fwd_levels when there is no apex
  std::vector<uint8_t> is_apex;            // per block
  std::vector<int32_t> apex_rows;          // solve rows of the apex, ascending
  std::vector<ApexBlock> apex_blocks;      // ascending apex position
  std::vector<int32_t> apex_anc;           // per apex block: its ancestors (apex block ids), parent first
  std::vector<int32_t> apex_c0;            // per apex row
  std::vector<int32_t> apex_blk;           // per apex row: its apex block
  std::vector<int64_t> apex_xf_off;        // apex rows + 1: X(i, apex_c0[i] .. i) at apex_xf_off[i]
  std::vector<double> apex_xf;
  std::vector<int64_t> apex_xb_off;        // apex rows + 1: X(path(j), j) at apex_xb_off[j]
  std::vector<double> apex_xb;
  std::vector<int64_t> apex_cptr;          // apex rows + 1
  std::vector<int32_t> apex_cidx;          // update-buffer positions written by non-apex blocks
};

struct PairHost {
  int32_t height = 0, width = 0, n = 0, nt = 0;
  double alpha = 0.0;
  std::vector<int32_t> xy;                 // [n][2]
  std::vector<int32_t> tri;                // [nt][3]
  MeshTables tab;
  std::vector<double> kval;                // stiffness on the t3 pattern
  std::vector<int64_t> mval;               // 24 * mass on the t3 pattern (integer)
  std::vector<int32_t> perm, iperm;        // perm[k] = node eliminated k-th
  Factor L;
  std::vector<int64_t> L_rowptr;           // strict lower pattern of L by rows,
  std::vector<int32_t> L_rowcol;           // columns ascending (from the symbolic phase)
  SolvePlan plan;
};

// Longest backward path (rows of a block plus rows of its ancestors) an apex
// may have; the device stages one path in 32 KB of LDS.
constexpr int32_t kApexPathMax = 2048;

struct OrderOptions {
  int32_t leaf_max = 32;                   // nested-dissection leaf size
  int32_t block_max = 96;                  // largest dense diagonal block
  double nd_balance = 0.3;                 // nested dissection: smallest side fraction of a cut
  int32_t nd_score = 1;                    // nested dissection cut score: 0 separator size,
                                           // 1 separator size / (left x right)
  int32_t apex_max = 1 << 30;              // most apex rows (0: no apex)
  int64_t apex_level_entries = 1 << 21;    // most entries of X one level may add (per direction)
};

// Each returns an empty string on success, else the reason.
std::string validate_mesh(const PairHost &p);
std::string build_tables(PairHost &p);
void build_operators(PairHost &p);
std::string nested_dissection(PairHost &p, const OrderOptions &opt,
                              std::vector<std::pair<int32_t, int32_t>> &ranges,
                              std::vector<int32_t> &range_parent);
// Symbolic + numeric factorisation of P (I + tau alpha K) P^T.  Returns "" or
// a message; sets *not_spd when a pivot is not positive.
std::string cholesky(PairHost &p, double tau, bool *not_spd);
// Numeric refactorisation with the symbolic structure of p.L reused.
std::string refactor(PairHost &p, double tau, bool *not_spd);
std::string build_solve_plan(PairHost &p, const std::vector<std::pair<int32_t, int32_t>> &ranges,
                             const std::vector<int32_t> &range_parent, const OrderOptions &opt);
// Numeric parts of the plan (after a refactor with unchanged structure).
void fill_dense_inverses(PairHost &p);
void fill_panels(PairHost &p);
// Chooses the apex (the longest top run of levels within opt.apex_max rows,
// whose backward paths fit kApexPathMax and each of whose levels adds at most
// opt.apex_level_entries entries to X) and builds its structure;
// fill_apex_inverse computes the entries of X.  Both return "" or a reason.
std::string build_apex(PairHost &p, const OrderOptions &opt);
std::string fill_apex_inverse(PairHost &p);

// Everything above in order.
std::string prepare_pair(PairHost &p, double tau, const OrderOptions &opt, bool *not_spd);

}  // namespace mr
