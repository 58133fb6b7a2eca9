// Sparse Cholesky factorisation of the projector matrices (spchol.cpp) and
// its solve on the device (spsolve.hip).
//
// The projectors of Sec. 2 and Sec. 3 need (Sigma^T Sigma)^+, G_ll^-1 and
// G_tp^-1 applied to vectors.  All three matrices are sparse and symmetric
// positive (semi)definite on a surface mesh: the cell graph Laplacian (4
// entries per row), the P1 mass matrix on the vertex graph (about 7), the
// mixed Gram matrix on cells sharing a vertex (about 13).  Each is factored
// once per mesh, P A P^T = L L^T, with a nested-dissection order P from the
// mesh coordinates (recursive bisection at the median of the longest axis;
// the nodes on one side with a neighbour on the other form the separator).
// Supernodes are the nodes of the dissection tree (leaves and separators,
// each a contiguous range of the order) with dense diagonal blocks; the
// factor is formed multifrontally in FP64.  A surface mesh is a planar-like
// graph, so the separators have O(sqrt n) nodes and the factor O(n log n)
// entries: a solve reads a few MB where the dense inverse reads 8 n^2 bytes.
//
// The Laplacian is singular (its kernel is the constant vector on a
// connected mesh).  It is factored as L + e_g e_g^T for the last node g of
// the order, which is SPD; for a mean-free y the solution x of
// (L + e_g e_g^T) x = y has x_g = 1^T y = 0, so L x = y, and
// L^+ y = x - mean(x).  The solve therefore projects its input and its output
// onto the mean-free vectors.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"
#include "symv.h"

namespace rfcmp {

// Symmetric sparse matrix with both triangles stored (CSR) and one point in
// space per row (its cell centroid or vertex).
struct SpMatrix {
  int n = 0;
  std::vector<int> ptr, idx;
  std::vector<double> val;
  std::vector<double> xyz;  // [n][3]
};

// Factor of one matrix, host side.  Supernodes are numbered in elimination
// order (children before parents).  For supernode s:
//   columns col0[s] .. col0[s+1]-1 of the permuted matrix (ncol of them);
//   struct rows str[str_off[s] .. str_off[s+1]) (permuted indices beyond its
//     columns, ascending; nstr of them);
//   its front has m = ncol + nstr rows: its columns, then its struct rows;
//   panel[panel_off[s] ..] holds the m x ncol block of L column-major (rows
//     as in the front; the strictly upper part of the diagonal block is 0);
//   parent[s]: the supernode that holds str[str_off[s]] (-1 at a root);
//   map[str_off[s] + t]: position of struct row t in the parent's front;
//   height[s]: 0 for a supernode without children, else 1 + the largest
//     height of its children.
struct SpFactor {
  int n = 0, nsn = 0;
  bool grounded = false;     // Laplacian: L + e_g e_g^T, g = last node
  std::vector<int> perm;     // perm[i] = row of the original matrix at position i
  std::vector<int> col0;     // [nsn + 1]
  std::vector<int> str_off;  // [nsn + 1]
  std::vector<int> str, map;
  std::vector<int64_t> panel_off;  // [nsn + 1]
  std::vector<double> panel;
  std::vector<int> parent, height;
  std::vector<int> child_off, child_idx;  // children of each supernode, ascending
  int max_front = 0;         // largest m
  double seconds = 0.0;      // host time of ordering, symbolic and numeric factorisation
  double sec_order = 0.0, sec_symbolic = 0.0, sec_numeric = 0.0;
  int64_t nnz() const { return panel_off.empty() ? 0 : panel_off.back(); }
};

// Factor A (SPD, or a connected graph Laplacian with grounded = true).
// leaf: most nodes in a dissection leaf.  threads: host threads for the
// independent subtrees.  Returns RFCMP_E_ARG if a pivot is not positive.
rfcmp_status spchol_factor(const SpMatrix& A, bool grounded, int leaf, int threads, SpFactor& F);

// Entries per tile of the permutation kernels (input, output, partial sums).
constexpr int kSpTile = 64;

// A factor on the device, in the layout the solve reads.
//
// The supernodes split into bottom subtrees (every supernode whose subtree
// spans at most about n/96 columns and holds only supernodes whose blocks
// have at most 1024 entries, grouped under the highest such supernodes) and
// the top supernodes above them.  A solve is a short chain of
// launches, each over many workgroups (and right-hand sides):
//   input: the right-hand side formed (the operator's gathers) and permuted,
//     a tile of entries by 16 right-hand sides per workgroup, transposed
//     through LDS (for the Laplacian also its partial sums, then their mean);
//   forward, bottom: one workgroup per subtree, its heights in order, one
//     wave per supernode, which loads the supernode's blocks, its gather
//     indices and its entries of the vector into LDS with all loads in
//     flight, then its children's update entries, and forms the products
//     from LDS (the Laplacian's input mean taken off as the columns are
//     read);
//   forward, top: one launch per height, one workgroup per supernode;
//   backward, top: heights down, one launch each (the highest height's
//     roots take their backward step in the forward launch);
//   backward, bottom: one workgroup per subtree;
//   output: permuted back (for the Laplacian less the mean of the result,
//     from partial sums over tiles).
// A supernode's forward step builds its front (its entries of the vector plus
// its children's update vectors, gathered per front entry in child order),
// forms y = L_ss^-1 v with the inverse of its diagonal block (formed on the
// host in FP64) and its update vector u = v_struct - L_21 y; its backward
// step forms z = y - L_21^T x_struct and x = L_ss^-T z.  Every matrix is stored
// column- and row-major, so that each step reads it with neighbouring lanes at
// neighbouring addresses.  A workgroup takes R right-hand sides at once (R
// chosen per launch from the grid it gives and the LDS its fronts need): each
// matrix entry it loads serves all R.
struct SpDevice {
  int n = 0, nsn = 0, grounded = 0;
  int max_front = 0, max_ncol = 0;
  int nsub = 0, ntop = 0;                    // bottom subtrees, top heights
  // LDS of a bottom supernode's wave (its blocks staged): ncol + nstr
  // entries per right-hand side (forward: the front; backward: x_struct and
  // z), its blocks (doubles) and its gather indices (ints); the largest over
  // the bottom supernodes, bot_fac even and bot_idx a multiple of 4; the
  // most columns of a bottom supernode (at most 32: staged blocks hold at
  // most 1024 entries)
  int bot_lds = 0, bot_fac = 0, bot_idx = 0, bot_ncol = 0;
  int64_t nstr_total = 0, front_total = 0;
  int64_t nnz = 0;            // doubles of the factor as stored (both copies)
  double seconds = 0.0;       // host factorisation time
  DevBuf perm, iperm, col0, str_off, str, front_off;
  // per front entry, the child update entries that land there: fr_k slots
  // each (fr_k = the most over the factor), unused slots -1
  DevBuf fr_src;
  int fr_k = 0;
  DevBuf linv_off, l21_off, l21, l21t, linv, linvt;
  // the blocks of each bottom supernode staged in LDS by the solve, L_ss^-1
  // then L_21 (both column-major) contiguously, at blk_off
  DevBuf blk_off, blk;
  // bottom subtrees: levels, and per position the supernode's descriptor
  // {col0, ncol, str_off, nstr}, {front_off, blk_off, 0, 0}
  DevBuf sub_ptr, sub_lvl, sub_desc;
  // top supernodes by height: per position the descriptor {col0, ncol,
  // str_off, nstr}, {front_off, linv_off, l21_off, 0}; the first position of
  // each height (host)
  DevBuf top_desc;
  std::vector<int> top_start;
  bool top_roots = false;  // the highest top height holds roots only (no struct rows)
  // per top height (host copies): supernodes, and the largest LDS need
  std::vector<int> top_count, top_lds;
  // complex128 entries of solve scratch per right-hand side: the permuted
  // vector x (n), the update vectors (nstr_total), partial sums of x over
  // tiles of kSpTile entries, and the two means of the Laplacian solve (of
  // the input and of the result).  The scratch holds them right-hand side
  // fastest: entry e of right-hand side r at e * nrhs + r, so that the
  // right-hand sides of a workgroup sit together.
  int64_t tiles() const { return (n + kSpTile - 1) / kSpTile; }
  int64_t scratch_entries() const { return n + nstr_total + tiles() + 2; }
};

// The device arrays of a factor, formed on the host.
struct SpArrays {
  int max_ncol = 0, nsub = 0, ntop = 0, bot_lds = 0, bot_fac = 0, bot_idx = 0, bot_ncol = 0;
  int64_t front_total = 0;
  std::vector<int> iperm, front_off, fr_src;
  int fr_k = 0;
  std::vector<long> linv_off, l21_off, blk_off;
  std::vector<double> l21, l21t, linv, linvt, blk;
  std::vector<int> sub_ptr, sub_lvl, sub_nodes, sub_desc, top_lvl, top_nodes, top_desc;
  std::vector<int> top_count, top_lds;
  bool top_roots = false;
};
void spchol_arrays(const SpFactor& F, SpArrays& out);

// Upload a host factor (enqueued on s; the host arrays must stay alive until
// the copies complete: the call synchronises s).
rfcmp_status spchol_upload(const SpFactor& F, SpDevice& D, hipStream_t s);

// y_r = A^-1 x_r (grounded: L^+ x_r) for nrhs right-hand sides of up to two
// factors in one launch, the inputs formed from SymvInput as in the dense
// products.  scratch: per job, nrhs * scratch_entries() complex128.
struct SpSolveJob {
  const SpDevice* F = nullptr;
  SymvInput in;
  double2* y = nullptr;        // [nrhs][n]
  double2* scratch = nullptr;
  int nrhs = 0;                // job 1 of a pair: 0 = the same as job 0
};
rfcmp_status spsolve_jobs(const SpSolveJob* jobs, int njobs, int nrhs, hipStream_t s, const char* tag);

// The three projector matrices of a mesh as sparse matrices (Sec. 2, Sec. 3).
void laplacian_matrix(const MeshHost& h, SpMatrix& A);   // Sigma^T Sigma
void gram_ll_matrix(const MeshHost& h, SpMatrix& A);     // P1 mass matrix
void gram_tp_matrix(const MeshHost& h, SpMatrix& A);     // mixed Gram (needs h.cell_nb_*)

}  // namespace rfcmp
