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

// A factor on the device, in the layout the solve reads.  The solve runs the
// dissection levels (supernodes grouped by height) as flat phases of
// independent row tasks:
//   forward, heights up:
//     fronts: each supernode's front (its entries of the vector, plus its
//       children's update vectors at their positions: a gather list per
//       front entry, in child order);
//     column tasks (one per column i of a supernode): y_i = (L_ss^-1 v)_i,
//       with the inverse of the diagonal block formed on the host in FP64;
//     struct tasks (one per struct row t): u_t = v_t - (L_21 y)_t;
//   backward, heights down:
//     column tasks: z_j = y_j - (L_21^T x_struct)_j;
//     column tasks: x_i = (L_ss^-T z)_i.
// Every matrix is stored twice, column-major and row-major, so that each
// phase reads it with consecutive tasks at consecutive addresses.
struct SpDevice {
  int n = 0, nsn = 0, nlev = 0, grounded = 0;
  int max_front = 0, max_ncol = 0;
  int64_t nstr_total = 0, front_total = 0;
  int64_t nnz = 0;            // doubles of the factor as stored (both copies)
  double seconds = 0.0;       // host factorisation time
  DevBuf perm, iperm, str;
  DevBuf fr_lvl, fr_dest, fr_xsrc, fr_ptr, fr_src;    // front gathers, by level
  DevBuf col_lvl, col_a, col_b, col_c;                 // column tasks, by level
  DevBuf str_lvl, str_a, str_b, str_c;                 // struct tasks, by level
  DevBuf lanes;                                        // int4 per level: lanes per task of the four phases
  DevBuf l21, l21t, linv, linvt;
  // complex128 entries of solve scratch per right-hand side: the permuted
  // vector x (n), z (n), update vectors (nstr_total), fronts (front_total)
  int64_t scratch_entries() const { return 2 * n + nstr_total + front_total; }
};

// The device arrays of a factor, formed on the host.
struct SpArrays {
  int nlev = 0, max_ncol = 0;
  int64_t front_total = 0;
  std::vector<int> iperm;
  std::vector<int> fr_lvl, fr_dest, fr_xsrc, fr_ptr, fr_src;
  std::vector<int> col_lvl, str_lvl;
  // column task (one per column i of a supernode): a = {c0, ncol, i, front
  // offset}, b = {offset of its inverse block, offset of its L_21 block},
  // c = {struct offset so, nstr}
  std::vector<int> col_a, col_c;
  std::vector<long> col_b;
  // struct task (one per struct row t of a supernode): a = {c0, ncol, t,
  // front offset}, b = {offset of its L_21 block + t, update index so + t},
  // c = {nstr, 0}
  std::vector<int> str_a, str_c;
  std::vector<long> str_b;
  // per level, the lanes that share one task's sum in the phases y = L^-1 v,
  // u = v - L_21 y, z = y - L_21^T x, x = L^-T z (a power of two up to 64,
  // chosen so that the level's tasks fill about one pass of the workgroup)
  std::vector<int> lanes;
  std::vector<double> l21, l21t, linv, linvt;
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
