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

// A factor on the device, in the layout the solve reads.  For supernode s:
//   l21 [l21_off[s] ..]: its struct rows of L, nstr x ncol column-major;
//   linv [linv_off[s] ..]: the inverse of its lower-triangular diagonal
//     block, ncol x ncol column-major (zero above the diagonal), formed on
//     the host in FP64, so that the diagonal solves are products;
//   its update vector in the solve's scratch at str_off[s] (nstr entries).
// Supernodes are listed by height (lvl_node[lvl_off[h] .. lvl_off[h+1])):
// the forward solve runs the heights up, the backward solve down.
struct SpDevice {
  int n = 0, nsn = 0, nlev = 0, grounded = 0;
  int max_front = 0, max_ncol = 0;
  int64_t nstr_total = 0;
  int64_t nnz = 0;            // doubles in l21 and linv
  double seconds = 0.0;       // host factorisation time
  DevBuf perm, iperm, col0, str_off, str, map, child_off, child_idx, lvl_off, lvl_node;
  DevBuf l21_off, linv_off, l21, linv;
  // complex128 entries of solve scratch per right-hand side: the permuted
  // vector (n) and the update vectors (nstr_total)
  int64_t scratch_entries() const { return n + nstr_total; }
};

// The device arrays of a factor, formed on the host.
struct SpArrays {
  int nlev = 0, max_ncol = 0;
  std::vector<int> iperm, lvl_off, lvl_node;
  std::vector<long> l21_off, linv_off;
  std::vector<double> l21, linv;
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
