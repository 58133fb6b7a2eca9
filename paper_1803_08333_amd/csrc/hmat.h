// Compressed EFIE blocks: T_A and V as hierarchical matrices whose far
// blocks are low-rank factors from adaptive cross approximation (ACA), the
// compression of the paper's large example (Sec. 4: T_A and T_Phi compressed
// separately with ACA).  T_Phi = Sigma V Sigma^T, so V is compressed in its
// place.
//
// Clusters.  The RWG edges are split by recursive bisection of their
// midpoints (median of the longest axis of the bounding box, the first part
// taking a multiple of kEdgeTile edges), so that every leaf is one tile of
// kEdgeTile consecutive edges of the permuted order (the last tile ragged).
// A cluster is a range of tiles.  Each cell belongs to the tile of its edge
// that comes first in the permuted order (its home tile), and V's clusters
// are the cells of a range of tiles, so both matrices share one block
// partition.  The box of a cluster bounds the vertices of every cell of its
// edges (which holds its home cells too).
//
// Blocks.  A pair of clusters is admissible when the distance of their boxes
// is at least the near distance (2 x the longest cell edge of the mesh, so no
// near cell pair lies in a compressed block) and min(diam) <= kHmEta x that
// distance; an admissible pair is a low-rank block, an inadmissible pair of
// leaves a dense block (a pair of tiles), and any other pair is split (a leaf
// kept whole against the other's children).  Both matrices are complex
// symmetric, so only the blocks whose row cluster precedes their column
// cluster (and the diagonal tiles) are stored; each stored off-diagonal block
// also serves its transpose.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "internal.h"

namespace rfcmp {

constexpr double kHmEta = 2.0;  // admissibility parameter
constexpr int kHmKmax = 128;    // largest rank of a low-rank block
constexpr int kHmR = 8;         // right-hand sides per pass of the compressed product

struct HmNode {
  int t0 = 0, t1 = 0;           // tiles [t0, t1)
  int64_t e0 = 0, e1 = 0;       // edge positions [e0, e1) of the permuted order
  int64_t c0 = 0, c1 = 0;       // cell positions [c0, c1) (cells by home tile)
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int child[2] = {-1, -1};
};

// The cluster tree and block partition of a mesh (host).
struct HmTree {
  int64_t N = 0, C = 0, ntiles = 0;
  std::vector<int> perm_e, iperm_e;    // position -> edge, edge -> position
  std::vector<int> perm_c, iperm_c;    // position -> cell (by home tile, then index), cell -> position
  std::vector<int> cell_start;         // [ntiles + 1] first cell position homed in each tile
  // tiles of the permuted order, as the assembly reads them: the cells each
  // tile touches (ptr/cell, ascending), the rows in the tile of their local
  // edges (8 bits each, 0xFF outside), the home tile of each cell
  std::vector<int> et_ptr, et_cell, et_rows, home;
  int et_cells_max = 0;
  std::vector<HmNode> nodes;           // nodes[0] is the root
  std::vector<int> dense_I, dense_J;   // dense blocks: tile pairs I <= J
  std::vector<int> lr_a, lr_b;         // low-rank blocks: node pairs, a's ranges before b's
  double near_dist = 0.0;
};

// Build the tree and the partition of a mesh (host, O(N log N) plus the
// number of blocks).
void hm_build_tree(const MeshHost& h, HmTree& t);

// A low-rank block in positions of the permuted order: rows [r0, r0 + m),
// columns [c0, c0 + n).
struct HmLr {
  int r0, m, c0, n;
};

// A tile list entry of one operator, resolved once its ranks are known:
// a low-rank entry's factor (U for the rows, V for the columns), the first
// row it covers in the permuted order, its length and rank, and the offset
// of its projections; the list code (4 b + kind) for every entry.
struct HmEnt {
  const float2* F;
  long zb;
  int start, len, k, code;
};

// The tree of a mesh on the device, built with the first compressed
// operator and kept with the mesh.
struct HmMesh {
  HmTree t;
  DevBuf perm_e, perm_c, iperm_c, cell_start;
  DevBuf et_ptr, et_cell, et_rows, home;
  DevBuf dense_ij;          // int2 [ndense]: tile pairs I <= J
  DevBuf vd_off;            // int64 [ndense]: offsets of the dense V blocks
  int64_t vd_total = 0;     // complex entries of the dense V blocks
  DevBuf lrA, lrV;          // HmLr [nlr] in edge and in cell positions
  // per tile, the blocks its rows meet, in a fixed order: code 4 b + kind,
  // kind 0: dense block b with I = tile, 1: dense block b with J = tile and
  // I < J (its transpose), 2: low-rank block b with the tile in its rows,
  // 3: the same with the tile in its columns (the transpose)
  DevBuf list_ptr, list_ent;
  std::vector<int> list_host;  // list_ent on the host
};

// The compressed blocks of one operator.
struct HmOp {
  double tol = 0.0;
  DevBuf TAd;               // complex64 [ndense][kEdgeTile][kEdgeTile]
  DevBuf Vd;                // complex64 dense V blocks (vd_off)
  DevBuf NV;                // complex64 [near pairs]: V of each near pair
  std::vector<std::unique_ptr<DevBuf>> store;  // low-rank factors (one buffer per ACA pass)
  DevBuf uA, vA, uV, vV;    // float2* [nlr]: U (m x k, column-major) and V (n x k) of each block
  DevBuf rankA, rankV;      // int [nlr]
  DevBuf zwA, zwV;          // int64 [nlr]: offsets of the projections in the product scratch
  DevBuf entA, entV;        // HmEnt [list entries] of T_A and V
  int64_t zw_total = 0;     // complex128 entries of that scratch
  std::vector<int> hrankA, hrankV;  // host copies of the ranks
  int64_t lr_entries[2] = {0, 0}, dense_entries[2] = {0, 0};  // complex64 entries stored (T_A, V)
  int unconverged = 0;      // blocks that reached kHmKmax above the tolerance
  DevBuf xp, yp, zw;        // product scratch: permuted input, projections
};

// Build (once per mesh) and upload the tree.
rfcmp_status hm_mesh_setup(rfcmp_mesh m, hipStream_t s);
// ACA of every low-rank block of T_A and V (after the dense blocks and the
// near pairs' V entries are assembled); waits for the stream.
rfcmp_status hm_aca(rfcmp_op op, hipStream_t s);
// y = M x or conj(M) x for M = T_A (which 0) or V (which 1), x, y complex128
// [nr][n] in the mesh's numbering.
rfcmp_status hm_matvec(rfcmp_op op, int which, bool conj, const double2* x, double2* y, int nr, hipStream_t s);
// The compressed blocks written out dense, complex64 [N][N] and [C][C].
rfcmp_status hm_export(rfcmp_op op, float2* TA, float2* V, hipStream_t s);

}  // namespace rfcmp
