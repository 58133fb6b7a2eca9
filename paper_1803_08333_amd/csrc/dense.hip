// The FP64 inverse used to build the dense projector matrices
// (L^+ = (Sigma^T Sigma)^+, G_ll^-1, G_tp^-1) of a mesh.
#include <algorithm>
#include <cmath>

#include <memory>
#include <vector>

#include "internal.h"

namespace rfcmp {

namespace {

// ------------------------------------------------------------------------
// Blocked symmetric sweep of an SPD matrix (no pivoting: every Schur
// complement of an SPD matrix is SPD).  The scalar sweep on pivot k,
//   d = 1 / a_kk,  a_ij -= a_ik a_kj d,  a_ik *= d,  a_kj *= d,  a_kk = -d,
// keeps a symmetric matrix symmetric, and sweeping every index yields -A^-1.
// Sweeping the 64 indices of pivot block P at once, with E = A_PP^-1:
//   A_PP <- -E,  A_PJ <- E A_PJ,  A_IJ <- A_IJ - A_PI^T E A_PJ   (I, J != P).
// Only the upper block triangle (tiles I <= J) is kept up to date, which
// halves the traffic and the flops of the rank-64 updates; a final pass
// mirrors it, flips the sign and applies the requested shift.
constexpr int kB = 64;

// Sweep of the 64 pivots of a diagonal tile held in registers (leaves -E),
// four pivots S = {k, .., k+3} at a time: with F = A_SS^-1,
//   A_SS <- -F,  a_Sj <- F a_Sj,  a_iS <- a_iS F,  a_ij <- a_ij - a_iS F a_Sj,
// which is what four scalar sweeps give.  Thread t keeps the 16-entry strip
// (rows 16 (t / 64) .. +16, column t % 64) in registers.  By symmetry the
// pivot rows equal the pivot columns, so per step only the four columns are
// published to LDS ([row][4], double-buffered: one barrier per four pivots);
// every thread then forms -F by a 4 x 4 sweep of A_SS and updates its strip
// branch-free: with m_j = F a_Sj (j not in S) or column j - k of -F
// (j in S), rows of S become m_j and every other entry
// (j in S ? 0 : a_ij) - a_iS m_j.
__device__ void sweep_tile(double (&r)[16], double (*col4)[kB][4]) {
  const int j = threadIdx.x % kB;
  const int i0 = (threadIdx.x / kB) * 16;
  for (int k = 0; k < kB; k += 4) {
    const int bsel = (k >> 2) & 1;
    if (j >= k && j < k + 4) {
#pragma unroll
      for (int u = 0; u < 16; ++u) col4[bsel][i0 + u][j - k] = r[u];
    }
    __syncthreads();
    // -F by a symmetric 4 x 4 sweep of A_SS[s][t] = a_{k+s, k+t}
    double f[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) f[s][t] = col4[bsel][k + s][t];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double d = 1.0 / f[q][q];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (s != q && t != q) f[s][t] = fma(-f[s][q] * d, f[q][t], f[s][t]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s != q) {
          f[s][q] *= d;
          f[q][s] *= d;
        }
      f[q][q] = -d;
    }
    const bool inS = (j >= k && j < k + 4);
    double m[4];
    {
      double aSj[4];  // a_{k+t, j} = a_{j, k+t}
#pragma unroll
      for (int t = 0; t < 4; ++t) aSj[t] = col4[bsel][j][t];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) v = fma(f[s][t], aSj[t], v);  // (-F a_Sj)_s
        double c = f[s][0];
#pragma unroll
        for (int t = 1; t < 4; ++t) c = (j - k == t) ? f[s][t] : c;  // column j - k of -F
        m[s] = inS ? c : -v;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i0 + u;
      const double* ai = col4[bsel][i];
      double acc = inS ? 0.0 : r[u];
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = fma(-ai[s], m[s], acc);
      double rowv = m[0];
#pragma unroll
      for (int s = 1; s < 4; ++s) rowv = (i - k == s) ? m[s] : rowv;
      r[u] = (i >= k && i < k + 4) ? rowv : acc;
    }
  }
}

// Sweep of diagonal tile K in place (the first pivot block only: later
// diagonal tiles are swept by the update kernel of the previous step).
__global__ __launch_bounds__(256) void k_gj_diag(double* __restrict__ A, long ld, int K) {
  __shared__ double col4[2][kB][4];
  const int j = threadIdx.x % kB;
  const int i0 = (threadIdx.x / kB) * 16;
  const long base = (long)K * kB;
  double r[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) r[u] = A[(base + i0 + u) * ld + base + j];
  sweep_tile(r, col4);
#pragma unroll
  for (int u = 0; u < 16; ++u) A[(base + i0 + u) * ld + base + j] = r[u];
}

// Panels of pivot block K: for each J != K, U_J = A_KJ (old; tile (J, K)
// transposed when J < K) and R_J = E U_J with E = -(tile K, K), written to
// the compact panel buffers ([nb][64][64] each).  Workgroup (J, h) forms rows
// 16 h .. 16 h + 15 of R_J from those rows of E and all of U_J (staged in LDS,
// transposed there when the stored tile is A_JK).  The tiles of A are only
// read here: four workgroups read each tile, so the new panel R_J goes back
// into A in the update kernel.
__global__ __launch_bounds__(256) void k_gj_panels(const double* __restrict__ A, long ld, int K,
                                                   double* __restrict__ Ubuf, double* __restrict__ Rbuf) {
  const int J = blockIdx.x, h = blockIdx.y;
  if (J == K) return;
  constexpr int HR = kB / 4;  // rows of R_J per workgroup
  __shared__ double E[HR][kB];
  __shared__ double U[kB][kB + 2];  // U[q][c] = (U_J)_qc
  const long pb = (long)K * kB, jb = (long)J * kB;
  const bool up = J > K;
  for (int t = threadIdx.x; t < kB * kB; t += 256) {
    const int i = t / kB, c = t % kB;
    if (up)
      U[i][c] = A[(pb + i) * ld + jb + c];
    else
      U[c][i] = A[(jb + i) * ld + pb + c];  // stored tile is A_JK = U_J^T
  }
  for (int t = threadIdx.x; t < HR * kB; t += 256) {
    const int i = t / kB, c = t % kB;
    E[i][c] = -A[(pb + h * HR + i) * ld + pb + c];
  }
  __syncthreads();
  double* Uo = Ubuf + (long)J * kB * kB;
  double* Ro = Rbuf + (long)J * kB * kB;
  for (int t = threadIdx.x; t < HR * kB; t += 256) {
    const int i = h * HR + t / kB, c = t % kB;
    Uo[i * kB + c] = U[i][c];
  }
  // thread: row i = t / 16 of this quarter, columns c = 4 (t % 16) .. + 3
  const int i = threadIdx.x / 16, c0 = (threadIdx.x % 16) * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int q = 0; q < kB; ++q) {
    const double e = E[i][q];
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fma(e, U[q][c0 + v], acc[v]);
  }
  const int gi = h * HR + i;
#pragma unroll
  for (int v = 0; v < 4; ++v) Ro[gi * kB + c0 + v] = acc[v];
}

// Rank-64 update of the upper tiles: A_IJ -= U_I^T R_J for I <= J, I, J != K;
// the workgroups of the pivot row and column tiles store the new panel.
// One 64 x 64 tile per workgroup on the FP64 matrix cores: wave w owns the
// 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 blocks of 16 x 16, each a
// v_mfma_f64_16x16x4 accumulator (value v of lane l: row 4 v + l / 16,
// column l % 16), loaded from A first so that the read overlaps the staging.
// K-chunks of 32 rows of U_I and R_J sit in LDS fragment-major: the 4 x 16
// operand of (row group g, column block b) is 64 consecutive doubles with
// lane l's value (row 4 g + l / 16, column 16 b + l % 16) at position l, so
// every operand read is one conflict-free 512-byte wave load.
// Workgroup 0 takes the next diagonal tile (K+1, K+1) and, once it is
// updated, sweeps it: the serial sweep of the next pivot block runs while
// the rest of the update streams.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, long ld, int nb, int K,
                                                   const double* __restrict__ Ubuf,
                                                   const double* __restrict__ Rbuf) {
  // upper-triangle index, with 0 and the index of (K+1, K+1) swapped
  const int nx = K + 1;
  const int inext = nx < nb ? nx * nb - nx * (nx - 1) / 2 : 0;
  int lin = blockIdx.x;
  if (lin == 0)
    lin = inext;
  else if (lin == inext)
    lin = 0;
  int I = 0, rem = lin;
  while (rem >= nb - I) {
    rem -= nb - I;
    ++I;
  }
  const int J = I + rem;
  if (I == K || J == K) {
    // a tile of the pivot row or column: store the new panel, R_J into
    // tile (K, J) for J > K, R_I^T into tile (I, K) for I < K
    if (I == J) return;  // the pivot tile holds -E already
    const long ib = (long)I * kB, jb = (long)J * kB;
    const bool row = (I == K);
    const double* Rt = Rbuf + (long)(row ? J : I) * kB * kB;
    for (int t = threadIdx.x; t < kB * kB; t += 256) {
      const int i = t / kB, c = t % kB;
      A[(ib + i) * ld + jb + c] = row ? Rt[i * kB + c] : Rt[c * kB + i];
    }
    return;
  }
  constexpr int KC = 32;
  __shared__ __align__(16) double lds[2 * KC * kB];  // U chunk, R chunk
  const long ib = (long)I * kB, jb = (long)J * kB;
  const double* Ui = Ubuf + (long)I * kB * kB;
  const double* Rj = Rbuf + (long)J * kB * kB;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int wr = w / 2, wc = w % 2;
  const int r0 = wr * 32 + lane / 16, c0 = wc * 32 + lane % 16;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = A[(ib + r0 + 16 * a + 4 * v) * ld + jb + c0 + 16 * b];
  for (int k0 = 0; k0 < kB; k0 += KC) {
    for (int t = threadIdx.x; t < KC * kB / 2; t += 256) {
      const int q = t / (kB / 2), c = (t % (kB / 2)) * 2;
      const int o = ((q / 4) * 4 + c / 16) * 64 + (q % 4) * 16 + c % 16;
      *reinterpret_cast<double2*>(lds + o) = reinterpret_cast<const double2*>(Ui + (k0 + q) * kB)[c / 2];
      *reinterpret_cast<double2*>(lds + KC * kB + o) = reinterpret_cast<const double2*>(Rj + (k0 + q) * kB)[c / 2];
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < KC / 4; ++g) {
      const double a0 = -lds[(g * 4 + wr * 2) * 64 + lane];
      const double a1 = -lds[(g * 4 + wr * 2 + 1) * 64 + lane];
      const double b0 = lds[KC * kB + (g * 4 + wc * 2) * 64 + lane];
      const double b1 = lds[KC * kB + (g * 4 + wc * 2 + 1) * 64 + lane];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  if (I == nx && J == nx) {
    // hand the tile to the sweep layout through LDS (free after the loop)
    double* t = lds;  // [64][64]
    static_assert(2 * KC * kB >= kB * kB, "LDS tile");
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) t[(r0 + 16 * a + 4 * v) * kB + c0 + 16 * b] = acc[a][b][v];
    __syncthreads();
    const int j = threadIdx.x % kB, i0 = (threadIdx.x / kB) * 16;
    double r[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) r[u] = t[(i0 + u) * kB + j];
    __shared__ double col4[2][kB][4];
    sweep_tile(r, col4);
#pragma unroll
    for (int u = 0; u < 16; ++u) A[(ib + i0 + u) * ld + jb + j] = r[u];
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(ib + r0 + 16 * a + 4 * v) * ld + jb + c0 + 16 * b] = acc[a][b][v];
}

// Final pass over the upper triangle (i <= j): the swept matrix holds -A^-1
// in its upper tiles; write -a_ij - shift to (i, j) and (j, i) inside the
// valid n x n block, the identity in the padding.
__global__ void k_gj_finish(double* __restrict__ A, long ld, long nvalid, double shift) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ld * ld) return;
  const long i = t / ld, j = t % ld;
  if (i > j) return;
  if (i < nvalid && j < nvalid) {
    const double w = -A[i * ld + j] - shift;
    A[i * ld + j] = w;
    A[j * ld + i] = w;
  } else {
    A[i * ld + j] = (i == j) ? 1.0 : 0.0;
    A[j * ld + i] = (i == j) ? 1.0 : 0.0;
  }
}

// Dense fills from a coordinate list of unique entries.
__global__ void k_fill(double* __restrict__ A, long ld, long nvalid, double inner, long total) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const long i = t / ld, j = t % ld;
  A[t] = (i < nvalid && j < nvalid) ? inner : (i == j ? 1.0 : 0.0);
}
__global__ void k_scatter_add(double* __restrict__ A, long ld, const int* __restrict__ ij,
                              const double* __restrict__ v, long nnz) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnz) return;
  A[(long)ij[2 * t] * ld + ij[2 * t + 1]] += v[t];
}
// L + J on top of the fill (1/C in the valid block): L = Sigma^T Sigma has 3
// on the diagonal and -1 at the two cells of every edge (two cells share at
// most one edge, so every entry has one writer).
__global__ void k_build_lap(double* __restrict__ A, long ld, int C, int N, const int* __restrict__ edge_cell) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < C) A[(long)t * ld + t] += 3.0;
  if (t < N) {
    const long a = edge_cell[2 * t], b = edge_cell[2 * t + 1];
    A[a * ld + b] -= 1.0;
    A[b * ld + a] -= 1.0;
  }
}
// G_ll (P1 mass matrix) on a zero fill: the entry of edge (a, b) is the sum of
// A/12 over its two cells; the diagonal entry of a vertex sums A/6 over its
// cells, which is the sum of the edge entries over the edges at the vertex
// (each cell there has two of them).
__global__ void k_build_gll(double* __restrict__ A, long ld, int V, int N, const int* __restrict__ ve_ptr,
                            const int* __restrict__ ve_idx, const int* __restrict__ edge_vtx,
                            const int* __restrict__ edge_cell, const double* __restrict__ area) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < V) {
    double dsum = 0.0;
    for (int q = ve_ptr[t]; q < ve_ptr[t + 1]; ++q) {
      const int e = ve_idx[q];
      dsum += (area[edge_cell[2 * e]] + area[edge_cell[2 * e + 1]]) / 12.0;
    }
    A[(long)t * ld + t] = dsum;
  }
  if (t < N) {
    const long a = edge_vtx[2 * t], b = edge_vtx[2 * t + 1];
    const double w = (area[edge_cell[2 * t]] + area[edge_cell[2 * t + 1]]) / 12.0;
    A[a * ld + b] = w;
    A[b * ld + a] = w;
  }
}
inline unsigned blocks_for(long n, int per) { return unsigned((n + per - 1) / per); }

}  // namespace

rfcmp_status spd_inverse_many(const SpdInverseJob* jobs, int njobs) {
  int steps = 0;
  for (int q = 0; q < njobs; ++q) {
    const SpdInverseJob& j = jobs[q];
    if (j.n % kB != 0 || j.nvalid > j.n || j.nvalid < 0) {
      set_error("spd_inverse: n=%lld (valid %lld) not a multiple of %d", (long long)j.n, (long long)j.nvalid, kB);
      return RFCMP_E_ARG;
    }
    steps = std::max(steps, int(j.n / kB));
  }
  // the jobs' launches interleaved step by step, so that every stream has
  // work queued from the start; each job is timed on its own stream
  std::vector<std::unique_ptr<ProfScope>> prof(njobs);
  for (int q = 0; q < njobs; ++q) {
    prof[q] = std::make_unique<ProfScope>("spd_inverse", jobs[q].s);
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, jobs[q].s, jobs[q].A, (long)jobs[q].n, 0);
  }
  for (int K = 0; K < steps; ++K)
    for (int q = 0; q < njobs; ++q) {
      const SpdInverseJob& j = jobs[q];
      const int nb = int(j.n / kB);
      if (K >= nb || nb == 1) continue;
      const unsigned ntiles = unsigned((long)nb * (nb + 1) / 2);
      hipLaunchKernelGGL(k_gj_panels, dim3(nb, 4), dim3(256), 0, j.s, j.A, (long)j.n, K, j.ubuf, j.rbuf);
      hipLaunchKernelGGL(k_gj_update, dim3(ntiles), dim3(256), 0, j.s, j.A, (long)j.n, nb, K, j.ubuf, j.rbuf);
    }
  for (int q = 0; q < njobs; ++q) {
    const SpdInverseJob& j = jobs[q];
    const long total = (long)j.n * j.n;
    hipLaunchKernelGGL(k_gj_finish, dim3(unsigned((total + 255) / 256)), dim3(256), 0, j.s, j.A, (long)j.n,
                       (long)j.nvalid, j.shift);
    prof[q].reset();
  }
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

rfcmp_status spd_inverse(double* A, int64_t n, int64_t nvalid, double shift, double* ubuf, double* rbuf,
                         hipStream_t s) {
  const SpdInverseJob j{A, n, nvalid, shift, ubuf, rbuf, s};
  return spd_inverse_many(&j, 1);
}

// Build L^+, G_ll^-1 (and G_tp^-1) of a mesh on the device, in FP64.
//   L = Sigma^T Sigma: 3 on the diagonal, -1 for cells sharing an edge;
//   L^+ = (L + 1 1^T/C)^-1 - 1 1^T/C (identity of Sec. 3.2).
//   G_ll (P1 mass): A/6 on the diagonal, A/12 off it, per cell.
//   G_tp: closed form of Sec. 3 (mixed dual-hat / cell Gram matrix).
rfcmp_status mesh_projectors(rfcmp_mesh m, bool need_gtp, hipStream_t s) {
  if (need_gtp) build_cell_nb(m->h);
  const MeshHost& h = m->h;
  MeshDev& d = m->d;
  const int64_t C = h.C, V = h.V, N = h.N;

  // Two internal streams: L^+ on the first, G_ll^-1 (then G_tp^-1) on the
  // second, both after the work already enqueued on s (the mesh upload).
  // Scratch is kept with the mesh per stream, sized once, so that nothing
  // here is released (a release waits for the device) and the host goes on
  // while the inverses run.
  for (int q = 0; q < 2; ++q) {
    if (!d.proj_stream[q]) {
      RF_HIP(hipStreamCreateWithFlags(&d.proj_stream[q], hipStreamNonBlocking));
      RF_HIP(hipEventCreateWithFlags(&d.proj_done[q], hipEventDisableTiming));
    }
  }
  if (!d.proj_start) RF_HIP(hipEventCreateWithFlags(&d.proj_start, hipEventDisableTiming));
  RF_HIP(hipEventRecord(d.proj_start, s));
  {
    const int64_t nn[2] = {(int64_t)round_up(C, kB), (int64_t)round_up(need_gtp ? std::max(C, V) : V, kB)};
    for (int q = 0; q < 2; ++q) {
      RF_HIP(hipStreamWaitEvent(d.proj_stream[q], d.proj_start, 0));
      if (d.gj_u[q].bytes < sizeof(double) * nn[q] * kB) {
        RF_TRY(d.gj_u[q].alloc(sizeof(double) * nn[q] * kB));
        RF_TRY(d.gj_r[q].alloc(sizeof(double) * nn[q] * kB));
      }
    }
    const size_t nnz = need_gtp ? (size_t)h.cell_nb_ptr[C] : 0;  // G_tp's coordinate list
    if (nnz > 0 && d.scat_v.bytes < sizeof(double) * nnz) {
      RF_TRY(d.scat_ij.alloc(sizeof(int) * 2 * nnz));
      RF_TRY(d.scat_v.alloc(sizeof(double) * nnz));
    }
  }
  auto build = [&](int q, DevBuf& buf, int64_t nvalid, int64_t& ld, double inner,
                   const std::vector<int>& ij, const std::vector<double>& val,
                   bool sub_inner_after) -> rfcmp_status {
    hipStream_t ps = d.proj_stream[q];
    ld = (int64_t)round_up(nvalid, kB);
    RF_TRY(buf.alloc(sizeof(double) * ld * ld));
    const long total = ld * ld;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(total, 256)), dim3(256), 0, ps, buf.as<double>(), (long)ld,
                       (long)nvalid, inner, total);
    DevBuf& dij = d.scat_ij;
    DevBuf& dv = d.scat_v;
    // pageable sources: the copies are staged before these calls return
    RF_HIP(hipMemcpyAsync(dij.p, ij.data(), sizeof(int) * ij.size(), hipMemcpyHostToDevice, ps));
    RF_HIP(hipMemcpyAsync(dv.p, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, ps));
    hipLaunchKernelGGL(k_scatter_add, dim3(blocks_for((long)val.size(), 256)), dim3(256), 0, ps,
                       buf.as<double>(), (long)ld, dij.as<int>(), dv.as<double>(), (long)val.size());
    RF_HIP(hipGetLastError());
    return spd_inverse(buf.as<double>(), ld, nvalid, sub_inner_after ? inner : 0.0, d.gj_u[q].as<double>(),
                       d.gj_r[q].as<double>(), ps);
  };

  // L + J and G_ll are formed on the device from the uploaded mesh arrays
  auto fill = [&](int q, DevBuf& buf, int64_t nvalid, int64_t& ld, double inner) -> rfcmp_status {
    ld = (int64_t)round_up(nvalid, kB);
    RF_TRY(buf.alloc(sizeof(double) * ld * ld));
    const long total = ld * ld;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(total, 256)), dim3(256), 0, d.proj_stream[q], buf.as<double>(),
                       (long)ld, (long)nvalid, inner, total);
    return RFCMP_OK;
  };
  RF_TRY(fill(0, d.Lp, C, d.ldL, 1.0 / double(C)));
  hipLaunchKernelGGL(k_build_lap, dim3(blocks_for(std::max(C, N), 256)), dim3(256), 0, d.proj_stream[0],
                     d.Lp.as<double>(), (long)d.ldL, (int)C, (int)N, d.edge_cell.as<int>());
  RF_TRY(fill(1, d.Gll_inv, V, d.ldG, 0.0));
  hipLaunchKernelGGL(k_build_gll, dim3(blocks_for(std::max(V, N), 256)), dim3(256), 0, d.proj_stream[1],
                     d.Gll_inv.as<double>(), (long)d.ldG, (int)V, (int)N, d.ve_ptr.as<int>(), d.ve_idx.as<int>(),
                     d.edge_vtx.as<int>(), d.edge_cell.as<int>(), d.area.as<double>());
  RF_HIP(hipGetLastError());
  {
    const SpdInverseJob jobs[2] = {
        {d.Lp.as<double>(), d.ldL, C, 1.0 / double(C), d.gj_u[0].as<double>(), d.gj_r[0].as<double>(),
         d.proj_stream[0]},
        {d.Gll_inv.as<double>(), d.ldG, V, 0.0, d.gj_u[1].as<double>(), d.gj_r[1].as<double>(), d.proj_stream[1]}};
    RF_TRY(spd_inverse_many(jobs, 2));
  }
  if (need_gtp) {
    std::vector<int> ij;
    std::vector<double> v;
    for (int64_t m2 = 0; m2 < C; ++m2) {
      const int* tm = &h.tri[3 * m2];
      for (int q = h.cell_nb_ptr[m2]; q < h.cell_nb_ptr[m2 + 1]; ++q) {
        const int n2 = h.cell_nb_idx[q];
        const int* tn = &h.tri[3 * n2];
        double val;
        if (n2 == m2) {
          val = 4.5;
          for (int i = 0; i < 3; ++i) val += 1.0 / h.noc[tm[i]];
        } else {
          int shared[3], ns = 0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              if (tm[i] == tn[j]) shared[ns++] = tm[i];
          if (ns == 2)
            val = 0.5 + 1.0 / h.noc[shared[0]] + 1.0 / h.noc[shared[1]];
          else
            val = 1.0 / h.noc[shared[0]];
        }
        ij.push_back(int(m2));
        ij.push_back(n2);
        v.push_back(val * (2.0 / 18.0));
      }
    }
    RF_TRY(build(1, d.Gtp_inv, C, d.ldT, 0.0, ij, v, false));
    d.has_gtp = true;
  }
  for (int q = 0; q < 2; ++q) RF_HIP(hipEventRecord(d.proj_done[q], d.proj_stream[q]));
  d.proj_pending = true;
  return RFCMP_OK;
}

rfcmp_status wait_projectors(rfcmp_mesh m, hipStream_t s) {
  MeshDev& d = m->d;
  if (!d.proj_pending) return RFCMP_OK;
  for (int q = 0; q < 2; ++q) RF_HIP(hipStreamWaitEvent(s, d.proj_done[q], 0));
  return RFCMP_OK;
}

}  // namespace rfcmp
