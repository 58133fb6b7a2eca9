// The FP64 inverse used to build the dense projector matrices
// (L^+ = (Sigma^T Sigma)^+, G_ll^-1, G_tp^-1) of a mesh.
#include <cmath>

#include "internal.h"

namespace rfcmp {

namespace {

// ------------------------------------------------------------------------
// Blocked Gauss-Jordan inverse of an SPD matrix (no pivoting: every Schur
// complement of an SPD matrix is SPD).  Pivot block P (64 x 64):
//   D = A_PP^-1,  A_PO <- D A_PO,  A_OP <- -A_OP D,  A_OO <- A_OO - A_OP_old D A_PO_old,
//   A_PP <- D.
// After all pivot blocks the matrix holds A^-1 (the sweep operator).
constexpr int kB = 64;

// Unblocked sweep of the 64 x 64 pivot block.  Thread t keeps the 16-entry
// strip (rows 16 (t / 64) .. +16, column t % 64) in registers for all 64
// pivots; per pivot the owners publish the pivot column and row to LDS
// (double-buffered, one barrier per pivot) and every entry is updated:
//   a_ij -= a_ik a_kj / a_kk,  a_kj /= a_kk,  a_ik = -a_ik / a_kk,  a_kk = 1 / a_kk.
// Written branch-free: with m_j = a_kj / a_kk (j != k) or 1 / a_kk (j == k),
// row k becomes m_j and every other entry (j != k ? a_ij : 0) - a_ik m_j.
// The strip's 16 pivot-column values are read from LDS together, before the
// updates, so the reads overlap.
__global__ __launch_bounds__(256) void k_gj_diag(double* __restrict__ A, long ld, int K) {
  __shared__ double colk[2][kB], rowk[2][kB];
  const int j = threadIdx.x % kB;
  const int i0 = (threadIdx.x / kB) * 16;
  const long base = (long)K * kB;
  double r[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) r[u] = A[(base + i0 + u) * ld + base + j];
  for (int k = 0; k < kB; ++k) {
    const int bsel = k & 1;
    if (j == k) {
#pragma unroll
      for (int u = 0; u < 16; ++u) colk[bsel][i0 + u] = r[u];
    }
    if (k >= i0 && k < i0 + 16) {
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) v = (i0 + u == k) ? r[u] : v;
      rowk[bsel][j] = v;
    }
    __syncthreads();
    double ck[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) ck[u] = colk[bsel][i0 + u];
    const double d = 1.0 / rowk[bsel][k];
    const bool pj = (j == k);
    const double m = pj ? d : rowk[bsel][j] * d;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double keep = pj ? 0.0 : r[u];
      const double nv = fma(-ck[u], m, keep);
      r[u] = (i0 + u == k) ? m : nv;
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) A[(base + i0 + u) * ld + base + j] = r[u];
}

// Column panel: Ccol = A_OP (old), A_OP <- -A_OP D.  Row panel: A_PO <- D A_PO.
// blockIdx.x = block index b (skip b == K); blockIdx.y = 0 column panel, 1 row panel.
// D and the old panel block are staged in LDS (the product overwrites the
// panel in place); each thread computes a 4 x 4 output tile.
__global__ __launch_bounds__(256) void k_gj_panels(double* __restrict__ A, long ld, int K,
                                                   double* __restrict__ Ccol) {
  const int b = blockIdx.x;
  if (b == K) return;
  __shared__ double D[kB][kB];
  __shared__ double S[kB][kB];
  const long pb = (long)K * kB, ob = (long)b * kB;
  const bool col = blockIdx.y == 0;
  for (int t = threadIdx.x; t < kB * kB; t += 256) {
    const int i = t / kB, j = t % kB;
    D[i][j] = A[(pb + i) * ld + pb + j];
    if (col) {
      const double v = A[(ob + i) * ld + pb + j];  // row ob+i, pivot column j
      S[i][j] = v;
      Ccol[(ob + i) * kB + j] = v;
    } else {
      S[i][j] = A[(pb + i) * ld + ob + j];  // pivot row i, column ob+j
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  // col: out = S D (rows of S times D); row: out = D S
  const double(*L)[kB] = col ? S : D;
  const double(*Rm)[kB] = col ? D : S;
#pragma unroll 8
  for (int q = 0; q < kB; ++q) {
    double lv[4], rv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) lv[u] = L[ty * 4 + u][q];
#pragma unroll
    for (int v = 0; v < 4; ++v) rv[v] = Rm[q][tx + 16 * v];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += lv[u] * rv[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ty * 4 + u, j = tx + 16 * v;
      if (col)
        A[(ob + i) * ld + pb + j] = -acc[u][v];
      else
        A[(pb + i) * ld + ob + j] = acc[u][v];
    }
}

// A_IJ -= Ccol_I R_J for I, J != K, with R = the updated pivot row panel.
// 64 x 64 output tile per block, 4 x 4 per thread, k-chunks of 32 in LDS.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, long ld, int K,
                                                   const double* __restrict__ Ccol) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I == K || J == K) return;
  constexpr int KC = 32;
  __shared__ double a[kB][KC + 1];
  __shared__ double r[KC][kB + 1];
  const long ib = (long)I * kB, jb = (long)J * kB, pb = (long)K * kB;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < kB; k0 += KC) {
    for (int t = threadIdx.x; t < kB * KC; t += 256) {
      const int i = t / KC, q = t % KC;
      a[i][q] = Ccol[(ib + i) * kB + k0 + q];
    }
    for (int t = threadIdx.x; t < KC * kB; t += 256) {
      const int q = t / kB, j = t % kB;
      r[q][j] = A[(pb + k0 + q) * ld + jb + j];
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < KC; ++q) {
      double av[4], rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = a[ty * 4 + u][q];
#pragma unroll
      for (int u = 0; u < 4; ++u) rv[u] = r[q][tx + 16 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * rv[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) A[(ib + ty * 4 + u) * ld + jb + tx + 16 * v] -= acc[u][v];
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
__global__ void k_sub_const(double* __restrict__ A, long ld, long nvalid, double c) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nvalid * nvalid) return;
  const long i = t / nvalid, j = t % nvalid;
  A[i * ld + j] -= c;
}

inline unsigned blocks_for(long n, int per) { return unsigned((n + per - 1) / per); }

}  // namespace

rfcmp_status spd_inverse(double* A, int64_t n, hipStream_t s) {
  if (n % kB != 0) {
    set_error("spd_inverse: n=%lld not a multiple of %d", (long long)n, kB);
    return RFCMP_E_ARG;
  }
  const int nb = int(n / kB);
  ProfScope prof("spd_inverse", s);
  DevBuf ccol;
  RF_TRY(ccol.alloc(sizeof(double) * n * kB));
  for (int K = 0; K < nb; ++K) {
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, s, A, (long)n, K);
    if (nb > 1) {
      hipLaunchKernelGGL(k_gj_panels, dim3(nb, 2), dim3(256), 0, s, A, (long)n, K, ccol.as<double>());
      hipLaunchKernelGGL(k_gj_update, dim3(nb, nb), dim3(256), 0, s, A, (long)n, K, ccol.as<double>());
    }
  }
  RF_HIP(hipGetLastError());
  // the scratch panel is released when ccol goes out of scope: wait first
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

// Build L^+, G_ll^-1 (and G_tp^-1) of a mesh on the device, in FP64.
//   L = Sigma^T Sigma: 3 on the diagonal, -1 for cells sharing an edge;
//   L^+ = (L + 1 1^T/C)^-1 - 1 1^T/C (identity of Sec. 3.2).
//   G_ll (P1 mass): A/6 on the diagonal, A/12 off it, per cell.
//   G_tp: closed form of Sec. 3 (mixed dual-hat / cell Gram matrix).
rfcmp_status mesh_projectors(rfcmp_mesh m, bool need_gtp, hipStream_t s) {
  const MeshHost& h = m->h;
  MeshDev& d = m->d;
  const int64_t C = h.C, V = h.V, N = h.N;

  auto build = [&](DevBuf& buf, int64_t nvalid, int64_t& ld, double inner,
                   const std::vector<int>& ij, const std::vector<double>& val,
                   bool sub_inner_after) -> rfcmp_status {
    ld = (int64_t)round_up(nvalid, kB);
    RF_TRY(buf.alloc(sizeof(double) * ld * ld));
    const long total = ld * ld;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(total, 256)), dim3(256), 0, s, buf.as<double>(), (long)ld,
                       (long)nvalid, inner, total);
    DevBuf dij, dv;
    RF_TRY(dij.alloc(sizeof(int) * ij.size()));
    RF_TRY(dv.alloc(sizeof(double) * val.size()));
    RF_HIP(hipMemcpyAsync(dij.p, ij.data(), sizeof(int) * ij.size(), hipMemcpyHostToDevice, s));
    RF_HIP(hipMemcpyAsync(dv.p, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scatter_add, dim3(blocks_for((long)val.size(), 256)), dim3(256), 0, s,
                       buf.as<double>(), (long)ld, dij.as<int>(), dv.as<double>(), (long)val.size());
    RF_HIP(hipGetLastError());
    RF_TRY(spd_inverse(buf.as<double>(), ld, s));  // synchronises before dij/dv are freed
    if (sub_inner_after) {
      hipLaunchKernelGGL(k_sub_const, dim3(blocks_for(nvalid * nvalid, 256)), dim3(256), 0, s,
                         buf.as<double>(), (long)ld, (long)nvalid, inner);
      RF_HIP(hipGetLastError());
    }
    return RFCMP_OK;
  };

  // L + J
  {
    std::vector<int> ij;
    std::vector<double> v;
    ij.reserve(2 * (C + 2 * N));
    for (int64_t c = 0; c < C; ++c) {
      ij.push_back(int(c));
      ij.push_back(int(c));
      v.push_back(3.0);
    }
    for (int64_t n = 0; n < N; ++n) {
      const int a = h.edge_cell[2 * n], b = h.edge_cell[2 * n + 1];
      ij.push_back(a); ij.push_back(b); v.push_back(-1.0);
      ij.push_back(b); ij.push_back(a); v.push_back(-1.0);
    }
    RF_TRY(build(d.Lp, C, d.ldL, 1.0 / double(C), ij, v, true));
  }
  // G_ll: the diagonal sums A/6 over the cells at a vertex; the entry of the
  // edge (a, b) sums A/12 over its two cells.  Keys are unique, as the
  // scatter needs.
  {
    std::vector<double> diag(V, 0.0);
    for (int64_t c = 0; c < C; ++c)
      for (int i = 0; i < 3; ++i) diag[h.tri[3 * c + i]] += h.area[c] / 6.0;
    std::vector<int> ij;
    std::vector<double> v;
    ij.reserve(2 * (V + 2 * N));
    v.reserve(V + 2 * N);
    for (int64_t a = 0; a < V; ++a) {
      ij.push_back(int(a));
      ij.push_back(int(a));
      v.push_back(diag[a]);
    }
    for (int64_t n = 0; n < N; ++n) {
      const int a = h.edge_vtx[2 * n], b = h.edge_vtx[2 * n + 1];
      const double w = (h.area[h.edge_cell[2 * n]] + h.area[h.edge_cell[2 * n + 1]]) / 12.0;
      ij.push_back(a); ij.push_back(b); v.push_back(w);
      ij.push_back(b); ij.push_back(a); v.push_back(w);
    }
    RF_TRY(build(d.Gll_inv, V, d.ldG, 0.0, ij, v, false));
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
    RF_TRY(build(d.Gtp_inv, C, d.ldT, 0.0, ij, v, false));
    d.has_gtp = true;
  }
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

}  // namespace rfcmp
