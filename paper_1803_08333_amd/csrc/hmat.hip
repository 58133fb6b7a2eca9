// Compressed EFIE blocks on the device (see hmat.h): the tree's upload,
// adaptive cross approximation of the low-rank blocks, the compressed product
// and the dense write-out.
//
// ACA (one workgroup per block, partial pivoting): the residual of pivot row
// i is formed from the block's entries less the terms so far, its largest
// entry (first on ties) is the column pivot j, v = row / row[j], the residual
// column j is u, and the next pivot row is the largest entry of u among the
// rows not yet taken.  The Frobenius norm of the approximation S_k is updated
// exactly, |S_k|^2 = |S_k-1|^2 + 2 Re sum_l<k (u_l^H u_k)(v_l^H v_k) +
// |u_k|^2 |v_k|^2, and the iteration stops when |u_k| |v_k| <= tol |S_k|.
// Entries are formed on the fly in FP32 by the far-pair rule (an admissible
// block holds no near cell pair): a T_A entry sums the four cell pairs of its
// two edges, (B++ + B--) + (B+- + B-+), a V entry is I_0 of its cell pair.
// Factors are complex64; each thread owns the rows (columns) i = tid mod 256
// of its block's factors, so the only values it reads from other threads are
// the pivots, staged in LDS after a barrier.
//
// Product y = M x (M = T_A or V, x [nr][n] complex128, FP64 accumulation):
// the input in the permuted order; per low-rank block z = V^T x_cols and
// w = U^T x_rows (k_hm_proj); per tile of output rows the sum, in a fixed
// order, of its dense blocks (and the transposes of those it is the column
// of), U z of the low-rank blocks it is a row of and V w of those it is a
// column of (k_hm_tile), written back in the mesh's numbering.
#include <algorithm>
#include <climits>
#include <cmath>
#include <numeric>

#include "farpair.h"
#include "hmat.h"
#include "internal.h"

rfcmp_mesh_s::rfcmp_mesh_s() = default;
rfcmp_mesh_s::~rfcmp_mesh_s() = default;

namespace rfcmp {
namespace {

constexpr int kAcaThreads = 256;
constexpr int kAcaWaves = kAcaThreads / 64;

struct AcaArgs {
  const int* perm;        // position -> edge (T_A) or cell (V)
  const int* edge_slot;   // [N][2]: 3 c + local index of each edge in c+ and c-
  const double* cen;
  const float4* qoff;
  const float4* fvoff;
  const float* sgn;
  RuleArgs rule;
  float kk;
  float tol;
  int kmax;
  const HmLr* blk;
  const long* uoff;       // pool offsets (complex64 entries) of U and V
  const long* voff;
  const long* toff;       // offsets of the taken-row flags
  float2* pool;
  unsigned char* taken;
  int* rank;
  int* flag;              // 1: stopped at kmax above the tolerance
};

__device__ float2 ta_entry(const AcaArgs& a, int m, int n) {
  float2 b00, b01, b10, b11;
#pragma unroll 1
  for (int pq = 0; pq < 4; ++pq) {
    const int p = pq >> 1, q = pq & 1;
    const int sa = a.edge_slot[2 * m + p], sb = a.edge_slot[2 * n + q];
    const int ca = sa / 3, la = sa - 3 * ca, cb = sb / 3, lb = sb - 3 * cb;
    Moments M;
    far_moments(a.qoff + (long)ca * kQ, a.qoff + (long)cb * kQ, (float)(a.cen[3 * ca] - a.cen[3 * cb]),
                    (float)(a.cen[3 * ca + 1] - a.cen[3 * cb + 1]), (float)(a.cen[3 * ca + 2] - a.cen[3 * cb + 2]),
                    a.rule, a.kk, M);
    const float2 v = b_entry(M, a.fvoff[3 * ca + la], a.fvoff[3 * cb + lb], a.sgn[3 * ca + la], a.sgn[3 * cb + lb]);
    if (pq == 0)
      b00 = v;
    else if (pq == 1)
      b01 = v;
    else if (pq == 2)
      b10 = v;
    else
      b11 = v;
  }
  return make_float2((b00.x + b11.x) + (b01.x + b10.x), (b00.y + b11.y) + (b01.y + b10.y));
}

__device__ float2 v_entry(const AcaArgs& a, int c, int cp) {
  return far_i0(a.qoff + (long)c * kQ, a.qoff + (long)cp * kQ, (float)(a.cen[3 * c] - a.cen[3 * cp]),
                    (float)(a.cen[3 * c + 1] - a.cen[3 * cp + 1]), (float)(a.cen[3 * c + 2] - a.cen[3 * cp + 2]),
                    a.rule, a.kk);
}

struct AcaLds {
  float v[kAcaWaves];
  int i[kAcaWaves];
  double d[kAcaWaves][2];
  float c[kAcaWaves][32];
};

// Largest value, smallest index on ties, over the workgroup; every thread
// receives it.
__device__ inline void block_argmax(float& v, int& idx, AcaLds& L) {
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    L.v[w] = v;
    L.i[w] = idx;
  }
  __syncthreads();
  v = L.v[0];
  idx = L.i[0];
  for (int q = 1; q < kAcaWaves; ++q)
    if (L.v[q] > v || (L.v[q] == v && L.i[q] < idx)) {
      v = L.v[q];
      idx = L.i[q];
    }
  __syncthreads();
}

// Sums of two doubles over the workgroup in a fixed order (lane 0 of each
// wave, then the waves in order).
__device__ inline void block_sum2(double& x, double& y, AcaLds& L) {
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_xor(x, o);
    y += __shfl_xor(y, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    L.d[w][0] = x;
    L.d[w][1] = y;
  }
  __syncthreads();
  x = L.d[0][0];
  y = L.d[0][1];
  for (int q = 1; q < kAcaWaves; ++q) {
    x += L.d[q][0];
    y += L.d[q][1];
  }
  __syncthreads();
}

__device__ inline void block_sum32(float (&v)[32], AcaLds& L) {
#pragma unroll
  for (int q = 0; q < 32; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 32; ++q) L.c[w][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    float s = L.c[0][q];
    for (int u = 1; u < kAcaWaves; ++u) s += L.c[u][q];
    v[q] = s;
  }
  __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(kAcaThreads) void k_aca(const AcaArgs a, int b0) {
  const int b = b0 + blockIdx.x;
  const HmLr B = a.blk[b];
  const int m = B.m, n = B.n;
  float2* U = a.pool + a.uoff[b];
  float2* V = a.pool + a.voff[b];
  unsigned char* taken = a.taken + a.toff[b];
  const int kcap = min(a.kmax, min(m, n));
  const int tid = threadIdx.x;
  __shared__ float2 sU[kHmKmax], sV[kHmKmax + 1];
  __shared__ AcaLds L;
  for (int i = tid; i < m; i += kAcaThreads) taken[i] = 0;
  __syncthreads();
  auto entry = [&](int pi, int pj) -> float2 {
    const int x = a.perm[B.r0 + pi], y = a.perm[B.c0 + pj];
    return KIND == 0 ? ta_entry(a, x, y) : v_entry(a, x, y);
  };
  double S2 = 0.0;
  int k = 0, i = 0, tries = 0;
  bool conv = false;
  while (k < kcap) {
    for (int l = tid; l < k; l += kAcaThreads) sU[l] = U[(long)l * m + i];
    __syncthreads();
    // residual of row i into V[k]
    float2* Vk = V + (long)k * n;
    float best = -1.f;
    int bj = INT_MAX;
    for (int j = tid; j < n; j += kAcaThreads) {
      float2 e = entry(i, j);
      for (int l = 0; l < k; ++l) {
        const float2 v = V[(long)l * n + j], u = sU[l];
        e.x -= u.x * v.x - u.y * v.y;
        e.y -= u.x * v.y + u.y * v.x;
      }
      Vk[j] = e;
      const float mg = e.x * e.x + e.y * e.y;
      if (mg > best) {
        best = mg;
        bj = j;
      }
    }
    block_argmax(best, bj, L);
    if (tid == 0) taken[i] = 1;
    __syncthreads();
    if (!(best > 0.f)) {
      // row i is represented already: the first row not yet taken
      int cand = INT_MAX;
      for (int ii = tid; ii < m; ii += kAcaThreads)
        if (!taken[ii]) {
          cand = ii;
          break;
        }
      float cv = cand < INT_MAX ? 0.f : -1.f;
      block_argmax(cv, cand, L);
      if (cand == INT_MAX || ++tries > m) break;
      i = cand;
      continue;
    }
    const float2 piv = Vk[bj];
    const float dd = piv.x * piv.x + piv.y * piv.y;
    const float2 inv = make_float2(piv.x / dd, -piv.y / dd);
    double nv = 0.0, nu = 0.0;
    for (int j = tid; j < n; j += kAcaThreads) {
      const float2 e = Vk[j];
      const float2 v = make_float2(e.x * inv.x - e.y * inv.y, e.x * inv.y + e.y * inv.x);
      Vk[j] = v;
      nv += (double)v.x * v.x + (double)v.y * v.y;
    }
    __syncthreads();
    for (int l = tid; l <= k; l += kAcaThreads) sV[l] = V[(long)l * n + bj];
    __syncthreads();
    // residual of column bj into U[k]
    float2* Uk = U + (long)k * m;
    float bu = -1.f;
    int bi = INT_MAX;
    for (int ii = tid; ii < m; ii += kAcaThreads) {
      float2 e = entry(ii, bj);
      for (int l = 0; l < k; ++l) {
        const float2 u = U[(long)l * m + ii], v = sV[l];
        e.x -= u.x * v.x - u.y * v.y;
        e.y -= u.x * v.y + u.y * v.x;
      }
      Uk[ii] = e;
      nu += (double)e.x * e.x + (double)e.y * e.y;
      if (!taken[ii]) {
        const float mg = e.x * e.x + e.y * e.y;
        if (mg > bu) {
          bu = mg;
          bi = ii;
        }
      }
    }
    // cross terms with the earlier terms, eight at a time
    double cr = 0.0;
    for (int l0 = 0; l0 < k; l0 += 8) {
      float pp[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) pp[q] = 0.f;
      for (int ii = tid; ii < m; ii += kAcaThreads) {
        const float2 u = Uk[ii];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (l0 + q < k) {
            const float2 w = U[(long)(l0 + q) * m + ii];
            pp[2 * q] += w.x * u.x + w.y * u.y;
            pp[2 * q + 1] += w.x * u.y - w.y * u.x;
          }
      }
      for (int j = tid; j < n; j += kAcaThreads) {
        const float2 v = Vk[j];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (l0 + q < k) {
            const float2 w = V[(long)(l0 + q) * n + j];
            pp[16 + 2 * q] += w.x * v.x + w.y * v.y;
            pp[16 + 2 * q + 1] += w.x * v.y - w.y * v.x;
          }
      }
      block_sum32(pp, L);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        cr += (double)pp[2 * q] * pp[16 + 2 * q] - (double)pp[2 * q + 1] * pp[16 + 2 * q + 1];
    }
    block_sum2(nu, nv, L);
    S2 += 2.0 * cr + nu * nv;
    ++k;
    if (nu * nv <= (double)a.tol * (double)a.tol * S2) {
      conv = true;
      break;
    }
    block_argmax(bu, bi, L);
    if (bi == INT_MAX) {  // every row taken: the block is exact
      conv = true;
      break;
    }
    i = bi;
  }
  if (k >= min(m, n)) conv = true;
  if (tid == 0) {
    a.rank[b] = k;
    a.flag[b] = conv ? 0 : 1;
  }
}

// The first rank[b] columns of each block's factors, from the pool to their
// own storage.
__global__ __launch_bounds__(256) void k_aca_compact(int b0, const HmLr* blk, const int* rank, const long* uoff,
                                                     const long* voff, const float2* pool, float2* const* ud,
                                                     float2* const* vd) {
  const int b = b0 + blockIdx.x;
  const long k = rank[b];
  const long nu = k * blk[b].m, nv = k * blk[b].n;
  const float2* su = pool + uoff[b];
  const float2* sv = pool + voff[b];
  float2* du = ud[b];
  float2* dv = vd[b];
  for (long e = threadIdx.x; e < nu; e += 256) du[e] = su[e];
  for (long e = threadIdx.x; e < nv; e += 256) dv[e] = sv[e];
}

// xp[r][p] = x[r][perm[p]]
__global__ void k_hm_gather(int n, int nr, const int* __restrict__ perm, const double2* __restrict__ x,
                            double2* __restrict__ xp) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * nr) return;
  const int r = (int)(e / n), p = (int)(e % n);
  xp[e] = x[(long)r * n + perm[p]];
}

// z = V^T x_cols and w = U^T x_rows of every low-rank block (conj: of the
// conjugated factors), nr <= R <= kHmR right-hand sides: a small GEMM per
// block (k x len times len x nr) over chunks of rows, the factor chunk
// (k x rows <= 4096 entries) and the input chunk (rows x R <= 1024) staged in
// LDS so that each is read from memory once.  The k R outputs are spread over
// the workgroup: with fewer than 256, G = 256 / (k R) threads (at most 8)
// share an output, thread group g taking the rows jj = g, g + G, ... of each
// chunk in two alternating sums, and the G partial sums are added in order at
// the end; with more, thread t takes outputs t, t + 256, ...  Every sum runs
// in a fixed order.
constexpr int kProjFactor = 4096;   // complex64 entries of a staged factor chunk
constexpr int kProjInput = 1024;    // complex128 entries of a staged input chunk
template <int R>
__global__ __launch_bounds__(256) void k_hm_proj(const HmLr* __restrict__ blk, const int* __restrict__ rank,
                                                 float2* const* __restrict__ Up, float2* const* __restrict__ Vp,
                                                 const long* __restrict__ zoff, const double2* __restrict__ xp,
                                                 int n, int nr, int conj, double2* __restrict__ zw) {
  __shared__ float2 sm[kProjFactor];
  __shared__ double2 sx[kProjInput];
  const int b = blockIdx.x;
  const int k = rank[b];
  if (k == 0) return;
  const HmLr B = blk[b];
  const int tid = threadIdx.x;
  const float sgn = conj ? -1.f : 1.f;
  constexpr int kOut = (kHmKmax * R + 255) / 256;  // outputs per thread at most
  const int nout = k * R;
  const int G = nout >= 256 ? 1 : min(8, 256 / nout);
  const int g = tid / (nout < 256 ? nout : 256);   // row group (G > 1 only)
  const int ob = tid % (nout < 256 ? nout : 256);  // first output of this thread
  const bool act = g < G;
  // rows per chunk: a multiple of 32, at most 256
  const int cr = max(32, min(256, min(kProjFactor / k, kProjInput / R)) / 32 * 32);
  double2* z = zw + zoff[b];
  for (int part = 0; part < 2; ++part) {     // 0: z from V and the columns, 1: w from U and the rows
    const float2* M = part == 0 ? Vp[b] : Up[b];
    const int len = part == 0 ? B.n : B.m, off = part == 0 ? B.c0 : B.r0;
    double2* out = z + (long)part * k * kHmR;
    double ar[kOut], ai[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) ar[q] = ai[q] = 0.0;
    for (int j0 = 0; j0 < len; j0 += cr) {
      const int nj = min(cr, len - j0);
      for (int e = tid; e < k * cr; e += 256) {
        const int l = e / cr, jj = e % cr;
        float2 v = jj < nj ? M[(long)l * len + j0 + jj] : make_float2(0.f, 0.f);
        v.y *= sgn;
        sm[e] = v;
      }
      for (int e = tid; e < cr * R; e += 256) {
        const int jj = e / R, r = e % R;
        sx[e] = (jj < nj && r < nr) ? xp[(long)r * n + off + j0 + jj] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int q = 0; q < kOut; ++q) {
          const int o = ob + 256 * q;
          if (o < nout) {
            const int l = o / R, r = o % R;
            const float2* mrow = sm + l * cr;
            double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
            int jj = g;
            for (; jj + G < nj; jj += 2 * G) {
              const float2 m0 = mrow[jj], m1 = mrow[jj + G];
              const double2 x0 = sx[jj * R + r], x1 = sx[(jj + G) * R + r];
              s0r += (double)m0.x * x0.x - (double)m0.y * x0.y;
              s0i += (double)m0.x * x0.y + (double)m0.y * x0.x;
              s1r += (double)m1.x * x1.x - (double)m1.y * x1.y;
              s1i += (double)m1.x * x1.y + (double)m1.y * x1.x;
            }
            if (jj < nj) {
              const float2 m0 = mrow[jj];
              const double2 x0 = sx[jj * R + r];
              s0r += (double)m0.x * x0.x - (double)m0.y * x0.y;
              s0i += (double)m0.x * x0.y + (double)m0.y * x0.x;
            }
            ar[q] += s0r + s1r;
            ai[q] += s0i + s1i;
          }
        }
      }
      __syncthreads();
    }
    if (G > 1) {  // the row groups' partial sums, added in order of g
      double2* red = reinterpret_cast<double2*>(sm);  // [G][nout], 256 entries at most
      static_assert(sizeof(sm) >= 256 * sizeof(double2), "partials fit the staging buffer");
      if (act) red[g * nout + ob] = make_double2(ar[0], ai[0]);
      __syncthreads();
      if (g == 0) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < G; ++q) {
          sr += red[q * nout + ob].x;
          si += red[q * nout + ob].y;
        }
        ar[0] = sr;
        ai[0] = si;
      }
      __syncthreads();
    }
    if (g == 0) {
#pragma unroll
      for (int q = 0; q < kOut; ++q) {
        const int o = ob + 256 * q;
        if (o < nout && o % R < nr) out[(o / R) * kHmR + o % R] = make_double2(ar[q], ai[q]);
      }
    }
  }
}

struct TileArgs {
  int n;                       // N or C
  const int* perm;             // position -> mesh index
  const int* row0;             // KIND 1: cell_start (rows of tile T: [row0[T], row0[T + 1]))
  const int* list_ptr;
  const HmEnt* ent;            // the list entries, resolved
  const int2* dense_ij;
  const float2* D;             // dense blocks
  const long* doff;            // KIND 1: offsets of the dense blocks (KIND 0: b * 4096)
  const HmLr* blk;
  const int* rank;
  float2* const* Up;
  float2* const* Vp;
  const long* zoff;
  const double2* zw;
  const double2* xp;
  int nr, conj;
  double2* y;
};

template <int KIND>
__device__ inline int tile_row0(const TileArgs& a, int T) {
  return KIND == 0 ? T * kEdgeTile : a.row0[T];
}
template <int KIND>
__device__ inline int tile_rows(const TileArgs& a, int T) {
  return KIND == 0 ? min(kEdgeTile, a.n - T * kEdgeTile) : a.row0[T + 1] - a.row0[T];
}

// One workgroup per tile of output rows; thread (row i, quarter g) keeps
// the sums of its row for every right-hand side.  Each block of the tile's
// list is staged in LDS with coalesced loads (all threads, many loads in
// flight), then used from there: a dense block (64 x 64, rows padded) with
// the input of its partner tile, or up to 32 factor columns of the rows of
// consecutive low-rank blocks with their projections (a block of rank above
// 32 in chunks of 32).  A dense V block larger than 64 x 64 (a tile homing
// more than 64 cells) is read directly instead.
constexpr int kTileLd = kEdgeTile + 1;  // padded row of a staged dense block
template <int KIND, int R>
__global__ __launch_bounds__(256) void k_hm_tile(const TileArgs a) {
  __shared__ float2 smat[kEdgeTile * kTileLd];   // dense block [r][c], or factor rows [l][i] (32 x 64)
  __shared__ double2 sx[kEdgeTile][kHmR];         // partner input [c][r], or projections [l][r]
  __shared__ int s_nent, s_cols, s_colent[32], s_coll[32], s_len[32], s_o[32];
  __shared__ const float2* s_F[32];
  __shared__ const double2* s_zb[32];
  const int T = blockIdx.x;
  const int tid = threadIdx.x;
  const int p0 = tile_row0<KIND>(a, T), nrow = tile_rows<KIND>(a, T);
  const int lane = tid & 63, g = tid >> 6;
  const float sgn = a.conj ? -1.f : 1.f;
  const int e0 = a.list_ptr[T], e1 = a.list_ptr[T + 1];
  for (int base = 0; base < nrow; base += 64) {
    const int i = base + lane;
    const bool valid = i < nrow;
    const int nb = min(64, nrow - base);   // rows of this pass
    double ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0.0;
    auto fma_x = [&](float2 mv, const double2* x) {
      const double mx = mv.x, my = sgn * mv.y;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 v = x[r];
        ar[r] += mx * v.x - my * v.y;
        ai[r] += mx * v.y + my * v.x;
      }
    };
    int e = e0;
    while (e < e1) {
      __syncthreads();   // every wave is done with the previous batch's descriptors
      // wave 0: the next entries that form a batch of low-rank blocks with at
      // most 32 factor columns in all (their descriptors into LDS)
      if (g == 0) {
        const int ej = e + lane;
        HmEnt E{nullptr, 0, 0, 0, 0, 0};
        if (ej < e1) E = a.ent[ej];
        const int cd = E.code;
        const bool lr = ej < e1 && (cd & 3) >= 2;
        const int kj = lr ? E.k : 0;
        int cum = kj;
        for (int o = 1; o < 64; o <<= 1) {
          const int t = __shfl_up(cum, o);
          if (lane >= o) cum += t;
        }
        const unsigned long long nonlr = __ballot(!lr);
        const int first_non = nonlr ? (int)__builtin_ctzll(nonlr) : 64;
        const bool ok = lane < first_non && lane < 32 && cum <= 32;
        const int nent = __popcll(__ballot(ok));
        const int cols = __shfl(cum, nent > 0 ? nent - 1 : 0);
        if (lane == 0) {
          s_nent = nent;
          s_cols = nent > 0 ? cols : 0;
        }
        if (ok) {
          s_F[lane] = E.F;
          s_len[lane] = E.len;
          s_o[lane] = p0 + base - E.start;
          s_zb[lane] = a.zw + E.zb;
          for (int c = cum - kj; c < cum; ++c) {
            s_colent[c] = lane;
            s_coll[c] = c - (cum - kj);
          }
        }
      }
      __syncthreads();
      const int nbatch = s_nent;
      if (nbatch > 0) {
        const int cols = s_cols;
        for (int q = tid; q < 32 * 64; q += 256) {
          const int c = q / 64, ii = q % 64;
          float2 v = make_float2(0.f, 0.f);
          if (c < cols && ii < nb) {
            const int j = s_colent[c];
            v = s_F[j][(long)s_coll[c] * s_len[j] + s_o[j] + ii];
          }
          smat[c * 64 + ii] = v;
        }
        {
          const int c = tid / kHmR, r = tid % kHmR;   // 32 x 8 = 256 entries
          sx[c][r] = (c < cols && r < a.nr) ? s_zb[s_colent[c]][(long)s_coll[c] * kHmR + r] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (valid)
          for (int c = g; c < cols; c += 4) fma_x(smat[c * 64 + lane], sx[c]);
        e += nbatch;
        continue;
      }
      const HmEnt E = a.ent[e];
      const int kind = E.code & 3, bi = E.code >> 2;
      ++e;
      if (kind < 2) {
        const int I = a.dense_ij[bi].x, J = a.dense_ij[bi].y;
        int qI, nI, qJ, nJ;
        const float2* D;
        if (KIND == 0) {
          qI = I * kEdgeTile;
          qJ = J * kEdgeTile;
          nI = min(kEdgeTile, a.n - qI);
          nJ = min(kEdgeTile, a.n - qJ);
          D = a.D + (long)bi * kEdgeTile * kEdgeTile;
        } else {
          qI = a.row0[I];
          nI = a.row0[I + 1] - qI;
          qJ = a.row0[J];
          nJ = a.row0[J + 1] - qJ;
          D = a.D + a.doff[bi];
        }
        const int ld = KIND == 0 ? kEdgeTile : nJ;
        // the partner's rows: columns of D (kind 0) or its rows (kind 1)
        const int qp = kind == 0 ? qJ : qI, np = kind == 0 ? nJ : nI;
        if (nI > 64 || nJ > 64) {  // direct reads (only a V block of a tile homing > 64 cells)
          if (valid) {
            if (kind == 0) {
              for (int c = g; c < nJ; c += 4) {
                double2 xv[R];
#pragma unroll
                for (int r = 0; r < R; ++r)
                  xv[r] = r < a.nr ? a.xp[(long)r * a.n + qJ + c] : make_double2(0.0, 0.0);
                fma_x(D[(long)i * ld + c], xv);
              }
            } else {
              for (int rr = g; rr < nI; rr += 4) {
                double2 xv[R];
#pragma unroll
                for (int r = 0; r < R; ++r)
                  xv[r] = r < a.nr ? a.xp[(long)r * a.n + qI + rr] : make_double2(0.0, 0.0);
                fma_x(D[(long)rr * ld + i], xv);
              }
            }
          }
          continue;
        }
        for (int q = tid; q < kEdgeTile * kEdgeTile; q += 256) {
          const int r = q / kEdgeTile, c = q % kEdgeTile;
          smat[r * kTileLd + c] = (r < nI && c < nJ) ? D[(long)r * ld + c] : make_float2(0.f, 0.f);
        }
        for (int q = tid; q < kEdgeTile * kHmR; q += 256) {
          const int c = q / kHmR, r = q % kHmR;
          sx[c][r] = (c < np && r < a.nr) ? a.xp[(long)r * a.n + qp + c] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (valid) {
          if (kind == 0) {
            for (int c = 16 * g; c < 16 * g + 16; ++c) fma_x(smat[(i - base) * kTileLd + c], sx[c]);
          } else {
            for (int rr = 16 * g; rr < 16 * g + 16; ++rr) fma_x(smat[rr * kTileLd + (i - base)], sx[rr]);
          }
        }
        __syncthreads();
      } else {
        const int k = E.k;
        const double2* zb = a.zw + E.zb;
        const float2* F = E.F;
        const int len = E.len;
        const int o = p0 + base - E.start;   // first row of this pass in the factor
        for (int l0 = 0; l0 < k; l0 += 32) {
          const int nl = min(32, k - l0);
          for (int q = tid; q < 32 * 64; q += 256) {
            const int l = q / 64, ii = q % 64;
            smat[l * 64 + ii] = (l < nl && ii < nb) ? F[(long)(l0 + l) * len + o + ii] : make_float2(0.f, 0.f);
          }
          {
            const int l = tid / kHmR, r = tid % kHmR;   // 32 x 8 = 256 entries
            sx[l][r] = (l < nl && r < a.nr) ? zb[(long)(l0 + l) * kHmR + r] : make_double2(0.0, 0.0);
          }
          __syncthreads();
          if (valid)
            for (int l = g; l < nl; l += 4) fma_x(smat[l * 64 + lane], sx[l]);
          __syncthreads();
        }
      }
    }
    __syncthreads();   // the last batch's reads of smat are done
    // the four quarters' sums in order, through LDS (smat reused)
    double2* red = reinterpret_cast<double2*>(smat);   // [3][64][kHmR] (quarters 1..3)
    static_assert(sizeof(smat) >= 3 * 64 * kHmR * sizeof(double2), "reduction fits the staging buffer");
    if (g > 0)
#pragma unroll
      for (int r = 0; r < R; ++r) red[((g - 1) * 64 + lane) * kHmR + r] = make_double2(ar[r], ai[r]);
    __syncthreads();
    if (g == 0 && valid) {
      const int dst = a.perm[p0 + i];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r >= a.nr) break;
        double sr = ar[r], si = ai[r];
        for (int q = 0; q < 3; ++q) {
          sr += red[(q * 64 + lane) * kHmR + r].x;
          si += red[(q * 64 + lane) * kHmR + r].y;
        }
        a.y[(long)r * a.n + dst] = make_double2(sr, si);
      }
    }
    __syncthreads();
  }
}

// Dense write-out (complex64, the mesh's numbering): dense blocks and their
// transposes, low-rank blocks U V^T and their transposes.
template <int KIND>
__global__ __launch_bounds__(256) void k_hm_out_dense(int n, const int* __restrict__ perm, const int* __restrict__ row0,
                                                      const int2* __restrict__ ij, const float2* __restrict__ D,
                                                      const long* __restrict__ doff, float2* __restrict__ out) {
  const int b = blockIdx.x;
  const int I = ij[b].x, J = ij[b].y;
  int qI, nI, qJ, nJ;
  const float2* Db;
  if (KIND == 0) {
    qI = I * kEdgeTile;
    qJ = J * kEdgeTile;
    nI = min(kEdgeTile, n - qI);
    nJ = min(kEdgeTile, n - qJ);
    Db = D + (long)b * kEdgeTile * kEdgeTile;
  } else {
    qI = row0[I];
    nI = row0[I + 1] - qI;
    qJ = row0[J];
    nJ = row0[J + 1] - qJ;
    Db = D + doff[b];
  }
  const int ld = KIND == 0 ? kEdgeTile : nJ;
  for (int e = threadIdx.x; e < nI * nJ; e += 256) {
    const int r = e / nJ, c = e % nJ;
    const float2 v = Db[(long)r * ld + c];
    const long pr = perm[qI + r], pc = perm[qJ + c];
    out[pr * n + pc] = v;
    if (I != J) out[pc * n + pr] = v;
  }
}

__global__ __launch_bounds__(256) void k_hm_out_lr(int n, const int* __restrict__ perm, const HmLr* __restrict__ blk,
                                                   const int* __restrict__ rank, float2* const* __restrict__ Up,
                                                   float2* const* __restrict__ Vp, float2* __restrict__ out) {
  const int b = blockIdx.x;
  const HmLr B = blk[b];
  const int k = rank[b];
  const float2* U = Up[b];
  const float2* V = Vp[b];
  for (long e = threadIdx.x; e < (long)B.m * B.n; e += 256) {
    const int i = (int)(e / B.n), j = (int)(e % B.n);
    double sr = 0.0, si = 0.0;
    for (int l = 0; l < k; ++l) {
      const float2 u = U[(long)l * B.m + i], v = V[(long)l * B.n + j];
      sr += (double)u.x * v.x - (double)u.y * v.y;
      si += (double)u.x * v.y + (double)u.y * v.x;
    }
    const float2 val = make_float2((float)sr, (float)si);
    const long pr = perm[B.r0 + i], pc = perm[B.c0 + j];
    out[pr * n + pc] = val;
    out[pc * n + pr] = val;
  }
}

template <class T>
rfcmp_status upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  RF_TRY(b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1)));
  if (!v.empty()) RF_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  return RFCMP_OK;
}

}  // namespace

rfcmp_status hm_mesh_setup(rfcmp_mesh m, hipStream_t s) {
  if (m->hm) return RFCMP_OK;
  auto H = std::make_unique<HmMesh>();
  HmTree& t = H->t;
  hm_build_tree(m->h, t);
  const int64_t nd = (int64_t)t.dense_I.size(), nlr = (int64_t)t.lr_a.size();
  std::vector<int2> ij(nd);
  std::vector<long> voff(nd);
  int64_t vt = 0;
  for (int64_t b = 0; b < nd; ++b) {
    ij[b] = make_int2(t.dense_I[b], t.dense_J[b]);
    voff[b] = vt;
    vt += (int64_t)(t.cell_start[t.dense_I[b] + 1] - t.cell_start[t.dense_I[b]]) *
          (t.cell_start[t.dense_J[b] + 1] - t.cell_start[t.dense_J[b]]);
  }
  H->vd_total = vt;
  std::vector<HmLr> la(nlr), lv(nlr);
  for (int64_t b = 0; b < nlr; ++b) {
    const HmNode& A = t.nodes[t.lr_a[b]];
    const HmNode& B = t.nodes[t.lr_b[b]];
    la[b] = HmLr{(int)A.e0, (int)(A.e1 - A.e0), (int)B.e0, (int)(B.e1 - B.e0)};
    lv[b] = HmLr{(int)A.c0, (int)(A.c1 - A.c0), (int)B.c0, (int)(B.c1 - B.c0)};
  }
  // per tile, the blocks its rows meet (dense first, then low-rank, each in
  // block order)
  std::vector<std::vector<int>> lists(t.ntiles);
  for (int64_t b = 0; b < nd; ++b) {
    lists[t.dense_I[b]].push_back((int)(4 * b + 0));
    if (t.dense_I[b] != t.dense_J[b]) lists[t.dense_J[b]].push_back((int)(4 * b + 1));
  }
  for (int64_t b = 0; b < nlr; ++b) {
    const HmNode& A = t.nodes[t.lr_a[b]];
    const HmNode& B = t.nodes[t.lr_b[b]];
    for (int q = A.t0; q < A.t1; ++q) lists[q].push_back((int)(4 * b + 2));
    for (int q = B.t0; q < B.t1; ++q) lists[q].push_back((int)(4 * b + 3));
  }
  std::vector<int> lp(t.ntiles + 1, 0), le;
  for (int64_t q = 0; q < t.ntiles; ++q) {
    le.insert(le.end(), lists[q].begin(), lists[q].end());
    lp[q + 1] = (int)le.size();
  }
  RF_TRY(upload(H->perm_e, t.perm_e, s));
  RF_TRY(upload(H->perm_c, t.perm_c, s));
  RF_TRY(upload(H->iperm_c, t.iperm_c, s));
  RF_TRY(upload(H->cell_start, t.cell_start, s));
  RF_TRY(upload(H->et_ptr, t.et_ptr, s));
  RF_TRY(upload(H->et_cell, t.et_cell, s));
  RF_TRY(upload(H->et_rows, t.et_rows, s));
  RF_TRY(upload(H->home, t.home, s));
  RF_TRY(upload(H->dense_ij, ij, s));
  RF_TRY(upload(H->vd_off, voff, s));
  RF_TRY(upload(H->lrA, la, s));
  RF_TRY(upload(H->lrV, lv, s));
  RF_TRY(upload(H->list_ptr, lp, s));
  RF_TRY(upload(H->list_ent, le, s));
  RF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  H->list_host = std::move(le);
  m->hm = std::move(H);
  return RFCMP_OK;
}

rfcmp_status hm_aca(rfcmp_op op, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  const MeshDev& d = m->d;
  const HmMesh& H = *m->hm;
  HmOp& P = *op->hm;
  const HmTree& t = H.t;
  const int64_t nlr = (int64_t)t.lr_a.size();
  P.lr_entries[0] = P.lr_entries[1] = 0;
  P.unconverged = 0;
  std::vector<long> zoff_all[2];
  int64_t zw_need = 0;
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<HmLr> blk(nlr);
    for (int64_t b = 0; b < nlr; ++b) {
      const HmNode& A = t.nodes[t.lr_a[b]];
      const HmNode& B = t.nodes[t.lr_b[b]];
      blk[b] = kind == 0 ? HmLr{(int)A.e0, (int)(A.e1 - A.e0), (int)B.e0, (int)(B.e1 - B.e0)}
                         : HmLr{(int)A.c0, (int)(A.c1 - A.c0), (int)B.c0, (int)(B.c1 - B.c0)};
    }
    // passes over the blocks whose working factors (kmax columns) fit a
    // bounded pool
    std::vector<long> uoff(nlr), voff(nlr), toff(nlr);
    std::vector<int64_t> pass_start{0};
    const long pool_cap = 1L << 29;  // complex64 entries (4 GB)
    long used = 0, tused = 0, pool_max = 1, taken_max = 1;
    for (int64_t b = 0; b < nlr; ++b) {
      const long kc = std::min<long>(kHmKmax, std::min(blk[b].m, blk[b].n));
      const long need = kc * (blk[b].m + blk[b].n);
      if (b > pass_start.back() && used + need > pool_cap) {
        pass_start.push_back(b);
        used = 0;
        tused = 0;
      }
      uoff[b] = used;
      voff[b] = used + kc * blk[b].m;
      toff[b] = tused;
      used += need;
      tused += blk[b].m;
      pool_max = std::max(pool_max, used);
      taken_max = std::max(taken_max, tused);
    }
    pass_start.push_back(nlr);
    DevBuf dblk, duoff, dvoff, dtoff, drank, dflag, pool, taken;
    DevBuf& up = kind == 0 ? P.uA : P.uV;
    DevBuf& vp = kind == 0 ? P.vA : P.vV;
    DevBuf& rk = kind == 0 ? P.rankA : P.rankV;
    RF_TRY(upload(dblk, blk, s));
    RF_TRY(upload(duoff, uoff, s));
    RF_TRY(upload(dvoff, voff, s));
    RF_TRY(upload(dtoff, toff, s));
    RF_TRY(rk.alloc(sizeof(int) * std::max<int64_t>(nlr, 1)));
    RF_TRY(dflag.alloc(sizeof(int) * std::max<int64_t>(nlr, 1)));
    RF_TRY(up.alloc(sizeof(float2*) * std::max<int64_t>(nlr, 1)));
    RF_TRY(vp.alloc(sizeof(float2*) * std::max<int64_t>(nlr, 1)));
    RF_TRY(pool.alloc(sizeof(float2) * pool_max));
    RF_TRY(taken.alloc((size_t)taken_max));
    AcaArgs a;
    a.perm = kind == 0 ? H.perm_e.as<int>() : H.perm_c.as<int>();
    a.edge_slot = d.edge_slot.as<int>();
    a.cen = d.cen.as<double>();
    a.qoff = d.qoff.as<float4>();
    a.fvoff = d.fvoff.as<float4>();
    a.sgn = d.sgn.as<float>();
    a.rule = rule_args();
    a.kk = (float)op->k;
    a.tol = (float)P.tol;
    a.kmax = kHmKmax;
    a.blk = dblk.as<HmLr>();
    a.uoff = duoff.as<long>();
    a.voff = dvoff.as<long>();
    a.toff = dtoff.as<long>();
    a.pool = pool.as<float2>();
    a.taken = taken.as<unsigned char>();
    a.rank = rk.as<int>();
    a.flag = dflag.as<int>();
    std::vector<int>& hr = kind == 0 ? P.hrankA : P.hrankV;
    hr.assign(nlr, 0);
    std::vector<float2*> hu(nlr, nullptr), hv(nlr, nullptr);
    {
      ProfScope prof(kind == 0 ? "hm_aca_ta" : "hm_aca_v", s);
      for (size_t q = 0; q + 1 < pass_start.size(); ++q) {
        const int64_t b0 = pass_start[q], b1 = pass_start[q + 1];
        if (b1 <= b0) continue;
        void (*kern)(const AcaArgs, int) = kind == 0 ? k_aca<0> : k_aca<1>;
        hipLaunchKernelGGL(kern, dim3((unsigned)(b1 - b0)), dim3(kAcaThreads), 0, s, a, (int)b0);
        RF_HIP(hipGetLastError());
        RF_HIP(hipMemcpyAsync(hr.data() + b0, rk.as<int>() + b0, sizeof(int) * (b1 - b0), hipMemcpyDeviceToHost, s));
        RF_HIP(hipStreamSynchronize(s));
        long tot = 0;
        for (int64_t b = b0; b < b1; ++b) tot += (long)hr[b] * (blk[b].m + blk[b].n);
        P.store.push_back(std::make_unique<DevBuf>());
        DevBuf& st = *P.store.back();
        RF_TRY(st.alloc(sizeof(float2) * std::max<long>(tot, 1)));
        long o = 0;
        for (int64_t b = b0; b < b1; ++b) {
          hu[b] = st.as<float2>() + o;
          o += (long)hr[b] * blk[b].m;
          hv[b] = st.as<float2>() + o;
          o += (long)hr[b] * blk[b].n;
        }
        P.lr_entries[kind] += tot;
        RF_HIP(hipMemcpyAsync(up.as<float2*>() + b0, hu.data() + b0, sizeof(float2*) * (b1 - b0),
                              hipMemcpyHostToDevice, s));
        RF_HIP(hipMemcpyAsync(vp.as<float2*>() + b0, hv.data() + b0, sizeof(float2*) * (b1 - b0),
                              hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_aca_compact, dim3((unsigned)(b1 - b0)), dim3(256), 0, s, (int)b0, dblk.as<HmLr>(),
                           rk.as<int>(), duoff.as<long>(), dvoff.as<long>(), pool.as<float2>(),
                           up.as<float2*>(), vp.as<float2*>());
        RF_HIP(hipGetLastError());
        RF_HIP(hipStreamSynchronize(s));  // the pool is reused by the next pass
      }
    }
    std::vector<int> hf(nlr, 0);
    if (nlr > 0)
      RF_HIP(hipMemcpyAsync(hf.data(), dflag.p, sizeof(int) * nlr, hipMemcpyDeviceToHost, s));
    RF_HIP(hipStreamSynchronize(s));
    for (int64_t b = 0; b < nlr; ++b) P.unconverged += hf[b];
    // offsets of the projections z, w (2 k kHmR complex128 per block)
    std::vector<long>& zo = zoff_all[kind];
    zo.assign(nlr, 0);
    long zt = 0;
    for (int64_t b = 0; b < nlr; ++b) {
      zo[b] = zt;
      zt += 2L * hr[b] * kHmR;
    }
    zw_need = std::max<int64_t>(zw_need, zt);
    // the tile lists' entries resolved for this operator
    std::vector<HmEnt> ent(H.list_host.size());
    for (size_t e = 0; e < ent.size(); ++e) {
      const int code = H.list_host[e], b = code >> 2;
      HmEnt E{nullptr, 0, 0, 0, 0, code};
      if ((code & 3) >= 2) {
        const bool rows = (code & 3) == 2;
        E.F = rows ? hu[b] : hv[b];
        E.start = rows ? blk[b].r0 : blk[b].c0;
        E.len = rows ? blk[b].m : blk[b].n;
        E.k = hr[b];
        E.zb = zo[b] + (rows ? 0 : (long)hr[b] * kHmR);
      }
      ent[e] = E;
    }
    RF_TRY(upload(kind == 0 ? P.entA : P.entV, ent, s));
    RF_HIP(hipStreamSynchronize(s));  // ent goes out of scope
  }
  RF_TRY(upload(P.zwA, zoff_all[0], s));
  RF_TRY(upload(P.zwV, zoff_all[1], s));
  P.zw_total = zw_need;
  RF_TRY(P.zw.alloc(sizeof(double2) * std::max<int64_t>(zw_need, 1)));
  RF_TRY(P.xp.alloc(sizeof(double2) * kHmR * std::max<int64_t>(std::max(t.N, t.C), 1)));
  RF_HIP(hipStreamSynchronize(s));
  if (P.unconverged > 0) {
    set_error("ACA: %d low-rank blocks reached rank %d above the tolerance %g", P.unconverged, kHmKmax, P.tol);
    return RFCMP_E_STATE;
  }
  return RFCMP_OK;
}

rfcmp_status hm_matvec(rfcmp_op op, int which, bool conj, const double2* x, double2* y, int nr, hipStream_t s) {
  const HmMesh& H = *op->mesh->hm;
  HmOp& P = *op->hm;
  const HmTree& t = H.t;
  const int n = (int)(which == 0 ? t.N : t.C);
  const int64_t nlr = (int64_t)t.lr_a.size();
  if (n == 0 || nr <= 0) return RFCMP_OK;
  ProfScope prof(profiling_enabled() ? profile_tag_suffix(which == 0 ? "hm_matvec_ta" : "hm_matvec_v", nr) : "hm", s);
  TileArgs ta;
  ta.n = n;
  ta.perm = which == 0 ? H.perm_e.as<int>() : H.perm_c.as<int>();
  ta.row0 = H.cell_start.as<int>();
  ta.list_ptr = H.list_ptr.as<int>();
  ta.ent = which == 0 ? P.entA.as<HmEnt>() : P.entV.as<HmEnt>();
  ta.dense_ij = H.dense_ij.as<int2>();
  ta.D = which == 0 ? P.TAd.as<float2>() : P.Vd.as<float2>();
  ta.doff = H.vd_off.as<long>();
  ta.blk = which == 0 ? H.lrA.as<HmLr>() : H.lrV.as<HmLr>();
  ta.rank = which == 0 ? P.rankA.as<int>() : P.rankV.as<int>();
  ta.Up = which == 0 ? P.uA.as<float2*>() : P.uV.as<float2*>();
  ta.Vp = which == 0 ? P.vA.as<float2*>() : P.vV.as<float2*>();
  ta.zoff = which == 0 ? P.zwA.as<long>() : P.zwV.as<long>();
  ta.zw = P.zw.as<double2>();
  ta.xp = P.xp.as<double2>();
  ta.conj = conj ? 1 : 0;
  for (int r0 = 0; r0 < nr; r0 += kHmR) {
    const int rr = std::min(kHmR, nr - r0);
    const long tot = (long)n * rr;
    hipLaunchKernelGGL(k_hm_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rr, ta.perm,
                       x + (long)r0 * n, P.xp.as<double2>());
    // kernels for 1, 2, 4 or 8 right-hand sides: the smallest that holds rr
    const int R = rr <= 1 ? 1 : (rr <= 2 ? 2 : (rr <= 4 ? 4 : 8));
    typedef void (*Proj)(const HmLr*, const int*, float2* const*, float2* const*, const long*, const double2*, int,
                         int, int, double2*);
    typedef void (*Tile)(const TileArgs);
    const Proj proj = R == 1 ? k_hm_proj<1> : (R == 2 ? k_hm_proj<2> : (R == 4 ? k_hm_proj<4> : k_hm_proj<8>));
    const Tile tile = which == 0 ? (R == 1 ? k_hm_tile<0, 1> : (R == 2 ? k_hm_tile<0, 2> : (R == 4 ? k_hm_tile<0, 4>
                                                                                                    : k_hm_tile<0, 8>)))
                                 : (R == 1 ? k_hm_tile<1, 1> : (R == 2 ? k_hm_tile<1, 2> : (R == 4 ? k_hm_tile<1, 4>
                                                                                                    : k_hm_tile<1, 8>)));
    if (nlr > 0)
      hipLaunchKernelGGL(proj, dim3((unsigned)nlr), dim3(256), 0, s, ta.blk, ta.rank, ta.Up, ta.Vp, ta.zoff,
                         P.xp.as<double2>(), n, rr, ta.conj, P.zw.as<double2>());
    ta.nr = rr;
    ta.y = y + (long)r0 * n;
    hipLaunchKernelGGL(tile, dim3((unsigned)t.ntiles), dim3(256), 0, s, ta);
    RF_HIP(hipGetLastError());
  }
  return RFCMP_OK;
}

rfcmp_status hm_export(rfcmp_op op, float2* TA, float2* V, hipStream_t s) {
  const HmMesh& H = *op->mesh->hm;
  const HmOp& P = *op->hm;
  const HmTree& t = H.t;
  const int64_t nd = (int64_t)t.dense_I.size(), nlr = (int64_t)t.lr_a.size();
  if (TA) {
    RF_HIP(hipMemsetAsync(TA, 0, sizeof(float2) * t.N * t.N, s));
    if (nd > 0)
      hipLaunchKernelGGL(k_hm_out_dense<0>, dim3((unsigned)nd), dim3(256), 0, s, (int)t.N, H.perm_e.as<int>(),
                         H.cell_start.as<int>(), H.dense_ij.as<int2>(), P.TAd.as<float2>(), H.vd_off.as<long>(), TA);
    if (nlr > 0)
      hipLaunchKernelGGL(k_hm_out_lr, dim3((unsigned)nlr), dim3(256), 0, s, (int)t.N, H.perm_e.as<int>(),
                         H.lrA.as<HmLr>(), P.rankA.as<int>(), P.uA.as<float2*>(), P.vA.as<float2*>(), TA);
    RF_HIP(hipGetLastError());
  }
  if (V) {
    RF_HIP(hipMemsetAsync(V, 0, sizeof(float2) * t.C * t.C, s));
    if (nd > 0)
      hipLaunchKernelGGL(k_hm_out_dense<1>, dim3((unsigned)nd), dim3(256), 0, s, (int)t.C, H.perm_c.as<int>(),
                         H.cell_start.as<int>(), H.dense_ij.as<int2>(), P.Vd.as<float2>(), H.vd_off.as<long>(), V);
    if (nlr > 0)
      hipLaunchKernelGGL(k_hm_out_lr, dim3((unsigned)nlr), dim3(256), 0, s, (int)t.C, H.perm_c.as<int>(),
                         H.lrV.as<HmLr>(), P.rankV.as<int>(), P.uV.as<float2*>(), P.vV.as<float2*>(), V);
    RF_HIP(hipGetLastError());
  }
  return RFCMP_OK;
}

}  // namespace rfcmp
