// Solves with the sparse projector factors on the device (FP64), and the
// upload of a host factor.  See spchol.h for the layout and the launches.
//
// Every sum runs in a fixed order (fixed lane groups, fixed shuffle trees,
// children in order): the results do not depend on timing or on how the
// work is spread over workgroups.
#include <algorithm>

#include "spchol.h"
#include "symv_input.h"

namespace rfcmp {
namespace {

constexpr int kSpTopMax = 40;  // top heights of a factor

struct SpArg {
  int n, grounded, nrhs;  // nrhs: this job's right-hand sides
  int nsub, ntop, fr_k, ntile;
  long nstr_total;
  const int *perm, *iperm, *col0, *str_off, *str, *front_off, *fr_src;
  const long *linv_off, *l21_off, *blk_off;
  const double *l21, *l21t, *linv, *linvt, *blk;
  const int *sub_ptr, *sub_lvl;
  const int4 *sub_desc, *top_desc;
  int top_start[kSpTopMax + 1];  // first top position of each height
  SymvInput in;
  double2* y;
  double2* scratch;  // x [n][nrhs], u [nstr_total][nrhs], partial sums [ntile][nrhs], two means [2][nrhs]
  __device__ double2* u() const { return scratch + (long)n * nrhs; }
  __device__ double2* psum() const { return scratch + ((long)n + nstr_total) * nrhs; }
  __device__ double2* mean(int which) const { return scratch + ((long)n + nstr_total + ntile + which) * nrhs; }
};
struct SpArgs {
  SpArg a[2];
};

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cfma(double a, double2 v, double2 acc) {
  return make_double2(fma(a, v.x, acc.x), fma(a, v.y, acc.y));
}

// Order the wave's LDS and global accesses: everything the wave wrote is
// visible to all its lanes afterwards.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <int TEAM>
__device__ inline void team_sync() {
  if (TEAM == 64)
    wave_sync();
  else
    __syncthreads();
}

// Sum over the 64 lanes of a wave, in a fixed order.
__device__ inline double2 wave_sum(double2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// Lanes of a team of T over R right-hand sides (R a power of two <= 16):
// lane t serves right-hand side r = t mod R; G lanes (ids R apart, in one
// wave) split each sum; S = T / (R G) rows are formed at once.  G is the
// largest power of two with R G <= 64 and rows R G <= T.
struct Lanes {
  int r, g, slot, G, S;
};
__device__ inline Lanes lanes_of(int t, int T, int R, int rows) {
  int G = 1;
  while (R * G * 2 <= 64 && rows * R * G * 2 <= T) G *= 2;
  Lanes l;
  l.G = G;
  l.r = t & (R - 1);
  const int q = t / R;
  l.g = q & (G - 1);
  l.slot = q / G;
  l.S = T / (R * G);
  return l;
}
__device__ inline double2 group_sum(double2 v, int R, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o * R);
    v.y += __shfl_xor(v.y, o * R);
  }
  return v;
}

// sum over j = j0 + g, j0 + g + G, ... < j1 of M[j ld + i] V[j R + r], with
// up to sixteen loads of M in flight per lane
__device__ inline double2 strided_dot(const double* __restrict__ M, int ld, int i, const double2* V, int R, int r,
                                      int j0, int j1, int g, int G) {
  double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
  int j = j0 + g;
#pragma unroll 2
  for (; j + 7 * G < j1; j += 8 * G) {
    double m[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) m[e] = M[(long)(j + e * G) * ld + i];
    a0 = cfma(m[0], V[j * R + r], a0);
    a1 = cfma(m[1], V[(j + G) * R + r], a1);
    a2 = cfma(m[2], V[(j + 2 * G) * R + r], a2);
    a3 = cfma(m[3], V[(j + 3 * G) * R + r], a3);
    a0 = cfma(m[4], V[(j + 4 * G) * R + r], a0);
    a1 = cfma(m[5], V[(j + 5 * G) * R + r], a1);
    a2 = cfma(m[6], V[(j + 6 * G) * R + r], a2);
    a3 = cfma(m[7], V[(j + 7 * G) * R + r], a3);
  }
  for (; j < j1; j += G) a0 = cfma(M[(long)j * ld + i], V[j * R + r], a0);
  return cadd(cadd(a0, a1), cadd(a2, a3));
}

// Forward step of a supernode (descriptor d0 = {col0, ncol, str_off, nstr},
// d1 = {front_off, linv_off, l21_off, 0}) for right-hand sides r0 .. r0+R-1
// on a team of TEAM lanes; lds: (2 ncol + nstr) R entries.
template <int TEAM>
__device__ void node_forward(const SpArg& A, int4 d0, int4 d1, int t, int R, int r0, double2* lds) {
  const int NR = A.nrhs;
  double2* x = A.scratch;
  double2* u = A.u();
  const int c0 = d0.x, ncol = d0.y, so = d0.z, nstr = d0.w;
  const int fo = d1.x, m = ncol + nstr, K = A.fr_k;
  double2* v = lds;              // front [m][R]
  double2* yv = lds + m * R;     // y [ncol][R]
  {  // the front: x on the columns (less the input mean of the Laplacian)
     // plus the children's update entries
    const int r = t & (R - 1), rg = r0 + r;
    const double2 mu = (A.grounded && rg < NR) ? A.mean(0)[rg] : make_double2(0.0, 0.0);
    for (int p = t / R; p < m; p += TEAM / R) {
      double2 val = make_double2(0.0, 0.0);
      if (rg < NR) {
        if (p < ncol) {
          const double2 xv = x[(long)(c0 + p) * NR + rg];
          val = make_double2(xv.x - mu.x, xv.y - mu.y);
        }
        // the gather indices of up to four sources first, then their
        // entries (added in source order)
        for (int k0 = 0; k0 < K; k0 += 4) {
          int q[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) q[k] = k0 + k < K ? A.fr_src[(long)(fo + p) * K + k0 + k] : -1;
          double2 w[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) w[k] = q[k] >= 0 ? u[(long)q[k] * NR + rg] : make_double2(0.0, 0.0);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (q[k] >= 0) val = cadd(val, w[k]);
        }
      }
      v[p * R + r] = val;
    }
  }
  team_sync<TEAM>();
  {  // y_i = (L_ss^-1 v)_i: columns j <= i
    const Lanes L = lanes_of(t, TEAM, R, ncol);
    const double* M = A.linv + d1.y;
    const int rg = r0 + L.r;
    for (int base = 0; base < ncol; base += L.S) {
      const int i = base + L.slot;
      const double2 acc = group_sum(strided_dot(M, ncol, i, v, R, L.r, 0, i < ncol ? i + 1 : 0, L.g, L.G), R, L.G);
      if (i < ncol && L.g == 0) {
        yv[i * R + L.r] = acc;
        if (rg < NR) x[(long)(c0 + i) * NR + rg] = acc;
      }
    }
  }
  team_sync<TEAM>();
  {  // u_q = v_(ncol + q) - (L_21 y)_q
    const Lanes L = lanes_of(t, TEAM, R, nstr);
    const double* M = A.l21 + d1.z;
    const int rg = r0 + L.r;
    for (int base = 0; base < nstr; base += L.S) {
      const int q = base + L.slot;
      const double2 acc = group_sum(strided_dot(M, nstr, q, yv, R, L.r, 0, q < nstr ? ncol : 0, L.g, L.G), R, L.G);
      if (q < nstr && L.g == 0 && rg < NR) {
        const double2 w = v[(ncol + q) * R + L.r];
        u[(long)(so + q) * NR + rg] = make_double2(w.x - acc.x, w.y - acc.y);
      }
    }
  }
  team_sync<TEAM>();
}

// Backward step of a supernode: x_s = L_ss^-T (y - L_21^T x_struct).
// ylds: y as the forward step left it in LDS (a root, right after its
// forward step), else null (y read from x).
template <int TEAM>
__device__ void node_backward(const SpArg& A, int4 d0, int4 d1, int t, int R, int r0, double2* lds,
                              const double2* ylds = nullptr) {
  const int NR = A.nrhs;
  double2* x = A.scratch;
  const int c0 = d0.x, ncol = d0.y, so = d0.z, nstr = d0.w;
  double2* xs = lds;              // x_struct [nstr][R]
  double2* z = lds + nstr * R;    // z [ncol][R]
  {
    const int r = t & (R - 1), rg = r0 + r;
    for (int q = t / R; q < nstr; q += TEAM / R)
      xs[q * R + r] = rg < NR ? x[(long)A.str[so + q] * NR + rg] : make_double2(0.0, 0.0);
  }
  team_sync<TEAM>();
  {  // z_j = y_j - (L_21^T x_struct)_j
    const Lanes L = lanes_of(t, TEAM, R, ncol);
    const double* M = A.l21t + d1.z;  // (q, j) at M[q * ncol + j]
    const int rg = r0 + L.r;
    for (int base = 0; base < ncol; base += L.S) {
      const int j = base + L.slot;
      const double2 acc = group_sum(strided_dot(M, ncol, j, xs, R, L.r, 0, j < ncol ? nstr : 0, L.g, L.G), R, L.G);
      if (j < ncol && L.g == 0) {
        const double2 yy = ylds ? ylds[j * R + L.r] : (rg < NR ? x[(long)(c0 + j) * NR + rg] : make_double2(0.0, 0.0));
        z[j * R + L.r] = make_double2(yy.x - acc.x, yy.y - acc.y);
      }
    }
  }
  team_sync<TEAM>();
  {  // x_i = (L_ss^-T z)_i: rows j >= i
    const Lanes L = lanes_of(t, TEAM, R, ncol);
    const double* M = A.linvt + d1.y;  // (i, j) of L_ss^-T at M[j * ncol + i]
    const int rg = r0 + L.r;
    for (int base = 0; base < ncol; base += L.S) {
      const int i = base + L.slot;
      const double2 acc =
          group_sum(strided_dot(M, ncol, i, z, R, L.r, i < ncol ? i : 0, i < ncol ? ncol : 0, L.g, L.G), R, L.G);
      if (i < ncol && L.g == 0 && rg < NR) x[(long)(c0 + i) * NR + rg] = acc;
    }
  }
  team_sync<TEAM>();
}

constexpr int kSpThreads = 1024;
constexpr int kSpTileR = 16;  // right-hand sides per workgroup of the permutation kernels
static_assert(kSpTile * kSpTileR == kSpThreads, "one permutation tile per workgroup");

// input: x = P (the right-hand side); a tile of kSpTile entries by kSpTileR
// right-hand sides per workgroup, read along the entries and written along
// the right-hand sides.  For the Laplacian also the tile's sums (each wave
// holds one right-hand side of the tile).
__global__ void __launch_bounds__(kSpThreads) k_sp_input(const SpArgs args) {
  const SpArg& A = args.a[blockIdx.z];
  const int g0 = blockIdx.x * kSpTile, r0 = blockIdx.y * kSpTileR, NR = A.nrhs;
  if (g0 >= A.n || r0 >= NR) return;
  __shared__ double2 tile[kSpTile][kSpTileR + 1];
  const int t = threadIdx.x;
  {
    const int gl = t % kSpTile, rl = t / kSpTile, g = g0 + gl, r = r0 + rl;
    const double2 v = (g < A.n && r < NR) ? input_entry(A.in, r, g) : make_double2(0.0, 0.0);
    tile[gl][rl] = v;
    if (A.grounded) {
      const double2 s = wave_sum(v);
      if (gl == 0 && r < NR) A.psum()[(long)blockIdx.x * NR + r] = s;
    }
  }
  __syncthreads();
  {
    const int rl = t % kSpTileR, gl = t / kSpTileR, g = g0 + gl, r = r0 + rl;
    if (g < A.n && r < NR) A.scratch[(long)A.iperm[g] * NR + r] = tile[gl][rl];
  }
}

// The Laplacian's partial sums of x over tiles of the permuted entries
// (after the backward sweep).
__global__ void __launch_bounds__(kSpThreads) k_sp_colsum(const SpArgs args) {
  const SpArg& A = args.a[blockIdx.z];
  const int i0 = blockIdx.x * kSpTile, r0 = blockIdx.y * kSpTileR, NR = A.nrhs;
  if (!A.grounded || i0 >= A.n || r0 >= NR) return;
  __shared__ double2 tile[kSpTile][kSpTileR + 1];
  const int t = threadIdx.x;
  {
    const int rl = t % kSpTileR, il = t / kSpTileR, i = i0 + il, r = r0 + rl;
    tile[il][rl] = (i < A.n && r < NR) ? A.scratch[(long)i * NR + r] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  {
    const int il = t % kSpTile, rl = t / kSpTile, r = r0 + rl;
    const double2 s = wave_sum(tile[il][rl]);
    if (il == 0 && r < NR) A.psum()[(long)blockIdx.x * NR + r] = s;
  }
}

// The Laplacian's mean (which 0: of the input, 1: of the result) from the
// partial sums, in a fixed order.
__global__ void __launch_bounds__(kSpThreads) k_sp_mean(const SpArgs args, int which) {
  const SpArg& A = args.a[blockIdx.z];
  const int r0 = blockIdx.x * kSpTileR, NR = A.nrhs;
  if (!A.grounded || r0 >= NR) return;
  __shared__ double2 red[kSpThreads / kSpTileR][kSpTileR];
  const int t = threadIdx.x, rl = t % kSpTileR, part = t / kSpTileR, r = r0 + rl;
  constexpr int P = kSpThreads / kSpTileR;
  double2 s = make_double2(0.0, 0.0);
  if (r < NR)
    for (int b = part; b < A.ntile; b += P) s = cadd(s, A.psum()[(long)b * NR + r]);
  red[part][rl] = s;
  __syncthreads();
  if (t < kSpTileR && r0 + t < NR) {
    double2 tot = make_double2(0.0, 0.0);
    for (int q = 0; q < P; ++q) tot = cadd(tot, red[q][t]);
    A.mean(which)[r0 + t] = make_double2(tot.x / A.n, tot.y / A.n);
  }
}

// output: y = P^T x (less the Laplacian's mean of the result); read along
// the right-hand sides, written along the entries
__global__ void __launch_bounds__(kSpThreads) k_sp_output(const SpArgs args) {
  const SpArg& A = args.a[blockIdx.z];
  const int g0 = blockIdx.x * kSpTile, r0 = blockIdx.y * kSpTileR, NR = A.nrhs;
  if (g0 >= A.n || r0 >= NR) return;
  __shared__ double2 tile[kSpTile][kSpTileR + 1];
  const int t = threadIdx.x;
  {
    const int rl = t % kSpTileR, gl = t / kSpTileR, g = g0 + gl, r = r0 + rl;
    double2 v = make_double2(0.0, 0.0);
    if (g < A.n && r < NR) {
      v = A.scratch[(long)A.iperm[g] * NR + r];
      if (A.grounded) {
        const double2 mu = A.mean(1)[r];
        v = make_double2(v.x - mu.x, v.y - mu.y);
      }
    }
    tile[gl][rl] = v;
  }
  __syncthreads();
  {
    const int gl = t % kSpTile, rl = t / kSpTile, g = g0 + gl, r = r0 + rl;
    if (g < A.n && r < NR) A.y[(long)r * A.n + g] = tile[gl][rl];
  }
}

// A bottom supernode is solved by one wave from LDS (staged) when its blocks
// hold at most kSpStageMax entries and its gather indices at most kSpIdxMax:
// the wave issues the loads of the indices, its entries of the vector and
// the blocks (512 entries per round) together, then those of the update
// entries of its children (or, backward, the entries of its struct rows),
// eight per lane per round, and forms both products from LDS, so a step
// costs a few round trips to memory instead of one per row.
// A supernode that cannot be staged, and its ancestors, belong to the top.
constexpr int kSpStageMax = 1024;
constexpr int kSpIdxMax = 256;
__host__ __device__ inline bool sp_staged(int ncol, int nstr, int K) {
  return ncol * (ncol + nstr) <= kSpStageMax && (ncol + nstr) * K <= kSpIdxMax;
}

// Forward step of a staged supernode (descriptor record d0 = {col0, ncol,
// str_off, nstr}, d1 = {front_off, blk_off, 0, 0}) on one wave (lane 0..63,
// R right-hand sides from r0; a lane holds rows p0 + P a, a < ROWS, of the
// node's columns: P ROWS >= ncol).  lds: the wave's slice, the front [m][R] first; F: the
// blocks (L_ss^-1, then L_21, both column-major, as stored contiguously per
// staged supernode at blk + blk_off); S: the gather indices.
template <int ROWS>
__device__ void wave_forward(const SpArg& A, int4 d0, int4 d1, int lane, int R, int r0, double2* lds, double* F,
                             int* S, bool leaf) {
  const int NR = A.nrhs, K = A.fr_k;
  double2* x = A.scratch;
  double2* u = A.u();
  const int c0 = d0.x, ncol = d0.y, so = d0.z, nstr = d0.w, fo = d1.x;
  const double* B = A.blk + d1.y;
  const int m = ncol + nstr, nn = ncol * ncol, nf = nn + ncol * nstr, nidx = leaf ? 0 : m * K;
  const int r = lane & (R - 1), rg = r0 + r, P = 64 / R, p0 = lane / R;
  const bool live = rg < NR;
  const double2 zero = make_double2(0.0, 0.0);
  double2* v = lds;
  // the blocks, the gather indices and the node's entries of the vector (the
  // Laplacian's input mean taken off), all issued before any is used
  int g[kSpIdxMax / 64];
#pragma unroll
  for (int i = 0; i < kSpIdxMax / 64; ++i) {
    const int e = lane + 64 * i;
    g[i] = e < nidx ? A.fr_src[(long)fo * K + e] : -1;
  }
  const double2 mu = (A.grounded && live) ? A.mean(0)[rg] : zero;
  double2 xv[ROWS];
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int p = p0 + P * a;
    xv[a] = (p < ncol && live) ? x[(long)(c0 + p) * NR + rg] : zero;
  }
  for (int e0 = lane; e0 < nf; e0 += 512) {
    double f[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = e0 + 64 * i < nf ? B[e0 + 64 * i] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (e0 + 64 * i < nf) F[e0 + 64 * i] = f[i];
  }
#pragma unroll
  for (int i = 0; i < kSpIdxMax / 64; ++i)
    if (lane + 64 * i < nidx) S[lane + 64 * i] = g[i];
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int p = p0 + P * a;
    if (p < ncol) v[p * R + r] = make_double2(xv[a].x - mu.x, xv[a].y - mu.y);
  }
  for (int p = p0; p < m; p += P)
    if (p >= ncol) v[p * R + r] = zero;
  wave_sync();
  // the children's update entries, added per front entry in child order
  if (!leaf) {
    const int nw = ((m - p0 + P - 1) / P) * K;
    for (int w0 = 0; w0 < nw; w0 += 8) {
      double2 t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int w = w0 + i;
        const int q = w < nw ? S[(p0 + P * (w / K)) * K + w % K] : -1;
        t[i] = (q >= 0 && live) ? u[(long)q * NR + rg] : zero;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int w = w0 + i;
        if (w < nw) {
          double2* vp = v + (p0 + P * (w / K)) * R + r;
          *vp = cadd(*vp, t[i]);
        }
      }
    }
    wave_sync();
  }
  // y = L_ss^-1 v_cols (rows p0 + P a), then into the front and x
  double2 y[ROWS];
#pragma unroll
  for (int a = 0; a < ROWS; ++a) y[a] = zero;
#pragma unroll 2
  for (int j = 0; j < ncol; ++j) {
    const double2 vj = v[j * R + r];
#pragma unroll
    for (int a = 0; a < ROWS; ++a) {
      const int i = p0 + P * a;
      if (i < ncol && j <= i) y[a] = cfma(F[j * ncol + i], vj, y[a]);
    }
  }
  wave_sync();
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int i = p0 + P * a;
    if (i < ncol) {
      v[i * R + r] = y[a];
      if (live) x[(long)(c0 + i) * NR + rg] = y[a];
    }
  }
  wave_sync();
  // u = v_struct - L_21 y
  for (int q0 = p0; q0 < nstr; q0 += ROWS * P) {
    double2 acc[ROWS];
#pragma unroll
    for (int b = 0; b < ROWS; ++b) acc[b] = zero;
#pragma unroll 2
    for (int j = 0; j < ncol; ++j) {
      const double2 yj = v[j * R + r];
#pragma unroll
      for (int b = 0; b < ROWS; ++b) {
        const int q = q0 + P * b;
        if (q < nstr) acc[b] = cfma(F[nn + j * nstr + q], yj, acc[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < ROWS; ++b) {
      const int q = q0 + P * b;
      if (q < nstr && live) {
        const double2 w = v[(ncol + q) * R + r];
        u[(long)(so + q) * NR + rg] = make_double2(w.x - acc[b].x, w.y - acc[b].y);
      }
    }
  }
  wave_sync();
}

// Backward step of a staged supernode on one wave: z = y - L_21^T x_struct,
// x = L_ss^-T z, from the same blocks as the forward step.
template <int ROWS>
__device__ void wave_backward(const SpArg& A, int4 d0, int4 d1, int lane, int R, int r0, double2* lds, double* F,
                              int* S) {
  const int NR = A.nrhs;
  double2* x = A.scratch;
  const int c0 = d0.x, ncol = d0.y, so = d0.z, nstr = d0.w;
  const double* B = A.blk + d1.y;
  const int nn = ncol * ncol, nf = nn + ncol * nstr;
  const int r = lane & (R - 1), rg = r0 + r, P = 64 / R, p0 = lane / R;
  const bool live = rg < NR;
  const double2 zero = make_double2(0.0, 0.0);
  double2* xs = lds;             // x_struct [nstr][R]
  double2* z = lds + nstr * R;   // z [ncol][R]
  int g[kSpIdxMax / 64];
#pragma unroll
  for (int i = 0; i < kSpIdxMax / 64; ++i) {
    const int e = lane + 64 * i;
    g[i] = e < nstr ? A.str[so + e] : 0;
  }
  double2 yv[ROWS];  // the forward step's y
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int j = p0 + P * a;
    yv[a] = (j < ncol && live) ? x[(long)(c0 + j) * NR + rg] : zero;
  }
  for (int e0 = lane; e0 < nf; e0 += 512) {
    double f[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = e0 + 64 * i < nf ? B[e0 + 64 * i] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (e0 + 64 * i < nf) F[e0 + 64 * i] = f[i];
  }
#pragma unroll
  for (int i = 0; i < kSpIdxMax / 64; ++i)
    if (lane + 64 * i < nstr) S[lane + 64 * i] = g[i];
  wave_sync();
  // x_struct: the solution on the struct rows
  for (int q0 = p0; q0 < nstr; q0 += 8 * P) {
    double2 t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = q0 + P * i;
      t[i] = (q < nstr && live) ? x[(long)S[q] * NR + rg] : zero;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = q0 + P * i;
      if (q < nstr) xs[q * R + r] = t[i];
    }
  }
  wave_sync();
  // z_j = y_j - (L_21^T x_struct)_j
  double2 acc[ROWS];
#pragma unroll
  for (int a = 0; a < ROWS; ++a) acc[a] = zero;
#pragma unroll 2
  for (int q = 0; q < nstr; ++q) {
    const double2 xq = xs[q * R + r];
#pragma unroll
    for (int a = 0; a < ROWS; ++a) {
      const int j = p0 + P * a;
      if (j < ncol) acc[a] = cfma(F[nn + j * nstr + q], xq, acc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int j = p0 + P * a;
    if (j < ncol) z[j * R + r] = make_double2(yv[a].x - acc[a].x, yv[a].y - acc[a].y);
  }
  wave_sync();
  // x_i = (L_ss^-T z)_i = sum over j >= i of (L_ss^-1)_ji z_j
#pragma unroll
  for (int a = 0; a < ROWS; ++a) acc[a] = zero;
#pragma unroll 2
  for (int j = 0; j < ncol; ++j) {
    const double2 zj = z[j * R + r];
#pragma unroll
    for (int a = 0; a < ROWS; ++a) {
      const int i = p0 + P * a;
      if (i <= j) acc[a] = cfma(F[i * ncol + j], zj, acc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    const int i = p0 + P * a;
    if (i < ncol && live) x[(long)(c0 + i) * NR + rg] = acc[a];
  }
  wave_sync();
}

// bottom subtrees: one workgroup per (subtree, R right-hand sides, job); the
// subtree's heights in order, one wave per (staged) supernode, at most
// kSpBottomWaves waves.  A wave's LDS slice (sp_slice entries): the fronts, `vec` entries
// per right-hand side, then the staged blocks (`fac` doubles, even) and the
// gather indices (`idx` ints, a multiple of 4).
constexpr int kSpBottomWaves = 8;
constexpr int kSpBottomMinWaves = 3;
constexpr int kSpBottomTarget = 512;
__host__ __device__ inline int sp_slice(int R, int vec, int fac, int idx) { return vec * R + fac / 2 + idx / 4; }
template <int ROWS>
__global__ void __launch_bounds__(64 * kSpBottomWaves)
    k_sp_bottom(const SpArgs args, int backward, int R, int vec, int fac, int idx) {
  const SpArg& A = args.a[blockIdx.z];
  const int b = blockIdx.x, r0 = blockIdx.y * R;
  if (b >= A.nsub || r0 >= A.nrhs) return;
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int slice = sp_slice(R, vec, fac, idx);
  double2* mine = lds + (long)wave * slice;
  double* F = reinterpret_cast<double*>(mine + vec * R);
  int* S = reinterpret_cast<int*>(F + fac);
  const int l0 = A.sub_ptr[b], nl = A.sub_ptr[b + 1] - l0 - 1;
  for (int q = 0; q < nl; ++q) {
    const int l = backward ? nl - 1 - q : q;
    // the wave's supernodes of this height, each one's descriptor record
    // loaded while the previous supernode is solved
    const int kend = A.sub_lvl[l0 + l + 1];
    int k = A.sub_lvl[l0 + l] + wave;
    int4 d0 = make_int4(0, 0, 0, 0), d1 = d0;
    if (k < kend) {
      d0 = A.sub_desc[2 * k];
      d1 = A.sub_desc[2 * k + 1];
    }
    for (; k < kend; k += W) {
      int4 n0 = make_int4(0, 0, 0, 0), n1 = n0;
      if (k + W < kend) {
        n0 = A.sub_desc[2 * (k + W)];
        n1 = A.sub_desc[2 * (k + W) + 1];
      }
      if (backward)
        wave_backward<ROWS>(A, d0, d1, lane, R, r0, mine, F, S);
      else
        wave_forward<ROWS>(A, d0, d1, lane, R, r0, mine, F, S, l == 0);
      d0 = n0;
      d1 = n1;
    }
    __syncthreads();
  }
}

// one top height: one workgroup per (supernode, R right-hand sides, job);
// backward 2: the forward and then the backward step (the highest height,
// whose supernodes are roots: no struct rows, so the backward step needs
// nothing but the forward step's result)
__global__ void __launch_bounds__(kSpThreads) k_sp_top(const SpArgs args, int level, int backward, int R) {
  const SpArg& A = args.a[blockIdx.z];
  const int r0 = blockIdx.y * R;
  if (level >= A.ntop || r0 >= A.nrhs) return;
  const int k = A.top_start[level] + blockIdx.x;
  if (k >= A.top_start[level + 1]) return;
  extern __shared__ double2 lds[];
  const int4 d0 = A.top_desc[2 * k], d1 = A.top_desc[2 * k + 1];
  if (backward == 0) {
    node_forward<kSpThreads>(A, d0, d1, threadIdx.x, R, r0, lds);
  } else if (backward == 1) {
    node_backward<kSpThreads>(A, d0, d1, threadIdx.x, R, r0, lds);
  } else {  // a root: the forward step leaves y at lds + ncol R, past the z the backward step writes
    node_forward<kSpThreads>(A, d0, d1, threadIdx.x, R, r0, lds);
    node_backward<kSpThreads>(A, d0, d1, threadIdx.x, R, r0, lds, lds + d0.y * R);
  }
}

// Right-hand sides per workgroup: the largest power of two up to 16 that
// still gives about `target` workgroups over `units` units of work and whose
// LDS (`need` entries per right-hand side, times `teams`) fits 64 KB.
int rhs_per_group(int nrhs, int units, int target, int need, int teams) {
  int R = 1;
  while (R < 16 && (int64_t)nrhs * units >= (int64_t)2 * R * target) R *= 2;
  while (R > 1 && (int64_t)teams * need * R * (int64_t)sizeof(double2) > 65536) R /= 2;
  return R;
}

}  // namespace

rfcmp_status spsolve_jobs(const SpSolveJob* jobs, int njobs, int nrhs, hipStream_t s, const char* tag) {
  if (njobs < 1 || njobs > 2 || nrhs <= 0) {
    set_error("spsolve: 1 or 2 jobs and nrhs > 0 required");
    return RFCMP_E_ARG;
  }
  SpArgs args{};
  int nsub = 0, ntop = 0, blds = 0, bfac = 0, bidx = 0, bncol = 0, ntile = 0;
  bool grounded = false;
  for (int q = 0; q < njobs; ++q) {
    const SpDevice& F = *jobs[q].F;
    SpArg& a = args.a[q];
    a.n = F.n;
    a.grounded = F.grounded;
    a.nsub = F.nsub;
    a.ntop = F.ntop;
    a.fr_k = F.fr_k;
    a.ntile = (int)F.tiles();
    a.nstr_total = F.nstr_total;
    a.perm = F.perm.as<int>();
    a.iperm = F.iperm.as<int>();
    a.col0 = F.col0.as<int>();
    a.str_off = F.str_off.as<int>();
    a.str = F.str.as<int>();
    a.front_off = F.front_off.as<int>();
    a.fr_src = F.fr_src.as<int>();
    a.linv_off = F.linv_off.as<long>();
    a.l21_off = F.l21_off.as<long>();
    a.blk_off = F.blk_off.as<long>();
    a.blk = F.blk.as<double>();
    a.l21 = F.l21.as<double>();
    a.l21t = F.l21t.as<double>();
    a.linv = F.linv.as<double>();
    a.linvt = F.linvt.as<double>();
    a.sub_ptr = F.sub_ptr.as<int>();
    a.sub_lvl = F.sub_lvl.as<int>();
    a.sub_desc = F.sub_desc.as<int4>();
    a.top_desc = F.top_desc.as<int4>();
    if (F.ntop > kSpTopMax) {
      set_error("spsolve: %d top heights (at most %d)", F.ntop, kSpTopMax);
      return RFCMP_E_STATE;
    }
    for (int l = 0; l <= F.ntop; ++l) a.top_start[l] = F.top_start[l];
    a.in = jobs[q].in;
    a.y = jobs[q].y;
    a.scratch = jobs[q].scratch;
    a.nrhs = (q == 1 && jobs[1].nrhs > 0) ? std::min(jobs[1].nrhs, nrhs) : nrhs;
    nsub = std::max(nsub, F.nsub);
    ntop = std::max(ntop, F.ntop);
    blds = std::max(blds, F.bot_lds);
    bfac = std::max(bfac, F.bot_fac);
    bidx = std::max(bidx, F.bot_idx);
    bncol = std::max(bncol, F.bot_ncol);
    ntile = std::max(ntile, a.ntile);
    grounded = grounded || F.grounded;
  }
  // bottom: about kSpBottomTarget workgroups, each of up to kSpBottomWaves
  // waves and at least kSpBottomMinWaves where their slices fit 64 KB; the
  // rows per lane from the widest bottom supernode
  int Rb = 1, W = 1, rows = 1;
  int64_t slice = 0;
  if (nsub > 0) {
    while (Rb < 16 && (int64_t)nrhs * nsub >= (int64_t)2 * Rb * kSpBottomTarget) Rb *= 2;
    while (Rb > 1 && (int64_t)kSpBottomMinWaves * sp_slice(Rb, blds, bfac, bidx) * (int64_t)sizeof(double2) > 65536)
      Rb /= 2;
    slice = sp_slice(Rb, blds, bfac, bidx);
    if (slice * (int64_t)sizeof(double2) > 65536) {
      set_error("spsolve: a front of %d entries does not fit the LDS", blds);
      return RFCMP_E_STATE;
    }
    W = (int)std::min<int64_t>(kSpBottomWaves, 65536 / (slice * (int64_t)sizeof(double2)));
    while (rows * (64 / Rb) < bncol) rows *= 2;
  }
  // top: per height, about 256 workgroups
  std::vector<int> Rt(ntop), nodes(ntop), need(ntop);
  for (int l = 0; l < ntop; ++l) {
    for (int q = 0; q < njobs; ++q) {
      const SpDevice& F = *jobs[q].F;
      if (l < F.ntop) {
        nodes[l] = std::max(nodes[l], F.top_count[l]);
        need[l] = std::max(need[l], F.top_lds[l]);
      }
    }
    Rt[l] = rhs_per_group(nrhs, nodes[l], 256, need[l], 1);
    if ((int64_t)need[l] * Rt[l] * (int64_t)sizeof(double2) > 65536) {
      set_error("spsolve: a front of %d entries does not fit the LDS", need[l]);
      return RFCMP_E_STATE;
    }
  }
  const unsigned nj = (unsigned)njobs, nrt = (unsigned)((nrhs + kSpTileR - 1) / kSpTileR);
  const dim3 tiles((unsigned)ntile, nrt, nj);
  ProfScope prof(tag, s);
  hipLaunchKernelGGL(k_sp_input, tiles, dim3(kSpThreads), 0, s, args);
  if (grounded) hipLaunchKernelGGL(k_sp_mean, dim3(nrt, 1, nj), dim3(kSpThreads), 0, s, args, 0);
  const dim3 bgrid((unsigned)nsub, (unsigned)((nrhs + Rb - 1) / Rb), nj);
  auto bottom = [&](int bwd) -> rfcmp_status {
    const size_t lds = (size_t)(W * slice) * sizeof(double2);
    switch (rows) {
      case 1: hipLaunchKernelGGL(k_sp_bottom<1>, bgrid, dim3(64 * W), lds, s, args, bwd, Rb, blds, bfac, bidx); break;
      case 2: hipLaunchKernelGGL(k_sp_bottom<2>, bgrid, dim3(64 * W), lds, s, args, bwd, Rb, blds, bfac, bidx); break;
      case 4: hipLaunchKernelGGL(k_sp_bottom<4>, bgrid, dim3(64 * W), lds, s, args, bwd, Rb, blds, bfac, bidx); break;
      case 8: hipLaunchKernelGGL(k_sp_bottom<8>, bgrid, dim3(64 * W), lds, s, args, bwd, Rb, blds, bfac, bidx); break;
      default:
        set_error("spsolve: %d rows per lane", rows);
        return RFCMP_E_STATE;
    }
    return RFCMP_OK;
  };
  if (nsub > 0)
    RF_TRY(bottom(0));
  auto top = [&](int l, int bwd) {
    hipLaunchKernelGGL(k_sp_top, dim3((unsigned)nodes[l], (unsigned)((nrhs + Rt[l] - 1) / Rt[l]), nj), dim3(kSpThreads),
                       (size_t)need[l] * Rt[l] * sizeof(double2), s, args, l, bwd, Rt[l]);
  };
  // the highest height in one launch when its supernodes are roots
  bool roots = true;
  for (int q = 0; q < njobs; ++q)
    if (jobs[q].F->ntop == ntop) roots = roots && jobs[q].F->top_roots;
  const int fused = (ntop > 0 && roots) ? 1 : 0;
  for (int l = 0; l < ntop - fused; ++l) top(l, 0);
  if (fused) top(ntop - 1, 2);
  for (int l = ntop - 1 - fused; l >= 0; --l) top(l, 1);
  if (nsub > 0)
    RF_TRY(bottom(1));
  if (grounded) {
    hipLaunchKernelGGL(k_sp_colsum, tiles, dim3(kSpThreads), 0, s, args);
    hipLaunchKernelGGL(k_sp_mean, dim3(nrt, 1, nj), dim3(kSpThreads), 0, s, args, 1);
  }
  hipLaunchKernelGGL(k_sp_output, tiles, dim3(kSpThreads), 0, s, args);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

void spchol_arrays(const SpFactor& F, SpArrays& a) {
  const int n = F.n, nsn = F.nsn;
  // block offsets and front offsets
  a.linv_off.assign(nsn + 1, 0);
  a.l21_off.assign(nsn + 1, 0);
  a.front_off.assign(nsn + 1, 0);
  a.max_ncol = 0;
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    a.linv_off[q + 1] = a.linv_off[q] + (long)ncol * ncol;
    a.l21_off[q + 1] = a.l21_off[q] + (long)nstr * ncol;
    a.front_off[q + 1] = a.front_off[q] + ncol + nstr;
    a.max_ncol = std::max(a.max_ncol, ncol);
  }
  a.front_total = a.front_off[nsn];
  // matrices: L_21 (nstr x ncol, column-major) and its transpose; the inverse
  // of the diagonal block (column-major) and its transpose
  a.l21.assign(a.l21_off[nsn], 0.0);
  a.l21t.assign(a.l21_off[nsn], 0.0);
  a.linv.assign(a.linv_off[nsn], 0.0);
  a.linvt.assign(a.linv_off[nsn], 0.0);
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    const int m = ncol + nstr;
    const double* P = &F.panel[F.panel_off[q]];
    for (int j = 0; j < ncol; ++j)
      for (int t = 0; t < nstr; ++t) {
        const double v = P[(size_t)j * m + ncol + t];
        a.l21[a.l21_off[q] + (long)j * nstr + t] = v;
        a.l21t[a.l21_off[q] + (long)t * ncol + j] = v;
      }
    // Z = L_ss^-1 column by column, by forward substitution on e_c
    double* Z = &a.linv[a.linv_off[q]];
    for (int c = 0; c < ncol; ++c)
      for (int i = c; i < ncol; ++i) {
        double acc = i == c ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) acc -= P[(size_t)k * m + i] * Z[(size_t)c * ncol + k];
        Z[(size_t)c * ncol + i] = acc / P[(size_t)i * m + i];
      }
    double* ZT = &a.linvt[a.linv_off[q]];
    for (int c = 0; c < ncol; ++c)
      for (int i = 0; i < ncol; ++i) ZT[(size_t)i * ncol + c] = Z[(size_t)c * ncol + i];
  }
  // front gathers: per front entry, the child update entries that land there
  // (in child order), fr_k slots per entry
  {
    std::vector<std::vector<int>> src(a.front_total);
    for (int q = 0; q < nsn; ++q)
      for (int qc = F.child_off[q]; qc < F.child_off[q + 1]; ++qc) {
        const int c = F.child_idx[qc];
        for (int t = F.str_off[c]; t < F.str_off[c + 1]; ++t) src[a.front_off[q] + F.map[t]].push_back(t);
      }
    a.fr_k = 1;
    for (const auto& v : src) a.fr_k = std::max(a.fr_k, (int)v.size());
    a.fr_src.assign((size_t)a.front_total * a.fr_k, -1);
    for (int64_t k = 0; k < a.front_total; ++k)
      for (size_t e = 0; e < src[k].size(); ++e) a.fr_src[(size_t)k * a.fr_k + e] = src[k][e];
  }
  // bottom subtrees: supernodes whose subtree spans at most `cap` columns;
  // each maximal one is a subtree, its supernodes listed by height.  n / 96
  // (about 128 subtrees of a nested dissection): measured against n / 12 to
  // n / 192 on the level-5 and level-6 spheres, the fastest 64-right-hand-side
  // Laplacian solve at both levels (0.38 and 1.37 ms against 0.50 and 2.10 at
  // n / 48) and the fastest G_ll solve at level 6; with the staged bottom
  // steps still the fastest Laplacian solve at level 5 (349 us against 364 at
  // n / 48 and 408 at n / 192)
  const int cap = std::max(128, n / 96);
  std::vector<int> first(nsn);  // first column of each supernode's subtree
  for (int q = 0; q < nsn; ++q) {
    first[q] = F.col0[q];
    for (int qc = F.child_off[q]; qc < F.child_off[q + 1]; ++qc) first[q] = std::min(first[q], first[F.child_idx[qc]]);
  }
  // a bottom subtree holds staged supernodes only (children come first)
  std::vector<char> bottom(nsn, 0);
  for (int q = 0; q < nsn; ++q) {
    bottom[q] = F.col0[q + 1] - first[q] <= cap &&
                sp_staged(F.col0[q + 1] - F.col0[q], F.str_off[q + 1] - F.str_off[q], a.fr_k);
    for (int qc = F.child_off[q]; qc < F.child_off[q + 1]; ++qc) bottom[q] = bottom[q] && bottom[F.child_idx[qc]];
  }
  a.sub_ptr.assign(1, 0);
  a.sub_lvl.clear();
  a.sub_nodes.clear();
  a.bot_lds = 0;
  a.bot_fac = 0;
  a.bot_idx = 0;
  a.bot_ncol = 0;
  auto lds_need = [&](int p) {
    const int ncol = F.col0[p + 1] - F.col0[p], nstr = F.str_off[p + 1] - F.str_off[p];
    return 2 * ncol + nstr;
  };
  // a bottom supernode's slice: its front (per right-hand side), its blocks
  // and its gather indices
  auto bottom_need = [&](int p) {
    const int ncol = F.col0[p + 1] - F.col0[p], nstr = F.str_off[p + 1] - F.str_off[p];
    a.bot_lds = std::max(a.bot_lds, ncol + nstr);
    a.bot_ncol = std::max(a.bot_ncol, ncol);
    a.bot_fac = std::max(a.bot_fac, (ncol * (ncol + nstr) + 1) / 2 * 2);
    a.bot_idx = std::max(a.bot_idx, ((ncol + nstr) * a.fr_k + 3) / 4 * 4);
  };
  int nsub = 0;
  for (int q = 0; q < nsn; ++q) {
    if (!bottom[q] || (F.parent[q] >= 0 && bottom[F.parent[q]])) continue;
    // q roots a subtree: its supernodes are those in q's column range
    std::vector<int> members;
    for (int p = 0; p <= q; ++p)
      if (F.col0[p] >= first[q] && F.col0[p + 1] <= F.col0[q + 1]) members.push_back(p);
    int hmax = 0;
    for (int p : members) hmax = std::max(hmax, F.height[p]);
    a.sub_lvl.push_back((int)a.sub_nodes.size());
    for (int h = 0; h <= hmax; ++h) {
      for (int p : members)
        if (F.height[p] == h) {
          a.sub_nodes.push_back(p);
          bottom_need(p);
        }
      a.sub_lvl.push_back((int)a.sub_nodes.size());
    }
    a.sub_ptr.push_back((int)a.sub_lvl.size());
    ++nsub;
  }
  a.nsub = nsub;
  // the staged bottom supernodes' blocks, L_ss^-1 then L_21 contiguously
  a.blk_off.assign(nsn, 0);
  a.blk.clear();
  for (int p : a.sub_nodes) {
    a.blk_off[p] = (long)a.blk.size();
    a.blk.insert(a.blk.end(), a.linv.begin() + a.linv_off[p], a.linv.begin() + a.linv_off[p + 1]);
    a.blk.insert(a.blk.end(), a.l21.begin() + a.l21_off[p], a.l21.begin() + a.l21_off[p + 1]);
  }
  // per bottom position, the supernode's columns, struct rows, front and
  // blocks: {col0, ncol, str_off, nstr}, {front_off, blk_off, 0, 0}
  a.sub_desc.clear();
  for (int p : a.sub_nodes) {
    const int ncol = F.col0[p + 1] - F.col0[p], nstr = F.str_off[p + 1] - F.str_off[p];
    a.sub_desc.insert(a.sub_desc.end(),
                      {F.col0[p], ncol, F.str_off[p], nstr, (int)a.front_off[p], (int)a.blk_off[p], 0, 0});
  }
  // top supernodes by height
  int H = 0;
  for (int q = 0; q < nsn; ++q)
    if (!bottom[q]) H = std::max(H, F.height[q]);
  std::vector<std::vector<int>> by_h(H + 1);
  for (int q = 0; q < nsn; ++q)
    if (!bottom[q]) by_h[F.height[q]].push_back(q);
  a.top_lvl.assign(1, 0);
  a.top_nodes.clear();
  a.top_count.clear();
  a.top_lds.clear();
  for (int h = 0; h <= H; ++h) {
    if (by_h[h].empty()) continue;
    int need = 0;
    for (int q : by_h[h]) {
      a.top_nodes.push_back(q);
      need = std::max(need, lds_need(q));
    }
    a.top_count.push_back((int)by_h[h].size());
    a.top_lds.push_back(need);
    a.top_lvl.push_back((int)a.top_nodes.size());
  }
  a.ntop = (int)a.top_lvl.size() - 1;
  a.top_roots = true;
  if (a.ntop > 0)
    for (int k = a.top_lvl[a.ntop - 1]; k < a.top_lvl[a.ntop]; ++k)
      a.top_roots = a.top_roots && F.str_off[a.top_nodes[k] + 1] == F.str_off[a.top_nodes[k]];
  // per top position, the supernode's descriptor {col0, ncol, str_off, nstr},
  // {front_off, linv_off, l21_off, 0}
  a.top_desc.clear();
  for (int p : a.top_nodes) {
    const int ncol = F.col0[p + 1] - F.col0[p], nstr = F.str_off[p + 1] - F.str_off[p];
    a.top_desc.insert(a.top_desc.end(), {F.col0[p], ncol, F.str_off[p], nstr, (int)a.front_off[p],
                                         (int)a.linv_off[p], (int)a.l21_off[p], 0});
  }
  a.iperm.assign(n, 0);
  for (int i = 0; i < n; ++i) a.iperm[F.perm[i]] = i;
}

rfcmp_status spchol_upload(const SpFactor& F, SpDevice& D, hipStream_t s) {
  const int n = F.n, nsn = F.nsn;
  SpArrays a;
  spchol_arrays(F, a);
  if (a.blk.size() > (size_t)INT32_MAX || a.front_total > INT32_MAX || a.linv_off[nsn] > INT32_MAX ||
      a.l21_off[nsn] > INT32_MAX) {
    set_error("spchol_upload: factor blocks beyond 32-bit offsets");
    return RFCMP_E_ARG;
  }
  D.n = n;
  D.nsn = nsn;
  D.grounded = F.grounded ? 1 : 0;
  D.max_front = F.max_front;
  D.max_ncol = a.max_ncol;
  D.nsub = a.nsub;
  D.ntop = a.ntop;
  D.bot_lds = a.bot_lds;
  D.bot_fac = a.bot_fac;
  D.bot_idx = a.bot_idx;
  D.bot_ncol = a.bot_ncol;
  D.top_roots = a.top_roots;
  D.fr_k = a.fr_k;
  D.top_count = a.top_count;
  D.top_lds = a.top_lds;
  D.seconds = F.seconds;
  D.nstr_total = F.str_off[nsn];
  D.front_total = a.front_total;
  D.nnz = (int64_t)(a.l21.size() + a.l21t.size() + a.linv.size() + a.linvt.size() + a.blk.size());
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> rfcmp_status {
    RF_TRY(b.alloc(std::max<size_t>(bytes, 16)));
    if (bytes) RF_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return RFCMP_OK;
  };
  auto upv = [&](DevBuf& b, const auto& v) { return up(b, v.data(), sizeof(v[0]) * v.size()); };
  RF_TRY(upv(D.perm, F.perm));
  RF_TRY(upv(D.iperm, a.iperm));
  RF_TRY(upv(D.col0, F.col0));
  RF_TRY(upv(D.str_off, F.str_off));
  RF_TRY(upv(D.str, F.str));
  RF_TRY(upv(D.front_off, a.front_off));
  RF_TRY(upv(D.fr_src, a.fr_src));
  RF_TRY(upv(D.linv_off, a.linv_off));
  RF_TRY(upv(D.l21_off, a.l21_off));
  RF_TRY(upv(D.blk_off, a.blk_off));
  RF_TRY(upv(D.blk, a.blk));
  RF_TRY(upv(D.l21, a.l21));
  RF_TRY(upv(D.l21t, a.l21t));
  RF_TRY(upv(D.linv, a.linv));
  RF_TRY(upv(D.linvt, a.linvt));
  RF_TRY(upv(D.sub_ptr, a.sub_ptr));
  RF_TRY(upv(D.sub_lvl, a.sub_lvl));
  RF_TRY(upv(D.sub_desc, a.sub_desc));
  RF_TRY(upv(D.top_desc, a.top_desc));
  D.top_start = a.top_lvl;
  // the host arrays above are locals: wait for the copies
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

// Leaf size of the dissection: measured on the level-4 and level-5 spheres
// (16: about 1.3 and 6 MB for L; 64 stores three times the entries of 8).
constexpr int kSpLeaf = 16;

HostFactor factor_mesh_matrix(const MeshHost& h, int which) {
  HostFactor r;
  try {
    SpMatrix A;
    if (which == 0)
      laplacian_matrix(h, A);
    else if (which == 1)
      gram_ll_matrix(h, A);
    else
      gram_tp_matrix(h, A);
    r.F = std::make_shared<SpFactor>();
    r.status = spchol_factor(A, which == 0, kSpLeaf, 1, *r.F);
    if (r.status < 0) r.error = last_error();
  } catch (const std::bad_alloc&) {
    r.status = RFCMP_E_OOM;
    r.error = "host allocation failed in the sparse factorisation";
  }
  return r;
}

rfcmp_status mesh_sparse_projectors(rfcmp_mesh m, bool need_gtp) {
  MeshDev& d = m->d;
  const int nq = need_gtp ? 3 : 2;
  bool todo = false;
  for (int q = 0; q < nq; ++q) todo |= !d.sp[q];
  if (!todo) return RFCMP_OK;
  if (!d.proj_stream[0]) {
    RF_HIP(hipStreamCreateWithFlags(&d.proj_stream[0], hipStreamNonBlocking));
    RF_HIP(hipEventCreateWithFlags(&d.proj_done[0], hipEventDisableTiming));
  }
  for (int q = 0; q < nq; ++q) {
    if (d.sp[q]) continue;
    HostFactor hf;
    if (q < 2 && m->fac_async[q].valid()) {
      hf = m->fac_async[q].get();
    } else {
      if (q == 2) build_cell_nb(m->h);
      hf = factor_mesh_matrix(m->h, q);
    }
    if (hf.status < 0) {
      set_error("%s", hf.error.c_str());
      return hf.status;
    }
    auto dev = std::make_unique<SpDevice>();
    RF_TRY(spchol_upload(*hf.F, *dev, d.proj_stream[0]));
    d.sp[q] = std::move(dev);
  }
  return RFCMP_OK;
}

}  // namespace rfcmp
