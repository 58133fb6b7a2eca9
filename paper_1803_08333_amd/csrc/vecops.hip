// Sparse incidence products and fused vector steps of the RF-CMP operator.
//
// Sigma and Lambda have two non-zeros per row (Sec. 2): Sigma^T x and
// Lambda^T x are short gathers, Sigma z and Lambda h are differences of two
// entries.  Each fused kernel below evaluates one line of the
// cancellation-free application on complex128 vectors; nrhs runs in
// blockIdx.y, vectors are [nrhs][n] contiguous.
#include "vecops.h"

namespace rfcmp {

namespace {

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// multiply by i*s
__device__ inline double2 cimul(double s, double2 a) { return make_double2(-s * a.y, s * a.x); }

__global__ void k_sigma_t(int C, int N, const int* __restrict__ cell_edge, const float* __restrict__ sgn,
                          const double2* __restrict__ x, double2* __restrict__ t) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const long r = blockIdx.y;
  const double2* xr = x + r * N;
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 v = xr[cell_edge[3 * c + i]];
    const double g = sgn[3 * c + i];
    s.x += g * v.x;
    s.y += g * v.y;
  }
  t[r * C + c] = s;
}

__global__ void k_lambda_t(int V, int N, const int* __restrict__ ptr, const int* __restrict__ idx,
                           const float* __restrict__ sg, const double2* __restrict__ x,
                           double2* __restrict__ g) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const long r = blockIdx.y;
  const double2* xr = x + r * N;
  double2 s = make_double2(0.0, 0.0);
  for (int q = ptr[v]; q < ptr[v + 1]; ++q) {
    const double2 e = xr[idx[q]];
    s.x += sg[q] * e.x;
    s.y += sg[q] * e.y;
  }
  g[r * V + v] = s;
}

// out[n] = ca*x[n] + cs*(z[c+] - z[c-])  (real ca, complex-by-real cs, with
// optional multiplication of the first term by i)
__global__ void k_axpy_sigma(int N, int C, const int* __restrict__ edge_cell, double ca, int ca_imag,
                             const double2* __restrict__ x, double cs, const double2* __restrict__ z,
                             double2* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long r = blockIdx.y;
  const double2 zd = csub(z[r * C + edge_cell[2 * n]], z[r * C + edge_cell[2 * n + 1]]);
  double2 a = x ? x[r * N + n] : make_double2(0.0, 0.0);
  a = ca_imag ? cimul(ca, a) : cscale(ca, a);
  out[r * N + n] = cadd(a, cscale(cs, zd));
}

// Sum over the workgroup (1024 threads), fixed-order tree; every thread gets the result.
// Sum over the 1024 threads of a workgroup, returned to every thread: an
// xor butterfly inside each wave (every lane ends with the same bits), then
// the 16 wave sums in wave order.  sr, si: LDS of at least 16 doubles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
__device__ double2 block_sum_1024(double ar, double ai, double* sr, double* si) {
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x / 64] = ar;
    si[threadIdx.x / 64] = ai;
  }
  __syncthreads();
  double tr = 0.0, ti = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    tr += sr[q];
    ti += si[q];
  }
  __syncthreads();  // sr/si may be reused
  return make_double2(tr, ti);
}

// out1[c] = [A_c] (fa a[c] + fb (b[c] - mean b));  out2[c] = f2 (out1[c] - mean out1)
// (area, a, b, out2 nullable).  One workgroup per right-hand side, so the
// means need no second launch.  Up to kCombRegs entries per thread are kept
// in registers between the passes (one round trip to memory); longer rows
// revisit the entries each thread wrote.
constexpr int kCombRegs = 8;
__global__ __launch_bounds__(1024) void k_comb_mean(int C, const double* __restrict__ area, double fa,
                                                    const double2* __restrict__ a, double fb,
                                                    const double2* __restrict__ b, double2* __restrict__ out1,
                                                    double f2, double2* __restrict__ out2) {
  __shared__ double sr[16], si[16];
  const long r = blockIdx.x;
  const int t = threadIdx.x;
  if (C <= kCombRegs * 1024) {
    double2 av[kCombRegs], bv[kCombRegs];
    double wv[kCombRegs];
    double br = 0.0, bi = 0.0;
#pragma unroll
    for (int u = 0; u < kCombRegs; ++u) {
      const int i = t + 1024 * u;
      const bool in = i < C;
      av[u] = (a && in) ? a[r * C + i] : make_double2(0.0, 0.0);
      bv[u] = (b && in) ? b[r * C + i] : make_double2(0.0, 0.0);
      wv[u] = (area && in) ? area[i] : 1.0;
      br += bv[u].x;
      bi += bv[u].y;
    }
    double2 mb = make_double2(0.0, 0.0);
    if (b) {
      const double2 tb = block_sum_1024(br, bi, sr, si);
      mb = make_double2(tb.x / C, tb.y / C);
    }
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int u = 0; u < kCombRegs; ++u) {
      const int i = t + 1024 * u;
      double2 v = cscale(fa, av[u]);
      if (b) v = cadd(v, cscale(fb, csub(bv[u], mb)));
      v = cscale(wv[u], v);
      av[u] = v;
      if (i < C) {
        out1[r * C + i] = v;
        ar += v.x;
        ai += v.y;
      }
    }
    if (!out2) return;
    const double2 to = block_sum_1024(ar, ai, sr, si);
    const double2 m1 = make_double2(to.x / C, to.y / C);
#pragma unroll
    for (int u = 0; u < kCombRegs; ++u) {
      const int i = t + 1024 * u;
      if (i < C) out2[r * C + i] = cscale(f2, csub(av[u], m1));
    }
    return;
  }
  double2 mb = make_double2(0.0, 0.0);
  if (b) {
    double br = 0.0, bi = 0.0;
    for (int i = t; i < C; i += 1024) {
      br += b[r * C + i].x;
      bi += b[r * C + i].y;
    }
    const double2 tb = block_sum_1024(br, bi, sr, si);
    mb = make_double2(tb.x / C, tb.y / C);
  }
  double ar = 0.0, ai = 0.0;
  for (int i = t; i < C; i += 1024) {
    double2 v = a ? cscale(fa, a[r * C + i]) : make_double2(0.0, 0.0);
    if (b) v = cadd(v, cscale(fb, csub(b[r * C + i], mb)));
    if (area) v = cscale(area[i], v);
    out1[r * C + i] = v;
    ar += v.x;
    ai += v.y;
  }
  if (!out2) return;
  const double2 to = block_sum_1024(ar, ai, sr, si);
  const double2 m1 = make_double2(to.x / C, to.y / C);
  for (int i = t; i < C; i += 1024) out2[r * C + i] = cscale(f2, csub(out1[r * C + i], m1));
}

// y = -(ik/alpha)(zA - Sigma s4) + Sigma g6
__global__ void k_left_y(int N, int C, const int* __restrict__ edge_cell, double ka,
                         const double2* __restrict__ zA, const double2* __restrict__ s4,
                         const double2* __restrict__ g6, double2* __restrict__ y) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long r = blockIdx.y;
  const int cp = edge_cell[2 * n], cm = edge_cell[2 * n + 1];
  const double2 pl = csub(zA[r * N + n], csub(s4[r * C + cp], s4[r * C + cm]));
  y[r * N + n] = cadd(cimul(-ka, pl), csub(g6[r * C + cp], g6[r * C + cm]));
}

// j = (i - Sigma s)/alpha + i (Sigma sg)/beta
__global__ void k_recover(int N, int C, const int* __restrict__ edge_cell, double ia, double ib,
                          const double2* __restrict__ x, const double2* __restrict__ s,
                          const double2* __restrict__ sg, double2* __restrict__ j) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long r = blockIdx.y;
  const int cp = edge_cell[2 * n], cm = edge_cell[2 * n + 1];
  const double2 ps = csub(s[r * C + cp], s[r * C + cm]);
  const double2 pg = csub(sg[r * C + cp], sg[r * C + cm]);
  j[r * N + n] = cadd(cscale(ia, csub(x[r * N + n], ps)), cimul(ib, pg));
}

// the two parts of k_recover apart: jl = ia (x - Sigma s), js = i ib Sigma sg
__global__ void k_recover_split(int N, int C, const int* __restrict__ edge_cell, double ia, double ib,
                                const double2* __restrict__ x, const double2* __restrict__ s,
                                const double2* __restrict__ sg, double2* __restrict__ jl,
                                double2* __restrict__ js) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long r = blockIdx.y;
  const int cp = edge_cell[2 * n], cm = edge_cell[2 * n + 1];
  const double2 ps = csub(s[r * C + cp], s[r * C + cm]);
  const double2 pg = csub(sg[r * C + cp], sg[r * C + cm]);
  jl[r * N + n] = cscale(ia, csub(x[r * N + n], ps));
  js[r * N + n] = cimul(ib, pg);
}

// out = Lambda h (n from the vertex differences)
__global__ void k_lambda(int N, int V, const int* __restrict__ edge_vtx, const double2* __restrict__ h,
                         double2* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const long r = blockIdx.y;
  out[r * N + n] = csub(h[r * V + edge_vtx[2 * n]], h[r * V + edge_vtx[2 * n + 1]]);
}

// Power-iteration branches: out[0] = Lambda h (V -> N), out[1] = a[1] - Sigma z
// (h and z single vectors, a two rows).
__global__ void k_power_branch(int N, int V, int C, const int* __restrict__ edge_vtx,
                               const int* __restrict__ edge_cell, const double2* __restrict__ h,
                               const double2* __restrict__ a, const double2* __restrict__ z,
                               double2* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  out[n] = csub(h[edge_vtx[2 * n]], h[edge_vtx[2 * n + 1]]);
  out[(long)N + n] = csub(a[(long)N + n], csub(z[edge_cell[2 * n]], z[edge_cell[2 * n + 1]]));
}

// ---------------------------------------------------------------- reductions
constexpr int kRedBlocks = 240;

// partial[b][r] = sum_{i in block b} conj(a[r][i]) b[r][i]
__global__ __launch_bounds__(256) void k_dot_partial(long n, const double2* __restrict__ a,
                                                     const double2* __restrict__ b,
                                                     double2* __restrict__ part) {
  __shared__ double sr[256], si[256];
  const long r = blockIdx.y;
  double ar = 0.0, ai = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double2 x = a[r * n + i], y = b[r * n + i];
    ar += x.x * y.x + x.y * y.y;
    ai += x.x * y.y - x.y * y.x;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[r * gridDim.x + blockIdx.x] = make_double2(sr[0], si[0]);
}

__global__ __launch_bounds__(256) void k_dot_final(int nb, const double2* __restrict__ part,
                                                   double2* __restrict__ out, double* __restrict__ re_out,
                                                   double* __restrict__ host_out) {
  __shared__ double sr[256], si[256];
  const long r = blockIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    ar += part[r * nb + i].x;
    ai += part[r * nb + i].y;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[r] = make_double2(sr[0], si[0]);
    if (re_out) re_out[r] = sr[0];
    if (host_out) host_out[r] = sr[0];
  }
}

// out[r] = sum_i conj(a[r][i]) b[r][i] in one workgroup per row (rows up
// to kDotOneBlock entries): strided per thread, then block_sum_1024.
constexpr long kDotOneBlock = 1L << 16;
__global__ __launch_bounds__(1024) void k_dot_rows(long n, const double2* __restrict__ a,
                                                   const double2* __restrict__ b, double2* __restrict__ out,
                                                   double* __restrict__ re_out, double* __restrict__ host_out) {
  __shared__ double sr[16], si[16];
  const long r = blockIdx.x;
  double ar = 0.0, ai = 0.0;
#pragma unroll 4
  for (long i = threadIdx.x; i < n; i += 1024) {
    const double2 x = a[r * n + i], y = b[r * n + i];
    ar += x.x * y.x + x.y * y.y;
    ai += x.x * y.y - x.y * y.x;
  }
  const double2 t = block_sum_1024(ar, ai, sr, si);
  if (threadIdx.x == 0) {
    out[r] = t;
    if (re_out) re_out[r] = t.x;
    if (host_out) host_out[r] = t.x;
  }
}

// x[r] *= 1/sqrt(re(nrm2[r]))
__global__ void k_normalize(long n, const double2* __restrict__ nrm2, const double2* __restrict__ x,
                            double2* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long r = blockIdx.y;
  const double s = 1.0 / sqrt(nrm2[r].x);
  out[r * n + i] = cscale(s, x[r * n + i]);
}

// out[r] = x[r] / |x[r]|_2 and nrm2[r] = |x[r]|^2, one workgroup per row
// (fixed-order sum: strided per thread, then a tree).
__global__ __launch_bounds__(1024) void k_normalize_rows(long n, const double2* __restrict__ x,
                                                         double2* __restrict__ out, double2* __restrict__ nrm2) {
  __shared__ double sr[16], si[16];
  const long r = blockIdx.x;
  double a = 0.0;
  for (long i = threadIdx.x; i < n; i += 1024) {
    const double2 v = x[r * n + i];
    a += v.x * v.x + v.y * v.y;
  }
  const double2 t = block_sum_1024(a, 0.0, sr, si);
  const double sc = 1.0 / sqrt(t.x);
  if (threadIdx.x == 0) nrm2[r] = make_double2(t.x, 0.0);
  for (long i = threadIdx.x; i < n; i += 1024) out[r * n + i] = cscale(sc, x[r * n + i]);
}

// End of one power-iteration application: the three raw vectors (rows 0
// and 1: w_r - Sigma z5_r, row 2: Sigma z10), each row's squared norm to
// nrm2[r], and the row divided by its norm to out.  One workgroup per row.
// Rows of up to kPowRegs * 1024 entries stay in registers between the norm
// and the scaling, with every thread's loads issued together (the edge's two
// cells, then the gathers); longer rows are written, then rescaled by the
// threads that wrote them.
constexpr int kPowRegs = 8;
__global__ __launch_bounds__(1024) void k_power_next(int N, int C, const int* __restrict__ edge_cell,
                                                     const double2* __restrict__ w, const double2* __restrict__ z5,
                                                     const double2* __restrict__ z10, double2* __restrict__ out,
                                                     double2* __restrict__ nrm2) {
  __shared__ double sr[16], si[16];
  const int r = blockIdx.x;
  double2* o = out + (long)r * N;
  const double2* z = r < 2 ? z5 + (long)r * C : z10;
  double a = 0.0;
  if (N <= kPowRegs * 1024) {
    int2 cells[kPowRegs];
    double2 v[kPowRegs];
#pragma unroll
    for (int u = 0; u < kPowRegs; ++u) {
      const int n = threadIdx.x + 1024 * u;
      cells[u] = n < N ? reinterpret_cast<const int2*>(edge_cell)[n] : make_int2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kPowRegs; ++u) {
      const int n = threadIdx.x + 1024 * u;
      if (n < N) {
        const double2 zd = csub(z[cells[u].x], z[cells[u].y]);
        v[u] = r < 2 ? csub(w[(long)r * N + n], zd) : zd;
        a += v[u].x * v[u].x + v[u].y * v[u].y;
      }
    }
    const double2 t = block_sum_1024(a, 0.0, sr, si);
    const double sc = 1.0 / sqrt(t.x);
    if (threadIdx.x == 0) nrm2[r] = make_double2(t.x, 0.0);
#pragma unroll
    for (int u = 0; u < kPowRegs; ++u) {
      const int n = threadIdx.x + 1024 * u;
      if (n < N) o[n] = cscale(sc, v[u]);
    }
    return;
  }
  for (int n = threadIdx.x; n < N; n += 1024) {
    const double2 zd = csub(z[edge_cell[2 * n]], z[edge_cell[2 * n + 1]]);
    const double2 v = r < 2 ? csub(w[(long)r * N + n], zd) : zd;
    o[n] = v;
    a += v.x * v.x + v.y * v.y;
  }
  const double2 t = block_sum_1024(a, 0.0, sr, si);
  const double sc = 1.0 / sqrt(t.x);
  if (threadIdx.x == 0) nrm2[r] = make_double2(t.x, 0.0);
  for (int n = threadIdx.x; n < N; n += 1024) o[n] = cscale(sc, o[n]);
}

__global__ void k_sub(long n, const double2* __restrict__ a, const double2* __restrict__ b,
                      double2* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = csub(a[i], b[i]);
}
__global__ void k_add_to(long n, const double2* __restrict__ a, double2* __restrict__ x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = cadd(x[i], a[i]);
}

// block CG: alpha_r = rho_r/pq_r for active r; x_r += alpha p_r; r_r -= alpha q_r
__global__ void k_cg_xr_blk(long n, const double* __restrict__ rho, const double* __restrict__ pq,
                            const int* __restrict__ active, double2* __restrict__ x, double2* __restrict__ r,
                            const double2* __restrict__ p, const double2* __restrict__ q) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = blockIdx.y;
  if (!active[k]) return;
  const double al = rho[k] / pq[k];
  const long o = (long)k * n + i;
  x[o] = cadd(x[o], cscale(al, p[o]));
  r[o] = csub(r[o], cscale(al, q[o]));
}
// block CG: p_r = r_r + (rho_new/rho_old) p_r for active r
__global__ void k_cg_p_blk(long n, const double* __restrict__ rnew, const double* __restrict__ rold,
                           const int* __restrict__ active, const double2* __restrict__ r, double2* __restrict__ p) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = blockIdx.y;
  if (!active[k]) return;
  const long o = (long)k * n + i;
  p[o] = cadd(r[o], cscale(rnew[k] / rold[k], p[o]));
}
__global__ void k_take_real_n(int nr, const double2* __restrict__ d, double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k < nr) out[k] = d[k].x;
}
__global__ void k_set_int(int* __restrict__ a, int v, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = v;
}

inline dim3 g1(long n, int nr = 1) { return dim3(unsigned((n + 255) / 256), unsigned(nr)); }

}  // namespace

#define RF_LAUNCH_CHECK() RF_HIP(hipGetLastError())

rfcmp_status sigma_t(const MeshDev& d, int64_t C, int64_t N, const double2* x, double2* t, int nr,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_sigma_t, g1(C, nr), dim3(256), 0, s, (int)C, (int)N, d.cell_edge.as<int>(),
                     d.sgn.as<float>(), x, t);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status lambda_t(const MeshDev& d, int64_t V, int64_t N, const double2* x, double2* g, int nr,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_lambda_t, g1(V, nr), dim3(256), 0, s, (int)V, (int)N, d.ve_ptr.as<int>(),
                     d.ve_idx.as<int>(), d.ve_sgn.as<float>(), x, g);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status lambda_n(const MeshDev& d, int64_t N, int64_t V, const double2* h, double2* out, int nr,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, g1(N, nr), dim3(256), 0, s, (int)N, (int)V, d.edge_vtx.as<int>(), h, out);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status axpy_sigma(const MeshDev& d, int64_t N, int64_t C, double ca, bool ca_imag, const double2* x,
                        double cs, const double2* z, double2* out, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_sigma, g1(N, nr), dim3(256), 0, s, (int)N, (int)C, d.edge_cell.as<int>(), ca,
                     (int)ca_imag, x, cs, z, out);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status comb_mean(int64_t C, const double* area, double fa, const double2* a, double fb, const double2* b,
                       double2* out1, double f2, double2* out2, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_comb_mean, dim3(nr), dim3(1024), 0, s, (int)C, area, fa, a, fb, b, out1, f2, out2);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}
rfcmp_status left_y(const MeshDev& d, int64_t N, int64_t C, double ka, const double2* zA, const double2* s4,
                    const double2* g6, double2* y, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_left_y, g1(N, nr), dim3(256), 0, s, (int)N, (int)C, d.edge_cell.as<int>(), ka, zA, s4,
                     g6, y);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status recover_j(const MeshDev& d, int64_t N, int64_t C, double ia, double ib, const double2* x,
                       const double2* sv, const double2* sg, double2* j, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_recover, g1(N, nr), dim3(256), 0, s, (int)N, (int)C, d.edge_cell.as<int>(), ia, ib, x,
                     sv, sg, j);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status recover_j_split(const MeshDev& d, int64_t N, int64_t C, double ia, double ib, const double2* x,
                             const double2* sv, const double2* sg, double2* jl, double2* js, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_recover_split, g1(N, nr), dim3(256), 0, s, (int)N, (int)C, d.edge_cell.as<int>(), ia, ib, x,
                     sv, sg, jl, js);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status dot(int64_t n, const double2* a, const double2* b, double2* part, double2* out, int nr,
                 hipStream_t s, double* re_out, double* host_out) {
  if (n <= kDotOneBlock) {
    hipLaunchKernelGGL(k_dot_rows, dim3(nr), dim3(1024), 0, s, (long)n, a, b, out, re_out, host_out);
  } else {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks, nr), dim3(256), 0, s, (long)n, a, b, part);
    hipLaunchKernelGGL(k_dot_final, dim3(nr), dim3(256), 0, s, kRedBlocks, part, out, re_out, host_out);
  }
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
int dot_partials() { return kRedBlocks; }
rfcmp_status normalize_rows(int64_t n, const double2* x, double2* out, double2* nrm2, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize_rows, dim3(nr), dim3(1024), 0, s, (long)n, x, out, nrm2);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}
rfcmp_status power_next(const MeshDev& d, int64_t N, int64_t C, const double2* w, const double2* z5,
                        const double2* z10, double2* out, double2* nrm2, hipStream_t s) {
  hipLaunchKernelGGL(k_power_next, dim3(3), dim3(1024), 0, s, (int)N, (int)C, d.edge_cell.as<int>(), w, z5, z10,
                     out, nrm2);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}
rfcmp_status power_branch(const MeshDev& d, int64_t N, int64_t V, int64_t C, const double2* h, const double2* a,
                          const double2* z, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_power_branch, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, (int)N, (int)V, (int)C,
                     d.edge_vtx.as<int>(), d.edge_cell.as<int>(), h, a, z, out);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}
rfcmp_status normalize(int64_t n, const double2* nrm2, const double2* x, double2* out, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, g1(n, nr), dim3(256), 0, s, (long)n, nrm2, x, out);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status cg_xr_blk(int64_t n, int nr, const double* rho, const double* pq, const int* active, double2* x,
                       double2* r, const double2* p, const double2* q, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xr_blk, g1(n, nr), dim3(256), 0, s, (long)n, rho, pq, active, x, r, p, q);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status cg_p_blk(int64_t n, int nr, const double* rnew, const double* rold, const int* active,
                      const double2* r, double2* p, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p_blk, g1(n, nr), dim3(256), 0, s, (long)n, rnew, rold, active, r, p);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status take_real_n(const double2* d, double* out, int nr, hipStream_t s) {
  hipLaunchKernelGGL(k_take_real_n, dim3(1), dim3(256), 0, s, nr, d, out);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status set_active(int* a, int v, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3((n + 255) / 256), dim3(256), 0, s, a, v, n);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status vsub(int64_t n, const double2* a, const double2* b, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, g1(n), dim3(256), 0, s, (long)n, a, b, out);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}
rfcmp_status vadd_to(int64_t n, const double2* a, double2* x, hipStream_t s) {
  hipLaunchKernelGGL(k_add_to, g1(n), dim3(256), 0, s, (long)n, a, x);
  RF_LAUNCH_CHECK();
  return RFCMP_OK;
}

}  // namespace rfcmp
