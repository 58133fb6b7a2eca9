// Complex products Y = M X (or conj(M) X) of a complex64 matrix stored whole
// with many complex128 right-hand sides, accumulated in FP64 on the FP64
// matrix cores (v_mfma_f64_16x16x4).  They serve the FP64-accumulated
// products of T_A and V (the refinement residual, the right-hand side, the
// FP32-path iterations) once there are enough right-hand sides that the
// products are bound by FP64 arithmetic rather than by the matrix stream:
// with 32 right-hand sides a pass does 192 flops per matrix entry (8 bytes),
// where the symmetric streaming product (symv.hip) can take 4.
//
// Three real products per complex one (Gauss): with M = Mr + i Mi and
// X = Xr + i Xi,
//   P1 = Mr Xr,  P2 = Mi Xi,  P3 = (Mr + Mi)(Xr + Xi),
//   Re Y = P1 - P2,  Im Y = P3 - P1 - P2,
// so 16 right-hand sides take three 16-column MFMA operands where the
// four-product form takes four.  In FP64 the extra rounding of the sums is
// of order 1e-16 relative to |M| |X|, far below the complex64 storage of M.
// A launch serves NG groups of 16 right-hand sides (NG = 2 from 17 on), so
// that each pass over the matrix does 3 NG MFMAs per K step.
//
// A workgroup (4 waves) owns 64 rows over one K slice; wave w takes rows
// 16 w .. 16 w + 15 (two waves fit a SIMD with 32 right-hand sides, three
// with 16; measured, one 16-row tile per wave beats two by a fifth: the
// occupancy matters more than the reuse of the X operands).  Per 32-column
// chunk each lane loads 8 consecutive complex64 entries of its row (64
// contiguous bytes: a wave reads 16 rows x 256 bytes), and MFMA step e uses
// entry e, so that the k index of lane l at step e is chunk column
// 8 (l / 16) + e; the X chunk sits in LDS in the same order, one 512-byte
// conflict-free wave read per operand.  Partial sums of the K slices go to a
// buffer [slice][32][n] (complex128); a second kernel adds the slices in
// order (the result does not depend on timing).
#include "internal.h"
#include "gemm.h"

namespace rfcmp {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float vf4 __attribute__((ext_vector_type(4)));

constexpr int kZThreads = 256;
constexpr int kZTiles = 1;                     // 16-row tiles per wave
constexpr int kZRowsWave = 16 * kZTiles;
constexpr int kZRows = 4 * kZRowsWave;         // rows per workgroup
constexpr int kZK = 32;                        // K chunk
constexpr int kZRhs = 32;                      // right-hand sides per launch (at most)

// lds[g][b][e][l]: operand b (0: Xr, 1: Xi, 2: Xr + Xi) of group g at step
// e for lane l (chunk column 8 (l / 16) + e, right-hand side 16 g + l % 16)
template <int NG>
struct ZStage {
  double v[NG][3][8][64];
};

// X chunk into the operand order.  The loads go to registers first
// (z_load_x, before the products of the current chunk) and to LDS after
// them (z_store_x).
template <int NG>
__device__ inline void z_load_x(double2 (&xr)[2 * NG], const double2* __restrict__ X, int n, int nr, int kc,
                                int k_end, int tid) {
#pragma unroll
  for (int u = 0; u < 2 * NG; ++u) {
    const int idx = tid + u * kZThreads;
    const int g = idx / 512, e = (idx / 64) % 8, ll = idx % 64;
    const int k = kc + 8 * (ll / 16) + e, r = 16 * g + ll % 16;
    xr[u] = (r < nr && k < k_end) ? X[(long)r * n + k] : make_double2(0.0, 0.0);
  }
}
template <int NG>
__device__ inline void z_store_x(ZStage<NG>& st, const double2 (&xr)[2 * NG], int tid) {
#pragma unroll
  for (int u = 0; u < 2 * NG; ++u) {
    const int idx = tid + u * kZThreads;
    const int g = idx / 512, e = (idx / 64) % 8, ll = idx % 64;
    st.v[g][0][e][ll] = xr[u].x;
    st.v[g][1][e][ll] = xr[u].y;
    st.v[g][2][e][ll] = xr[u].x + xr[u].y;
  }
}

// the matrix: 8 consecutive entries of each of the wave's four rows
__device__ inline void z_load_m(float2 (&av)[kZTiles][8], const float2* __restrict__ M, int n, long ld, int row0, int kc,
                                int k_end, int lane) {
  const int kq = kc + 8 * (lane >> 4);
#pragma unroll
  for (int a = 0; a < kZTiles; ++a) {
    const int row = row0 + 16 * a;
    const float2* src = M + (long)row * ld + kq;
    if (row < n && kq + 8 <= k_end) {
      const vf4* s4 = reinterpret_cast<const vf4*>(src);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const vf4 v = __builtin_nontemporal_load(s4 + e);
        av[a][2 * e] = make_float2(v.x, v.y);
        av[a][2 * e + 1] = make_float2(v.z, v.w);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) av[a][e] = (row < n && kq + e < k_end) ? src[e] : make_float2(0.f, 0.f);
    }
  }
}

template <bool CONJ, int NG>
__device__ inline void z_mfma(dbl4 (&acc)[kZTiles][NG][3], const float2 (&av)[kZTiles][8], const ZStage<NG>& st,
                              int lane) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    double xb[NG][3];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int b = 0; b < 3; ++b) xb[g][b] = st.v[g][b][e][lane];
    double mb[3][kZTiles];
#pragma unroll
    for (int a = 0; a < kZTiles; ++a) {
      mb[0][a] = (double)av[a][e].x;
      mb[1][a] = CONJ ? -(double)av[a][e].y : (double)av[a][e].y;
      mb[2][a] = mb[0][a] + mb[1][a];
    }
    // each accumulator is taken once per step, 3 NG kZTiles instructions apart
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < kZTiles; ++a)
#pragma unroll
        for (int g = 0; g < NG; ++g)
          acc[a][g][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(mb[b][a], xb[g][b], acc[a][g][b], 0, 0, 0);
  }
}

// Two chunks in flight: the loads of chunk c + 1 (matrix into registers, X
// into the other LDS stage) are issued before the products of chunk c.
template <bool CONJ, int NG>
__global__ __launch_bounds__(kZThreads) void k_zgemm(const float2* __restrict__ M, int n, long ld,
                                                     const double2* __restrict__ X, int nr, int kslice,
                                                     double2* __restrict__ part) {
  __shared__ ZStage<NG> st[2];
  const int rb = blockIdx.x, ks = blockIdx.y;
  const int k_begin = ks * kslice, k_end = min(n, k_begin + kslice);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int row0 = rb * kZRows + w * kZRowsWave + (lane & 15);
  dbl4 acc[kZTiles][NG][3];
#pragma unroll
  for (int a = 0; a < kZTiles; ++a)
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[a][g][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  float2 va[kZTiles][8], vb[kZTiles][8];
  double2 xr[2 * NG];
  z_load_m(va, M, n, ld, row0, k_begin, k_end, lane);
  z_load_x<NG>(xr, X, n, nr, k_begin, k_end, tid);
  z_store_x<NG>(st[0], xr, tid);
  __syncthreads();
  for (int kc = k_begin; kc < k_end; kc += 2 * kZK) {
    const int k1 = kc + kZK, k2 = kc + 2 * kZK;
    if (k1 < k_end) {
      z_load_m(vb, M, n, ld, row0, k1, k_end, lane);
      z_load_x<NG>(xr, X, n, nr, k1, k_end, tid);
    }
    z_mfma<CONJ, NG>(acc, va, st[0], lane);
    __builtin_amdgcn_sched_barrier(0);  // the X stores wait for their loads here, after the products
    if (k1 < k_end) z_store_x<NG>(st[1], xr, tid);
    __syncthreads();  // stage 1 written, stage 0 read
    if (k1 >= k_end) break;
    if (k2 < k_end) {
      z_load_m(va, M, n, ld, row0, k2, k_end, lane);
      z_load_x<NG>(xr, X, n, nr, k2, k_end, tid);
    }
    z_mfma<CONJ, NG>(acc, vb, st[1], lane);
    __builtin_amdgcn_sched_barrier(0);
    if (k2 < k_end) z_store_x<NG>(st[0], xr, tid);
    __syncthreads();  // stage 0 written, stage 1 read
  }
  // accumulator value v of lane l: row 4 v + l / 16 of the tile,
  // right-hand side 16 g + l % 16
  double2* pd = part + (long)ks * kZRhs * n;
#pragma unroll
  for (int a = 0; a < kZTiles; ++a)
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rb * kZRows + w * kZRowsWave + 16 * a + 4 * v + (lane >> 4);
        const int r = 16 * g + (lane & 15);
        const double p1 = acc[a][g][0][v], p2 = acc[a][g][1][v], p3 = acc[a][g][2][v];
        if (row < n && r < nr) pd[(long)r * n + row] = make_double2(p1 - p2, p3 - p1 - p2);
      }
}

// Y[r][i] = sum over the slices, in order, of part[s][r][i]
__global__ __launch_bounds__(256) void k_zgemm_sum(const double2* __restrict__ part, int n, int nr, int nslice,
                                                   double2* __restrict__ Y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nr * n) return;
  const int r = (int)(t / n), i = (int)(t % n);
  double2 s = make_double2(0.0, 0.0);
  for (int q = 0; q < nslice; ++q) {
    const double2 v = part[((long)q * kZRhs + r) * n + i];
    s.x += v.x;
    s.y += v.y;
  }
  Y[(long)r * n + i] = s;
}

// K slices of a launch: about 15 workgroups per compute unit (measured at
// n = 20480 and 30720 against 2-12 slices), at most 16 slices.
int zgemm_slices(int64_t n) {
  const int64_t rbs = (n + kZRows - 1) / kZRows;
  return (int)std::min<int64_t>(16, std::max<int64_t>(1, (3840 + rbs / 2) / rbs));
}

}  // namespace

size_t zgemm_scratch_bytes(int64_t n) { return sizeof(double2) * (size_t)zgemm_slices(n) * kZRhs * (size_t)n; }

rfcmp_status zgemm_c64(const float2* M, int64_t n, int64_t ld, bool conj, const double2* X, double2* Y, int nrhs,
                       void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag) {
  if (n <= 0 || nrhs <= 0) return RFCMP_OK;
  if (ld < n || ld % 4 != 0 || n > INT32_MAX / 2) {
    set_error("zgemm: n = %lld, ld = %lld (ld >= n, a multiple of 4)", (long long)n, (long long)ld);
    return RFCMP_E_ARG;
  }
  if (scratch_bytes < zgemm_scratch_bytes(n)) {
    set_error("zgemm: needs %zu bytes of scratch, %zu given", zgemm_scratch_bytes(n), scratch_bytes);
    return RFCMP_E_ARG;
  }
  const int ns = zgemm_slices(n);
  const int kslice = (int)(((n + ns - 1) / ns + kZK - 1) / kZK * kZK);
  const int nsl = (int)((n + kslice - 1) / kslice);
  const dim3 grid((unsigned)((n + kZRows - 1) / kZRows), (unsigned)nsl);
  double2* part = static_cast<double2*>(scratch);
  for (int r0 = 0; r0 < nrhs; r0 += kZRhs) {
    const int nr = std::min(kZRhs, nrhs - r0);
    ProfScope prof(profile_tag_suffix(tag, nr), s);
    auto kern = conj ? (nr > 16 ? k_zgemm<true, 2> : k_zgemm<true, 1>) : (nr > 16 ? k_zgemm<false, 2> : k_zgemm<false, 1>);
    hipLaunchKernelGGL(kern, grid, dim3(kZThreads), 0, s, M, (int)n, (long)ld, X + (long)r0 * n, nr, kslice, part);
    hipLaunchKernelGGL(k_zgemm_sum, dim3((unsigned)(((long)nr * n + 255) / 256)), dim3(256), 0, s, part, (int)n, nr,
                       nsl, Y + (long)r0 * n);
  }
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

}  // namespace rfcmp
