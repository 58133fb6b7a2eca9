// Tall-skinny complex products of the block CG (see blockcg.h).
//
// Gram: a fixed grid of workgroups, each summing its rows in chunks of 32
// (both blocks staged in LDS, rows fastest, so a wave reads its X entry as a
// broadcast and neighbouring lanes neighbouring Y entries), thread t owning
// the outputs (i, j) = (t / 64 + 4 q, t % 64); the partials of the
// workgroups are added in a fixed order by a second kernel.
// Update: one thread per row and group of 8 output columns, the small
// matrix in LDS.
#include "blockcg.h"

namespace rfcmp {
namespace {

constexpr int kGramRows = 32;
constexpr int kGramGroups = 240;  // workgroups of the first pass (fixed: the sum order does not depend on N)

__global__ __launch_bounds__(256) void k_gram_part(const double2* __restrict__ X, int a, const double2* __restrict__ Y,
                                                   int b, long N, double2* __restrict__ part) {
  __shared__ double2 sX[kGramRows][kBlockMax];
  __shared__ double2 sY[kGramRows][kBlockMax];
  const int tid = threadIdx.x;
  const int j = tid % 64;
  double cr[16], ci[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) cr[q] = ci[q] = 0.0;
  const long per = (N + gridDim.x - 1) / gridDim.x;
  const long n0 = (long)blockIdx.x * per, n1 = min(N, n0 + per);
  for (long c0 = n0; c0 < n1; c0 += kGramRows) {
    const int nr = (int)min((long)kGramRows, n1 - c0);
    for (int e = tid; e < kGramRows * kBlockMax; e += 256) {
      const int col = e / kGramRows, rr = e % kGramRows;
      sX[rr][col] = (col < a && rr < nr) ? X[(long)col * N + c0 + rr] : make_double2(0.0, 0.0);
      sY[rr][col] = (col < b && rr < nr) ? Y[(long)col * N + c0 + rr] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double2 y = sY[rr][j];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double2 x = sX[rr][tid / 64 + 4 * q];
        cr[q] += x.x * y.x + x.y * y.y;
        ci[q] += x.x * y.y - x.y * y.x;
      }
    }
    __syncthreads();
  }
  double2* out = part + (long)blockIdx.x * kBlockMax * kBlockMax;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = tid / 64 + 4 * q;
    out[i * kBlockMax + j] = make_double2(cr[q], ci[q]);
  }
}

// One wave per output: lane l adds the partials of workgroups l, l + 64, ...
// in order, then the lanes are combined by a fixed butterfly (lane 0's
// value is stored).
__global__ __launch_bounds__(256) void k_gram_sum(int a, int b, int groups, const double2* __restrict__ part,
                                                  double2* __restrict__ C) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= a * b) return;
  const int i = o / b, j = o % b;
  double sr = 0.0, si = 0.0;
  for (int g = lane; g < groups; g += 64) {
    const double2 v = part[(long)g * kBlockMax * kBlockMax + i * kBlockMax + j];
    sr += v.x;
    si += v.y;
  }
  for (int m = 32; m > 0; m >>= 1) {
    sr += __shfl_xor(sr, m);
    si += __shfl_xor(si, m);
  }
  if (lane == 0) C[o] = make_double2(sr, si);
}

constexpr int kTsmmCols = 8;

__global__ __launch_bounds__(256) void k_tsmm(const double2* __restrict__ X, int a, const double2* __restrict__ S,
                                              int ncol, long N, double2* __restrict__ Y, double sgn, int accumulate) {
  __shared__ double2 sS[kBlockMax][kTsmmCols];
  const int c0 = blockIdx.y * kTsmmCols;
  for (int e = threadIdx.x; e < kBlockMax * kTsmmCols; e += 256) {
    const int l = e / kTsmmCols, c = e % kTsmmCols;
    sS[l][c] = (l < a && c0 + c < ncol) ? S[l * ncol + c0 + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const long n = (long)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double yr[kTsmmCols], yi[kTsmmCols];
#pragma unroll
  for (int c = 0; c < kTsmmCols; ++c) yr[c] = yi[c] = 0.0;
  for (int l = 0; l < a; ++l) {
    const double2 x = X[(long)l * N + n];
#pragma unroll
    for (int c = 0; c < kTsmmCols; ++c) {
      const double2 s = sS[l][c];
      yr[c] += x.x * s.x - x.y * s.y;
      yi[c] += x.x * s.y + x.y * s.x;
    }
  }
#pragma unroll
  for (int c = 0; c < kTsmmCols; ++c) {
    if (c0 + c >= ncol) break;
    double2* yp = Y + (long)(c0 + c) * N + n;
    double2 v = make_double2(sgn * yr[c], sgn * yi[c]);
    if (accumulate) {
      const double2 o = *yp;
      v.x += o.x;
      v.y += o.y;
    }
    *yp = v;
  }
}

}  // namespace

size_t gram_scratch_bytes(int64_t) { return sizeof(double2) * (size_t)kGramGroups * kBlockMax * kBlockMax; }

rfcmp_status gram_c128(const double2* X, int a, const double2* Y, int b, int64_t N, double2* C, void* scratch,
                       size_t scratch_bytes, hipStream_t s) {
  if (a <= 0 || b <= 0 || a > kBlockMax || b > kBlockMax || N <= 0) {
    set_error("gram_c128: bad sizes a %d b %d N %lld", a, b, (long long)N);
    return RFCMP_E_ARG;
  }
  if (scratch_bytes < gram_scratch_bytes(N)) {
    set_error("gram_c128: scratch too small");
    return RFCMP_E_STATE;
  }
  double2* part = static_cast<double2*>(scratch);
  ProfScope prof("block_gram", s);
  hipLaunchKernelGGL(k_gram_part, dim3(kGramGroups), dim3(256), 0, s, X, a, Y, b, (long)N, part);
  hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)((a * b + 3) / 4)), dim3(256), 0, s, a, b, kGramGroups, part, C);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

rfcmp_status tsmm_c128(const double2* X, int a, const double2* S, int ncol, int64_t N, double2* Y, double sgn,
                       bool accumulate, hipStream_t s) {
  if (a < 0 || ncol <= 0 || a > kBlockMax || ncol > kBlockMax || N <= 0) {
    set_error("tsmm_c128: bad sizes a %d ncol %d N %lld", a, ncol, (long long)N);
    return RFCMP_E_ARG;
  }
  ProfScope prof("block_update", s);
  hipLaunchKernelGGL(k_tsmm, dim3((unsigned)((N + 255) / 256), (unsigned)((ncol + kTsmmCols - 1) / kTsmmCols)),
                     dim3(256), 0, s, X, a, S, ncol, (long)N, Y, sgn, accumulate ? 1 : 0);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

}  // namespace rfcmp
