// BF16x3 split-precision products on the gfx950 matrix cores (MFMA), for
// many right-hand sides at once:  Y = M X,  M complex (or real) n x K,
// X complex128 [nrhs][K].
//
// Split precision (Henry, Tang, Heinecke, "Leveraging the bfloat16 artificial
// intelligence datatype for higher-precision computations", ARITH 2019):
// every operand v is stored as hi = bf16(v), lo = bf16(v - hi), and a product
// a b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo lo term, 2^-18
// relative, is dropped), accumulated in FP32 by the MFMA.  The relative error
// of a product is ~2^-16, so these products serve inner iterations whose
// residual is recomputed with the FP64-accumulated complex64 product.
//
// Storage: a complex matrix is four bf16 planes (Re hi, Re lo, Im hi, Im lo),
// 8 bytes per entry -- the same as complex64; a real matrix two planes.
// Planes hold rows_pad x kpad entries (rows_pad and kpad multiples of 128,
// zero-padded) fragment-major: 32 x 32 tiles in which each wave's MFMA
// operand for one K-step is 1 KB contiguous, so the matrix stream is read
// in whole 1 KB wave loads.  X is split per call into two planes
// [ncp][kpad] (column 2r + 0/1 = Re/Im of right-hand side r; ncp = 2 nrhs
// rounded up to 32, at most 128).
//
// Kernel: a workgroup (4 waves) owns 128 rows and all ncp columns over one
// slice of K (split-K to about one workgroup per compute unit).  Each wave
// computes 32 rows with v_mfma_f32_32x32x16_bf16; the X tile of a 64-wide K
// chunk is staged in LDS (two buffers), and the next chunk's matrix rows and
// X are loaded while the current one is multiplied.
// Within a chunk, lane l of a wave covers k = 32 (l / 32) + 8 s + e for
// sub-step s and element e on both operands (the contraction order is free),
// so each lane reads 64 contiguous bytes of its matrix row.  Partial sums go
// to an FP32 buffer [slice][plane][rows_pad][ncp]; a combine kernel adds the
// slices in a fixed order in FP64 and forms the complex result.
#include "hmat.h"
#include "internal.h"
#include "gemm.h"
#include "spchol.h"

namespace rfcmp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16;

constexpr int kRowsWG = 128;
constexpr int kKpad = 128;       // K padding of the planes (and of the K slices: 4 chunks)
constexpr int kKc = 32;          // K chunk per pipeline stage
constexpr int kSub = kKc / 16;   // MFMA K-steps per chunk
constexpr int kLdsK = kKc + 8;   // padded column stride in LDS (bf16 units)

__device__ inline u16 bf16_bits(float x) {
  const __bf16 h = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(u16, h);
}
__device__ inline float bf16_val(u16 b) { return (float)__builtin_bit_cast(__bf16, b); }

// Offset of matrix entry (i, k) in a plane stored fragment-major: 32-row x
// 32-k tiles, each [s][lane][8] so that one wave's MFMA operand for one
// K-step is 1 KB contiguous (lane l: row l % 32, k = 16 (l / 32) + 8 s + e).
__device__ inline long frag_offset(long i, long k, long nkc) {
  const long rb = i >> 5, li = i & 31, kc = k >> 5, kk = k & 31;
  const long lane = li + 32 * (kk >> 4), sub = (kk >> 3) & 1, e = kk & 7;
  return (((rb * nkc + kc) * 2 + sub) * 64 + lane) * 8 + e;
}

// complex64 [n][ld] -> planes [4][rows_pad x kpad], fragment-major.  tri > 0
// (a multiple of 32): M is symmetric and only its entries with
// k >= tri floor(i / tri) are stored; the others are read transposed.  One
// 32 x 32 tile (32 rows, one 32-wide K chunk: one 1024-entry fragment per
// plane) per workgroup: the entries staged in LDS, read along k, or for a
// tile below the stored triangle as the stored transposed tile, read along
// i; then each plane's fragment written contiguously, 4 entries per thread.
__global__ __launch_bounds__(256) void k_split_c64(const float2* __restrict__ M, long n, long ld, long tri,
                                                   u16* __restrict__ P, long rows_pad, long kpad) {
  __shared__ float2 t[32][33];  // [row][k] of the tile
  const long kc = blockIdx.x, rb = blockIdx.y;
  const long i0 = rb * 32, k0 = kc * 32;
  const bool lower = tri > 0 && k0 < (i0 / tri) * tri;
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int a = e >> 5, b = e & 31;
    if (!lower) {
      const long i = i0 + a, k = k0 + b;
      t[a][b] = (i < n && k < n) ? M[i * ld + k] : make_float2(0.f, 0.f);
    } else {
      const long k = k0 + a, i = i0 + b;
      t[b][a] = (i < n && k < n) ? M[k * ld + i] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  // fragment entry f: sub f / 512, lane (f / 8) % 64, e f % 8, i.e. row
  // lane % 32 and k = 16 (lane / 32) + 8 sub + e of the tile (frag_offset)
  const long plane = rows_pad * kpad;
  const long base = (rb * (kpad / 32) + kc) * 1024;
  const int f0 = threadIdx.x * 4;
  typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
  u16x4 rh, rl, ih, il;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = f0 + j;
    const int sub = f >> 9, lane = (f >> 3) & 63, e = f & 7;
    const float2 v = t[lane & 31][16 * (lane >> 5) + 8 * sub + e];
    const u16 a = bf16_bits(v.x), c = bf16_bits(v.y);
    rh[j] = a;
    rl[j] = bf16_bits(v.x - bf16_val(a));
    ih[j] = c;
    il[j] = bf16_bits(v.y - bf16_val(c));
  }
  *reinterpret_cast<u16x4*>(P + base + f0) = rh;
  *reinterpret_cast<u16x4*>(P + plane + base + f0) = rl;
  *reinterpret_cast<u16x4*>(P + 2 * plane + base + f0) = ih;
  *reinterpret_cast<u16x4*>(P + 3 * plane + base + f0) = il;
}

// real FP64 [n][ld] -> planes [2][rows_pad x kpad], fragment-major
__global__ void k_split_f64(const double* __restrict__ M, long n, long ld, u16* __restrict__ P, long rows_pad,
                            long kpad) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows_pad * kpad) return;
  const long i = t / kpad, k = t % kpad;
  const float v = (i < n && k < n) ? (float)M[i * ld + k] : 0.f;
  const long o = frag_offset(i, k, kpad / 32);
  const u16 h = bf16_bits(v);
  P[o] = h;
  P[rows_pad * kpad + o] = bf16_bits(v - bf16_val(h));
}

// X complex128 [nrhs][K] -> planes [2][ncp][kpad], column 2r + part
__global__ void k_split_x(const double2* __restrict__ X, int nrhs, long K, u16* __restrict__ P, int ncp,
                          long kpad, int conj_x) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)ncp * kpad) return;
  const long col = t / kpad, k = t % kpad;
  const long r = col / 2;
  float v = 0.f;
  if (r < nrhs && k < K) {
    const double2 x = X[r * K + k];
    v = (col & 1) ? (float)(conj_x ? -x.y : x.y) : (float)x.x;
  }
  const u16 h = bf16_bits(v);
  P[t] = h;
  P[(long)ncp * kpad + t] = bf16_bits(v - bf16_val(h));
}

template <int NCT, bool CPLX>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const u16* __restrict__ A, long rows_pad, long kpad,
                                                     const u16* __restrict__ Xs, int ncp, long kslice,
                                                     float* __restrict__ part) {
  constexpr int NPL = CPLX ? 2 : 1;             // matrix planes pairs (Re, Im)
  constexpr int XW = 2 * NCT * 32 * (kKc / 8);  // 16-byte words of one staged X chunk (two planes)
  constexpr int XPT = XW / 256;                 // ... per thread
  static_assert(XW % 256 == 0 && kKc == 32, "chunk shape");
  __shared__ u16 bs[2][2][NCT * 32][kLdsK];  // [buffer][plane][column][k]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long row0 = (long)blockIdx.x * kRowsWG + wave * 32;
  const long k_begin = (long)blockIdx.y * kslice;
  const long k_end = min(kpad, k_begin + kslice);
  const int nch = (int)((k_end - k_begin) / kKc);
  const long plane = rows_pad * kpad;
  const long xplane = (long)ncp * kpad;
  const long nkc = kpad / kKc;

  f32x16 acc[NPL][NCT];
#pragma unroll
  for (int p = 0; p < NPL; ++p)
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[p][c][q] = 0.f;

  // fragment-major planes: this wave's operand for chunk kc, step s is the
  // 1 KB at ((rb nkc + kc) 2 + s) 512 elements; this lane's 16 bytes in it
  const u16* abase = A + ((row0 >> 5) * nkc + k_begin / kKc) * 2 * 512 + lane * 8;
  const int khalf = (lane >> 5) * (kKc / 2);

#define GEMM_LOAD_A(SET, CH)                                                                     \
  _Pragma("unroll") for (int p = 0; p < 2 * NPL; ++p)                                            \
    _Pragma("unroll") for (int s = 0; s < kSub; ++s)                                             \
      SET[p][s] = __builtin_nontemporal_load(                                                    \
          reinterpret_cast<const bf16x8*>(abase + p * plane + ((long)(CH) * 2 + s) * 512));
#define GEMM_LOAD_X(CH)                                                                          \
  _Pragma("unroll") for (int w = 0; w < XPT; ++w) {                                              \
    const int e = threadIdx.x + 256 * w;                                                         \
    const int pl = e / (NCT * 32 * (kKc / 8));                                                   \
    const int rem = e % (NCT * 32 * (kKc / 8));                                                  \
    const int col = rem / (kKc / 8), kk = (rem % (kKc / 8)) * 8;                                 \
    xr[w] = *reinterpret_cast<const bf16x8*>(Xs + pl * xplane + (long)col * kpad + k_begin +     \
                                             (long)(CH) * kKc + kk);                             \
  }
#define GEMM_STORE_X(BUF)                                                                        \
  _Pragma("unroll") for (int w = 0; w < XPT; ++w) {                                              \
    const int e = threadIdx.x + 256 * w;                                                         \
    const int pl = e / (NCT * 32 * (kKc / 8));                                                   \
    const int rem = e % (NCT * 32 * (kKc / 8));                                                  \
    const int col = rem / (kKc / 8), kk = (rem % (kKc / 8)) * 8;                                 \
    *reinterpret_cast<bf16x8*>(&bs[BUF][pl][col][kk]) = xr[w];                                   \
  }
#define GEMM_COMPUTE(SET, BUF)                                                                   \
  _Pragma("unroll") for (int s = 0; s < kSub; ++s) {                                             \
    bf16x8 bh[NCT], bl[NCT];                                                                     \
    _Pragma("unroll") for (int c = 0; c < NCT; ++c) {                                            \
      const int col = c * 32 + (lane & 31);                                                      \
      bh[c] = *reinterpret_cast<const bf16x8*>(&bs[BUF][0][col][khalf + 8 * s]);                 \
      bl[c] = *reinterpret_cast<const bf16x8*>(&bs[BUF][1][col][khalf + 8 * s]);                 \
    }                                                                                            \
    /* three passes (hi.hi, hi.lo, lo.hi), each over all accumulators, so    \
       consecutive MFMAs never wait on one another's accumulator */          \
    _Pragma("unroll") for (int p = 0; p < NPL; ++p)                                              \
      _Pragma("unroll") for (int c = 0; c < NCT; ++c)                                            \
        acc[p][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(SET[2 * p][s], bh[c], acc[p][c], 0, 0, 0);     \
    _Pragma("unroll") for (int p = 0; p < NPL; ++p)                                              \
      _Pragma("unroll") for (int c = 0; c < NCT; ++c)                                            \
        acc[p][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(SET[2 * p][s], bl[c], acc[p][c], 0, 0, 0);     \
    _Pragma("unroll") for (int p = 0; p < NPL; ++p)                                              \
      _Pragma("unroll") for (int c = 0; c < NCT; ++c)                                            \
        acc[p][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(SET[2 * p + 1][s], bh[c], acc[p][c], 0, 0, 0); \
  }

  // Pipeline over 32-wide K chunks: matrix operands four chunks deep in
  // registers (sets a0 .. a3 in rotation), X one chunk ahead in registers
  // and double-buffered in LDS; one barrier per chunk.  Within an
  // iteration X is loaded before the matrix rows, so waiting for X never
  // waits for the newest matrix loads.  The chunk count is a multiple of 4
  // (K slices of whole 128-wide blocks) and the loads past the last chunk
  // repeat the last one, so every iteration issues the same loads: the
  // compiler's wait counts then leave the three younger sets in flight
  // (with loads behind branches it waits for all of them at every chunk).
  bf16x8 a0[2 * NPL][kSub], a1[2 * NPL][kSub], a2[2 * NPL][kSub], a3[2 * NPL][kSub];
  bf16x8 xr[XPT];
  const int last = nch - 1;
  GEMM_LOAD_X(0)
  __builtin_amdgcn_sched_barrier(0);
  GEMM_LOAD_A(a0, 0)
  GEMM_LOAD_A(a1, min(1, last))
  GEMM_LOAD_A(a2, min(2, last))
  GEMM_LOAD_A(a3, min(3, last))
  GEMM_STORE_X(0)
  GEMM_LOAD_X(min(1, last))
  __syncthreads();
#define GEMM_STEP(SET, CH)                                                                       \
  {                                                                                              \
    const int buf = (CH) & 1;                                                                    \
    GEMM_COMPUTE(SET, buf)                                                                       \
    GEMM_STORE_X(buf ^ 1)                                                                        \
    GEMM_LOAD_X(min((CH) + 2, last))                                                             \
    __builtin_amdgcn_sched_barrier(0); /* X's loads stay ahead of the matrix rows' */            \
    GEMM_LOAD_A(SET, min((CH) + 4, last))                                                        \
    __syncthreads();                                                                             \
  }
  for (int ch = 0; ch < nch; ch += 4) {
    GEMM_STEP(a0, ch)
    GEMM_STEP(a1, ch + 1)
    GEMM_STEP(a2, ch + 2)
    GEMM_STEP(a3, ch + 3)
  }
#undef GEMM_STEP
#undef GEMM_COMPUTE
#undef GEMM_STORE_X
#undef GEMM_LOAD_X
#undef GEMM_LOAD_A
  // partial[slice][p][row][col]
#pragma unroll
  for (int p = 0; p < NPL; ++p)
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const long row = row0 + 8 * (q / 4) + (lane >> 5) * 4 + (q % 4);
        const int col = c * 32 + (lane & 31);
        part[(((long)blockIdx.y * NPL + p) * rows_pad + row) * ncp + col] = acc[p][c][q];
      }
}

// Y[r][i] from the slice partials (fixed summation order, FP64):
//   complex: re = P1[2r] - s P2[2r+1], im = P1[2r+1] + s P2[2r] (s = -1 for conj(M))
//   real:    re = P1[2r], im = P1[2r+1]
__global__ void k_gemm_combine(const float* __restrict__ part, int nslice, int npl, long rows_pad, int ncp,
                               long n, int nrhs, int conj_m, double2* __restrict__ Y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const long i = t % n, r = t / n;
  double p1r = 0, p1i = 0, p2r = 0, p2i = 0;
  for (int s = 0; s < nslice; ++s) {
    const float* b1 = part + (((long)s * npl + 0) * rows_pad + i) * ncp;
    p1r += b1[2 * r];
    p1i += b1[2 * r + 1];
    if (npl == 2) {
      const float* b2 = part + (((long)s * npl + 1) * rows_pad + i) * ncp;
      p2r += b2[2 * r];
      p2i += b2[2 * r + 1];
    }
  }
  const double sg = conj_m ? -1.0 : 1.0;
  Y[r * n + i] = make_double2(p1r - sg * p2i, p1i + sg * p2r);
}

}  // namespace

rfcmp_status SplitMatrix::from_c64(const float2* M, int64_t n_, int64_t ld, int64_t tri, hipStream_t s) {
  n = n_;
  cplx = true;
  rows_pad = (int64_t)round_up(n, kRowsWG);
  kpad = (int64_t)round_up(n, kKpad);
  if (tri % 32 != 0 || rows_pad / 32 > 65535) {
    set_error("split: tri = %lld (a multiple of 32), n = %lld", (long long)tri, (long long)n);
    return RFCMP_E_ARG;
  }
  RF_TRY(planes.alloc(sizeof(u16) * 4 * rows_pad * kpad));
  hipLaunchKernelGGL(k_split_c64, dim3((unsigned)(kpad / 32), (unsigned)(rows_pad / 32)), dim3(256), 0, s, M,
                     (long)n, (long)ld, (long)tri, planes.as<u16>(), (long)rows_pad, (long)kpad);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

rfcmp_status SplitMatrix::from_f64(const double* M, int64_t n_, int64_t ld, hipStream_t s) {
  n = n_;
  cplx = false;
  rows_pad = (int64_t)round_up(n, kRowsWG);
  kpad = (int64_t)round_up(n, kKpad);
  RF_TRY(planes.alloc(sizeof(u16) * 2 * rows_pad * kpad));
  const long tot = rows_pad * kpad;
  hipLaunchKernelGGL(k_split_f64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, (long)n, (long)ld,
                     planes.as<u16>(), (long)rows_pad, (long)kpad);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

size_t gemm_scratch_bytes(int64_t n, int nrhs) {
  const int64_t rows_pad = (int64_t)round_up(n, kRowsWG), kpad = (int64_t)round_up(n, kKpad);
  const int nr = std::min(nrhs, 64);
  const int ncp = (int)round_up(2 * nr, 32);
  return round_up(sizeof(u16) * 2 * ncp * kpad, 256) + sizeof(float) * 16 * 2 * rows_pad * ncp + 1024;
}

rfcmp_status gemm_bf16x3(const SplitMatrix& M, bool conj_m, const double2* X, double2* Y, int nrhs, void* scratch,
                         size_t scratch_bytes, hipStream_t s, const char* tag) {
  const int64_t n = M.n;
  for (int r0 = 0; r0 < nrhs; r0 += 64) {
    const int nr = std::min(64, nrhs - r0);
    const int ncp = (int)round_up(2 * nr, 32);
    const int nct = ncp / 32;
    const long nrb = (long)(M.rows_pad / kRowsWG);
    // split K so that the grid fills the compute units, one workgroup each
    // (the accumulators and two register sets of matrix rows fill the
    // register file): the fewest slices (at most 16) for which the last
    // round of workgroups keeps at least 90 % of the units busy, else the
    // fullest last round
    long nslice = 1;
    {
      double best = 0.0;
      for (long ns = 1; ns <= 16; ++ns) {
        const long wg = nrb * ns;
        const double fill = (double)wg / (256.0 * (double)((wg + 255) / 256));
        if (fill > best + 1e-9) {
          best = fill;
          nslice = ns;
        }
        if (fill >= 0.9) break;
      }
    }
    long kslice = (long)round_up((M.kpad + nslice - 1) / nslice, kKpad);
    nslice = (M.kpad + kslice - 1) / kslice;
    const int npl = M.cplx ? 2 : 1;
    const size_t xs_bytes = round_up(sizeof(u16) * 2 * ncp * M.kpad, 256);
    const size_t need = xs_bytes + sizeof(float) * nslice * npl * M.rows_pad * ncp;
    if (need > scratch_bytes) {
      set_error("gemm_bf16x3: scratch of %zu bytes too small (%zu needed)", scratch_bytes, need);
      return RFCMP_E_STATE;
    }
    u16* xs = static_cast<u16*>(scratch);
    float* part = reinterpret_cast<float*>(static_cast<char*>(scratch) + xs_bytes);
    ProfScope prof(tag, s);
    const long xt = (long)ncp * M.kpad;
    // conj(M) X = conj(M conj X) is handled in the combine; X is split as is
    hipLaunchKernelGGL(k_split_x, dim3((unsigned)((xt + 255) / 256)), dim3(256), 0, s, X + (long)r0 * n, nr,
                       (long)n, xs, ncp, (long)M.kpad, 0);
    dim3 grid((unsigned)nrb, (unsigned)nslice);
#define RF_GEMM(NCTV)                                                                                       \
  if (M.cplx)                                                                                              \
    hipLaunchKernelGGL((k_gemm_bf16x3<NCTV, true>), grid, dim3(256), 0, s, M.planes.as<u16>(),              \
                       (long)M.rows_pad, (long)M.kpad, xs, ncp, kslice, part);                              \
  else                                                                                                     \
    hipLaunchKernelGGL((k_gemm_bf16x3<NCTV, false>), grid, dim3(256), 0, s, M.planes.as<u16>(),             \
                       (long)M.rows_pad, (long)M.kpad, xs, ncp, kslice, part);
    switch (nct) {
      case 1: RF_GEMM(1) break;
      case 2: RF_GEMM(2) break;
      case 3: RF_GEMM(3) break;
      default: RF_GEMM(4) break;
    }
#undef RF_GEMM
    const long ot = (long)n * nr;
    hipLaunchKernelGGL(k_gemm_combine, dim3((unsigned)((ot + 255) / 256)), dim3(256), 0, s, part, (int)nslice, npl,
                       (long)M.rows_pad, ncp, (long)n, nr, conj_m ? 1 : 0, Y + (long)r0 * n);
    RF_HIP(hipGetLastError());
  }
  return RFCMP_OK;
}

MeshDev::MeshDev() = default;
MeshDev::~MeshDev() {
  for (int q = 0; q < 2; ++q) {
    if (proj_stream[q]) {
      (void)hipStreamSynchronize(proj_stream[q]);
      (void)hipStreamDestroy(proj_stream[q]);
    }
    if (proj_done[q]) (void)hipEventDestroy(proj_done[q]);
  }
  if (proj_start) (void)hipEventDestroy(proj_start);
}

}  // namespace rfcmp

rfcmp_op_s::rfcmp_op_s() = default;
rfcmp_op_s::~rfcmp_op_s() {
  if (host_scal) (void)hipHostFree(host_scal);
  if (bcg_host) (void)hipHostFree(bcg_host);
  for (int q = 0; q < 2; ++q)
    if (cg_exec[q]) (void)hipGraphExecDestroy(cg_exec[q]);
  if (cg_stream) {
    (void)hipStreamSynchronize(cg_stream);
    (void)hipStreamDestroy(cg_stream);
  }
}
