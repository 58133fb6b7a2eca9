// BF16x3 split-precision matrix products on MFMA (see gemm.hip).
#pragma once

#include "internal.h"

namespace rfcmp {

// A matrix stored as bf16 hi/lo planes (four for complex, two for real).
struct SplitMatrix {
  int64_t n = 0, rows_pad = 0, kpad = 0;
  bool cplx = false;
  DevBuf planes;
  // tri > 0: M symmetric, stored as the upper triangle of tri-wide blocks.
  rfcmp_status from_c64(const float2* M, int64_t n, int64_t ld, int64_t tri, hipStream_t s);
  rfcmp_status from_f64(const double* M, int64_t n, int64_t ld, hipStream_t s);
};

// Bytes of scratch gemm_bf16x3 needs for an n x n matrix and nrhs columns.
size_t gemm_scratch_bytes(int64_t n, int nrhs);

// Y[r] = M X[r] (or conj(M) X[r]) for r < nrhs; X, Y complex128 [nrhs][n].
rfcmp_status gemm_bf16x3(const SplitMatrix& M, bool conj_m, const double2* X, double2* Y, int nrhs,
                         void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag);

// FP64-accumulated complex products Y = M X (conj: conj(M) X) of a complex64
// n x n matrix stored whole (row-major, ld a multiple of 4) with complex128
// X, Y [nrhs][n], on the FP64 matrix cores (zgemm.hip): for many right-hand
// sides, where they are bound by FP64 arithmetic.  Deterministic.
size_t zgemm_scratch_bytes(int64_t n);
rfcmp_status zgemm_c64(const float2* M, int64_t n, int64_t ld, bool conj, const double2* X, double2* Y, int nrhs,
                       void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag);
// Right-hand sides from which the complex64 products take zgemm_c64 instead
// of the symmetric streaming product.
constexpr int kZgemmMinRhs = 8;

}  // namespace rfcmp
