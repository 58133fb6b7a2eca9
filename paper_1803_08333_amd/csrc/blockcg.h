// Tall-skinny complex products of the block CG (rfcmp.hip): Gram matrices of
// blocks of columns and updates of a block by a small matrix, complex128
// throughout, fixed summation order.  A block of a columns of length N is
// stored column after column ([a][N], as every batch of vectors here).
#pragma once

#include "internal.h"

namespace rfcmp {

constexpr int kBlockMax = 64;  // largest block width

// Device scratch of gram_c128.
size_t gram_scratch_bytes(int64_t N);

// C[i][j] = sum_n conj(X[i][n]) Y[j][n], i < a, j < b (a, b <= kBlockMax);
// C: device complex128 [a][b].
rfcmp_status gram_c128(const double2* X, int a, const double2* Y, int b, int64_t N, double2* C, void* scratch,
                       size_t scratch_bytes, hipStream_t s);

// Y[c][n] = sgn sum_l X[l][n] S[l][c] (+ Y[c][n] when accumulate), c < ncol,
// l < a (a, ncol <= kBlockMax); S: device complex128 [a][ncol]; Y may not
// alias X.
rfcmp_status tsmm_c128(const double2* X, int a, const double2* S, int ncol, int64_t N, double2* Y, double sgn,
                       bool accumulate, hipStream_t s);

}  // namespace rfcmp
