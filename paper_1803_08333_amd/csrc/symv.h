// Symmetric streaming products with fused input gathers (symv.hip).
#pragma once

#include "internal.h"

namespace rfcmp {

// How a product forms its input x[r][g], g < n, from vectors already in HBM.
// Every source vector is complex128 with a per-right-hand-side stride.  The
// gathers are the sparse incidence products of the operator (Sigma^T,
// Lambda^T) and two of its fused lines, so those never make a round trip
// through HBM of their own.
struct SymvInput {
  enum Mode : int {
    kPlain = 0,    // x = p0
    kSigmaT = 1,   // x = Sigma^T p0:  x[c] = sum_l sgn[c][l] p0[cell_edge[c][l]]
    kLambdaT = 2,  // x = Lambda^T p0: x[v] = sum over the edges e at v of sgn p0[e]
    kVin = 3,      // x = i c0 (p0 - Sigma p1) - c1 Sigma p2       (p0: N, p1/p2: C)
    kMiddleW = 4,  // x = c0 Lambda p0 + c1 (p1 - Sigma p2) + c2 Sigma p3   (p0: V, p1: N, p2/p3: C)
    kProjLH = 5,   // x = p0 - Sigma p1                                     (p0: N, p1: C)
  };
  int mode = kPlain;
  const double2* p[4] = {nullptr, nullptr, nullptr, nullptr};
  long stride[4] = {0, 0, 0, 0};
  double c[3] = {0.0, 0.0, 0.0};
  const int* idx0 = nullptr;   // cell_edge [C][3] | ve_ptr [V+1] | edge_cell [N][2] (c+, c-)
  const int* idx1 = nullptr;   // ve_idx | edge_vtx [N][2]
  const float* sgn = nullptr;  // cell sign [C][3] | ve_sgn
};

// One product y = M x of a symmetric M [n][ld] (complex64 or FP64).
struct SymvJob {
  const void* M = nullptr;
  int64_t n = 0, ld = 0;
  SymvInput in;
  double2* y = nullptr;  // [nrhs][n]
  int nrhs = 0;          // job 1 of a pair: 1 of 2 right-hand sides, or 0 = all
};

// Bytes of scratch one job of size n needs (partial sums, up to 4
// right-hand sides per pass); jobs launched together need the sum.
size_t symv_scratch_bytes(int64_t n, int nrhs);

// y = M x for one or two jobs in one launch (same element type and
// conjugation), nrhs right-hand sides.  Calls sharing a scratch must not
// overlap.  tag names the launch for the kernel timers.
rfcmp_status csymv_jobs(const SymvJob* jobs, int njobs, bool conj, int nrhs, void* scratch, size_t scratch_bytes,
                        hipStream_t s, const char* tag);
rfcmp_status dsymv_jobs(const SymvJob* jobs, int njobs, int nrhs, void* scratch, size_t scratch_bytes,
                        hipStream_t s, const char* tag);

// out[r][g] = x[r][g] of the input, g < n (for the products that need the
// input in HBM: the BF16x3 GEMM).
rfcmp_status symv_form_input(const SymvInput& in, int64_t n, int nrhs, double2* out, hipStream_t s);

// Plain single products (input read as is).
rfcmp_status csymv(const float2* M, int64_t n, int64_t ld, bool conj, const double2* x, double2* y, int nrhs,
                   void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag = "csymv");
rfcmp_status dsymv(const double* M, int64_t n, int64_t ld, const double2* x, double2* y, int nrhs,
                   void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag = "dsymv");

}  // namespace rfcmp
