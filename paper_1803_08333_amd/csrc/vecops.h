// Launch wrappers of the sparse incidence products and fused vector steps.
#pragma once

#include "internal.h"

namespace rfcmp {

// t = Sigma^T x  (N -> C)
rfcmp_status sigma_t(const MeshDev& d, int64_t C, int64_t N, const double2* x, double2* t, int nr, hipStream_t s);
// g = Lambda^T x  (N -> V)
rfcmp_status lambda_t(const MeshDev& d, int64_t V, int64_t N, const double2* x, double2* g, int nr, hipStream_t s);
// out = Lambda h  (V -> N)
rfcmp_status lambda_n(const MeshDev& d, int64_t N, int64_t V, const double2* h, double2* out, int nr, hipStream_t s);
// out = ca*x (times i if ca_imag; x nullable) + cs * Sigma z
rfcmp_status axpy_sigma(const MeshDev& d, int64_t N, int64_t C, double ca, bool ca_imag, const double2* x,
                        double cs, const double2* z, double2* out, int nr, hipStream_t s);
// out1 = [area .*] (fa a + fb (b - mean b)), out2 = f2 (out1 - mean out1), the
// means formed in the same launch (area, a, b, out2 nullable)
rfcmp_status comb_mean(int64_t C, const double* area, double fa, const double2* a, double fb, const double2* b,
                       double2* out1, double f2, double2* out2, int nr, hipStream_t s);
// y = -i ka (zA - Sigma s4) + Sigma g6
rfcmp_status left_y(const MeshDev& d, int64_t N, int64_t C, double ka, const double2* zA, const double2* s4,
                    const double2* g6, double2* y, int nr, hipStream_t s);
// jl = ia (x - Sigma sv), js = i ib Sigma sg (the two parts of recover_j)
rfcmp_status recover_j_split(const MeshDev& d, int64_t N, int64_t C, double ia, double ib, const double2* x,
                             const double2* sv, const double2* sg, double2* jl, double2* js, int nr, hipStream_t s);
// j = ia (x - Sigma sv) + i ib Sigma sg
rfcmp_status recover_j(const MeshDev& d, int64_t N, int64_t C, double ia, double ib, const double2* x,
                       const double2* sv, const double2* sg, double2* j, int nr, hipStream_t s);
// out[r] = sum conj(a[r]) b[r]; part needs dot_partials()*nr entries.  The
// real parts also go to re_out[r] and host_out[r] when those are non-null
// (host_out: the device address of mapped pinned host memory).
rfcmp_status dot(int64_t n, const double2* a, const double2* b, double2* part, double2* out, int nr,
                 hipStream_t s, double* re_out = nullptr, double* host_out = nullptr);
int dot_partials();
// out[r] = x[r] / |x[r]|, nrm2[r] = |x[r]|^2 (one launch)
rfcmp_status normalize_rows(int64_t n, const double2* x, double2* out, double2* nrm2, int nr, hipStream_t s);
// Rows 0, 1: w_r - Sigma z5_r; row 2: Sigma z10; normalised into out [3][N],
// squared norms into nrm2 [3].
rfcmp_status power_next(const MeshDev& d, int64_t N, int64_t C, const double2* w, const double2* z5,
                        const double2* z10, double2* out, double2* nrm2, hipStream_t s);
// power iteration: out[0] = Lambda h, out[1] = a[1] - Sigma z  (h [V], z [C], a and out [2][N])
rfcmp_status power_branch(const MeshDev& d, int64_t N, int64_t V, int64_t C, const double2* h, const double2* a,
                          const double2* z, double2* out, hipStream_t s);
// out[r] = x[r] / sqrt(re nrm2[r])
rfcmp_status normalize(int64_t n, const double2* nrm2, const double2* x, double2* out, int nr, hipStream_t s);
// block CG updates over nr right-hand sides (frozen where active[r] == 0)
rfcmp_status cg_xr_blk(int64_t n, int nr, const double* rho, const double* pq, const int* active, double2* x,
                       double2* r, const double2* p, const double2* q, hipStream_t s);
rfcmp_status cg_p_blk(int64_t n, int nr, const double* rnew, const double* rold, const int* active,
                      const double2* r, double2* p, hipStream_t s);
rfcmp_status take_real_n(const double2* d, double* out, int nr, hipStream_t s);
rfcmp_status set_active(int* a, int v, int n, hipStream_t s);
rfcmp_status vsub(int64_t n, const double2* a, const double2* b, double2* out, hipStream_t s);
rfcmp_status vadd_to(int64_t n, const double2* a, double2* x, hipStream_t s);

}  // namespace rfcmp
