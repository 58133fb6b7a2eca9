// The RF-CMP operator, its right-hand side, recovery, scalings and CG solve,
// and the C ABI.
//
// System (Sec. 3, eq. NewFormulation; scalings of Sec. 4):
//   A = P_o^H T^H P_m T P_o,  b = -P_o^H T^H P_m e,  j = P_o i,
//   P_o = P_LH/alpha + i P_s/beta,  P_m = Lam G_ll^-1 Lam^T/alpha^2 + P_LH/gamma
//         + Sig L^+ G_pp^-1 L^+ Sig^T/beta^2,  T = i k T_A + Sig V Sig^T/(i k),
// T^H x = conj(T conj x) (Sec. 3.4).  Application order (every product that
// vanishes identically is left out, so no O(1/k) term meets an O(k) one):
//   t1 = Sig^T x, s1 = L^+ t1                    u_S = Sig s1 (P_Sigma) or Sig L^+ G_tp^-1 t1
//   a  = T_A((ik/alpha) u_L - (k/beta) u_S),     vphi = V Sig^T u_S
//   s2 = L^+ Sig^T a,  h = G_ll^-1 Lam^T a
//   t4 = diag(A) (s2 + (vphi - mean vphi)/(k beta)),  s3 = L^+ t4
//   w  = Lam h/alpha^2 + (a - Sig s2)/gamma + Sig s3/beta^2,  Sig^T w_S = (t4 - mean t4)/beta^2
//   zA = conj(T_A) w,  vw = conj(V) Sig^T w_S,  s4 = L^+ Sig^T zA
//   y  = -(ik/alpha)(zA - Sig s4) + Sig G6 [-(k/beta) s4 + (vw - mean vw)/(k beta)]
// with G6 = I for P_Sigma and G_tp^-1 for P_gSigma.  Uses L^+ L = I - 1 1^T/C
// and Sig^T P_LH = 0, Sig^T Lam = 0.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstring>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>

#include "blockcg.h"
#include "gemm.h"
#include "hmat.h"
#include "spchol.h"
#include "symv.h"
#include "vecops.h"

namespace rfcmp {
const char* last_error();

namespace {

// projector option values; the automatic choice takes the sparse factors
// where the dense inverse's cubic set-up dominates (above 12288 cells: 0.36 s
// at 20480 against 29 ms), the dense inverses below, where one streaming pass
// (22 us at 5120 cells) beats a sparse solve (about 0.25 ms)
constexpr int kProjAuto = 0, kProjSparse = 1, kProjDense = 2;
constexpr int64_t kAutoSparseCells = 12288;

// ------------------------------------------------------------------ workspace
// Complex128 scratch of one operator for R right-hand sides per pass.
struct Work {
  int R = 0;
  double2 *nA, *nB, *nC, *nD;        // [R][N]
  double2* c[14];                    // [R][C]
  double2 *v1, *v2;                  // [R][V]
  double2 *part, *dout;              // reductions
  double2 *x, *r, *p, *q, *b, *d, *b0;  // block CG vectors [R][N]
  double2 *pv, *pw;                  // power iteration [3][N]
  double2 *xN, *xC, *xV;             // formed product inputs for the BF16x3 path [R][N|C|V]
  double *rho, *pq;                  // device CG scalars: rho[2][R], pq[R]
  int* active;                       // [R]
};

size_t work_doubles2(int64_t N, int64_t C, int64_t V, int R) {
  return (size_t)(4 * R * N + 14 * R * C + 2 * R * V + (dot_partials() + 1) * R + 7 * R * N + 6 * N +
                  2 * R + 2 * R + R * (N + C + V));
}

Work carve(rfcmp_op op) {
  const MeshHost& h = op->mesh->h;
  const int64_t N = h.N, C = h.C, V = h.V;
  const int R = op->work_nrhs;
  double2* p = op->work.as<double2>();
  Work w;
  w.R = R;
  auto take = [&](int64_t n) {
    double2* q = p;
    p += n;
    return q;
  };
  w.nA = take(R * N); w.nB = take(R * N); w.nC = take(R * N); w.nD = take(R * N);
  for (auto& c : w.c) c = take(R * C);
  w.v1 = take(R * V); w.v2 = take(R * V);
  w.part = take((int64_t)dot_partials() * R);
  w.dout = take(R);
  w.x = take(R * N); w.r = take(R * N); w.p = take(R * N); w.q = take(R * N); w.b = take(R * N); w.d = take(R * N);
  w.b0 = take(R * N);
  w.pv = take(3 * N); w.pw = take(3 * N);
  w.xN = take(R * N); w.xC = take(R * C); w.xV = take(R * V);
  w.rho = reinterpret_cast<double*>(take(R));     // 2R doubles
  w.pq = reinterpret_cast<double*>(take(R / 2 + 1));
  w.active = reinterpret_cast<int*>(take(R / 4 + 1));
  return w;
}

// Scratch of the sparse projector solves for the workspace's right-hand
// sides: one region per factor of the mesh (L, G_ll, G_tp), so that the two
// solves of a paired launch never share one.  Sized once the factors exist.
rfcmp_status ensure_sp_scratch(rfcmp_op op) {
  if (op->opt.projector != kProjSparse) return RFCMP_OK;
  const MeshDev& d = op->mesh->d;
  int64_t off[3] = {0, 0, 0}, total = 0;
  for (int q = 0; q < 3; ++q) {
    off[q] = total;
    if (d.sp[q]) total += (int64_t)op->work_nrhs * d.sp[q]->scratch_entries();
  }
  if (total == 0) return RFCMP_OK;
  if (op->sp_scratch.p && op->sp_scratch.bytes >= sizeof(double2) * (size_t)total && op->sp_scratch_nrhs == op->work_nrhs &&
      op->sp_region[2] == off[2] && op->sp_region[1] == off[1])
    return RFCMP_OK;
  if (op->sp_scratch.p) RF_HIP(hipDeviceSynchronize());  // the old scratch may still be in use
  RF_TRY(op->sp_scratch.alloc(sizeof(double2) * (size_t)total));
  for (int q = 0; q < 3; ++q) op->sp_region[q] = off[q];
  op->sp_scratch_nrhs = op->work_nrhs;
  return RFCMP_OK;
}

// Scratch of the FP64 multi-right-hand-side products (zgemm_c64): sized
// for both blocks (the slice count depends on the order).
rfcmp_status ensure_z_scratch(rfcmp_op op) {
  const size_t need = std::max(zgemm_scratch_bytes(op->mesh->h.N), zgemm_scratch_bytes(op->mesh->h.C));
  if (op->z_scratch.bytes >= need) return RFCMP_OK;
  if (op->z_scratch.p) RF_HIP(hipDeviceSynchronize());  // the old scratch may still be in use
  return op->z_scratch.alloc(need);
}

// Grow the workspace (and pinned host scalars) to at least R right-hand sides.
rfcmp_status ensure_work(rfcmp_op op, int R) {
  R = std::max(R, 4);
  if (op->work.p && op->work_nrhs >= R) return RFCMP_OK;
  const MeshHost& h = op->mesh->h;
  if (op->work.p) RF_HIP(hipDeviceSynchronize());  // the old workspace may still be in use by queued work
  RF_TRY(op->work.alloc(sizeof(double2) * work_doubles2(h.N, h.C, h.V, R) + 4096));
  op->work_nrhs = R;
  if (op->host_scal) (void)hipHostFree(op->host_scal);
  op->host_scal = nullptr;
  op->host_scal_dev = nullptr;
  RF_HIP(hipHostMalloc((void**)&op->host_scal, sizeof(double) * (16 + 8 * R), hipHostMallocMapped));
  RF_HIP(hipHostGetDevicePointer((void**)&op->host_scal_dev, op->host_scal, 0));
  return ensure_sp_scratch(op);
}

// ------------------------------------------------------------------ dense products
// The five dense matrices of the operator.  In complex64/FP64 each product is
// a symmetric streaming pass (<= 4 right-hand sides per pass) whose input is
// formed while it is staged (plain vector, Sigma^T / Lambda^T gather, or a
// fused operator line); two independent products of the same element type
// share one launch.  As BF16x3 MFMA products (<= 64 right-hand sides per
// pass) the input is formed into the workspace first.
enum Mat { kTA, kV, kLP, kGLL, kGTP };

struct Dense {
  rfcmp_op op;
  hipStream_t s;
  bool bf16;
  const Work* W = nullptr;  // workspace for formed inputs (BF16x3 and FP64 multi-RHS products)

  SymvJob job(Mat m, const SymvInput& in, double2* y) const {
    const MeshHost& h = op->mesh->h;
    const MeshDev& d = op->mesh->d;
    SymvJob j;
    switch (m) {
      case kTA: j.M = op->TA.p; j.n = h.N; j.ld = op->ldA; break;
      case kV: j.M = op->Vb.p; j.n = h.C; j.ld = op->ldV; break;
      case kLP: j.M = d.Lp.p; j.n = h.C; j.ld = d.ldL; break;
      case kGLL: j.M = d.Gll_inv.p; j.n = h.V; j.ld = d.ldG; break;
      default: j.M = d.Gtp_inv.p; j.n = h.C; j.ld = d.ldT; break;
    }
    j.in = in;
    j.y = y;
    return j;
  }
  const SplitMatrix& split(Mat m) const {
    const MeshDev& d = op->mesh->d;
    switch (m) {
      case kTA: return *op->TA16;
      case kV: return *op->V16;
      case kLP: return *d.Lp16;
      case kGLL: return *d.Gll16;
      default: return *d.Gtp16;
    }
  }
  static const char* tag(Mat m) {
    static const char* t[] = {"cmatvec_ta", "cmatvec_v", "dmatvec_lp", "dmatvec_gll", "dmatvec_gtp"};
    return t[m];
  }
  static const char* gemm_tag(Mat m) {
    static const char* t[] = {"gemm_ta", "gemm_v", "gemm_lp", "gemm_gll", "gemm_gtp"};
    return t[m];
  }
  static bool complex_matrix(Mat m) { return m == kTA || m == kV; }
  static const char* zgemm_tag(Mat m) { return m == kTA ? "zgemm_ta" : "zgemm_v"; }

  // FP64-accumulated product on the FP64 matrix cores (many right-hand
  // sides): form the input (unless plain) and run zgemm_c64.
  rfcmp_status zgemm(Mat m, bool conj, const SymvInput& in, double2* y, int nr) const {
    const SymvJob j = job(m, in, y);
    const double2* x = in.p[0];
    if (in.mode != SymvInput::kPlain || in.stride[0] != j.n) {
      double2* buf = j.n == op->mesh->h.N ? W->xN : W->xC;
      RF_TRY(symv_form_input(in, j.n, nr, buf, s));
      x = buf;
    }
    RF_TRY(ensure_z_scratch(op));
    return zgemm_c64(static_cast<const float2*>(j.M), j.n, j.ld, conj, x, y, nr, op->z_scratch.p,
                     op->z_scratch.bytes, s, zgemm_tag(m));
  }

  // BF16x3: form the input (unless plain) and run the GEMM.
  rfcmp_status gemm(Mat m, bool conj, const SymvInput& in, double2* y, int nr) const {
    const SymvJob j = job(m, in, y);
    const double2* x = in.p[0];
    if (in.mode != SymvInput::kPlain || in.stride[0] != j.n) {
      double2* buf = j.n == op->mesh->h.N ? W->xN : (j.n == op->mesh->h.C ? W->xC : W->xV);
      RF_TRY(symv_form_input(in, j.n, nr, buf, s));
      x = buf;
    }
    return gemm_bf16x3(split(m), conj, x, y, nr, op->gemm_scratch.p, op->gemm_scratch.bytes, s, gemm_tag(m));
  }

  // The projector matrices as sparse FP64 factors (projector option 1): in
  // both precisions.
  bool sparse(Mat m) const { return !complex_matrix(m) && op->opt.projector == kProjSparse; }
  static int sp_index(Mat m) { return m == kLP ? 0 : (m == kGLL ? 1 : 2); }
  static const char* sp_tag(Mat m0, const Mat* m1) {
    static const char* t[] = {"spsolve_lp", "spsolve_gll", "spsolve_gtp"};
    static const char* tp[] = {"spsolve_lp+gll", "spsolve_lp+gtp"};
    if (!m1) return t[sp_index(m0)];
    return *m1 == kGLL ? tp[0] : tp[1];
  }
  rfcmp_status sp_solve(Mat m0, const SymvInput& in0, double2* y0, const Mat* m1, const SymvInput* in1,
                        double2* y1, int nr, int nr1) const {
    const MeshDev& d = op->mesh->d;
    SpSolveJob j[2];
    const Mat ms[2] = {m0, m1 ? *m1 : m0};
    const int nj = m1 ? 2 : 1;
    for (int q = 0; q < nj; ++q) {
      const int fi = sp_index(ms[q]);
      if (!d.sp[fi]) {
        set_error("sparse projector factor %d not built for this mesh", fi);
        return RFCMP_E_STATE;
      }
      // the job's right-hand sides must fit its scratch region
      const int64_t need = (int64_t)(q ? (nr1 > 0 ? nr1 : nr) : nr) * d.sp[fi]->scratch_entries();
      if (op->sp_scratch_nrhs < (q ? (nr1 > 0 ? nr1 : nr) : nr) ||
          (op->sp_region[fi] + need) * (int64_t)sizeof(double2) > (int64_t)op->sp_scratch.bytes) {
        set_error("sparse projector solve: scratch region %d too small", fi);
        return RFCMP_E_STATE;
      }
      j[q].F = d.sp[fi].get();
      j[q].in = q ? *in1 : in0;
      j[q].y = q ? y1 : y0;
      j[q].scratch = op->sp_scratch.as<double2>() + op->sp_region[fi];
      j[q].nrhs = q ? nr1 : 0;
    }
    if (nr > op->work_nrhs) {
      set_error("sparse projector solve: %d right-hand sides, scratch for %d", nr, op->work_nrhs);
      return RFCMP_E_STATE;
    }
    const char* tag = sp_tag(m0, m1);
    return spsolve_jobs(j, nj, nr, s, nr == 1 ? tag : profile_tag_suffix(tag, nr));
  }

  // y = M x (conj: conj(M) x, complex matrices only).
  // The projector matrices (L^+, G_ll^-1, G_tp^-1) are applied in FP64 in
  // both precisions; BF16x3 serves the blocks T_A and V.
  // Compressed blocks (options.aca_tol > 0): form the input (unless plain)
  // and run the hierarchical product.
  rfcmp_status hprod(Mat m, bool conj, const SymvInput& in, double2* y, int nr) const {
    const int64_t n = m == kTA ? op->mesh->h.N : op->mesh->h.C;
    const double2* x = in.p[0];
    if (in.mode != SymvInput::kPlain || in.stride[0] != n) {
      double2* buf = m == kTA ? W->xN : W->xC;
      RF_TRY(symv_form_input(in, n, nr, buf, s));
      x = buf;
    }
    return hm_matvec(op, m == kTA ? 0 : 1, conj, x, y, nr, s);
  }

  rfcmp_status prod(Mat m, bool conj, const SymvInput& in, double2* y, int nr) const {
    if (sparse(m)) return sp_solve(m, in, y, nullptr, nullptr, nullptr, nr, 0);
    if (op->hm && complex_matrix(m)) return hprod(m, conj, in, y, nr);
    if (bf16 && complex_matrix(m)) return gemm(m, conj, in, y, nr);
    if (complex_matrix(m) && nr >= kZgemmMinRhs && W) return zgemm(m, conj, in, y, nr);
    const SymvJob j = job(m, in, y);
    if (complex_matrix(m))
      return csymv_jobs(&j, 1, conj, nr, op->symv_scratch.p, op->symv_scratch.bytes, s, tag(m));
    return dsymv_jobs(&j, 1, nr, op->symv_scratch.p, op->symv_scratch.bytes, s, tag(m));
  }
  rfcmp_status prod(Mat m, bool conj, const double2* x, double2* y, int nr) const {
    return prod(m, conj, plain(x, job(m, SymvInput{}, y).n), y, nr);
  }
  // Two independent products of the same element type in one launch.
  // nr1 > 0: the second product takes only nr1 of the nr right-hand sides.
  rfcmp_status pair(Mat m0, const SymvInput& in0, double2* y0, Mat m1, const SymvInput& in1, double2* y1,
                    bool conj, int nr, int nr1 = 0) const {
    if (sparse(m0) && sparse(m1)) return sp_solve(m0, in0, y0, &m1, &in1, y1, nr, nr1);
    if (sparse(m0) || sparse(m1) || (op->hm && complex_matrix(m0))) {
      RF_TRY(prod(m0, conj, in0, y0, nr));
      return prod(m1, conj, in1, y1, nr1 > 0 ? nr1 : nr);
    }
    if (bf16 && complex_matrix(m0)) {
      RF_TRY(gemm(m0, conj, in0, y0, nr));
      return gemm(m1, conj, in1, y1, nr1 > 0 ? nr1 : nr);
    }
    if (complex_matrix(m0) && nr >= kZgemmMinRhs && W) {
      RF_TRY(prod(m0, conj, in0, y0, nr));
      return prod(m1, conj, in1, y1, nr1 > 0 ? nr1 : nr);
    }
    SymvJob j[2] = {job(m0, in0, y0), job(m1, in1, y1)};
    j[1].nrhs = nr1;
    static const char* pair_tag[] = {"cmatvec_ta+v", "dmatvec_lp+gll", "dmatvec_lp+gtp"};
    if (complex_matrix(m0))
      return csymv_jobs(j, 2, conj, nr, op->symv_scratch.p, op->symv_scratch.bytes, s, pair_tag[0]);
    return dsymv_jobs(j, 2, nr, op->symv_scratch.p, op->symv_scratch.bytes, s,
                      m1 == kGLL ? pair_tag[1] : pair_tag[2]);
  }

  // --- inputs
  static SymvInput plain(const double2* x, int64_t n) {
    SymvInput in;
    in.p[0] = x;
    in.stride[0] = n;
    return in;
  }
  SymvInput sigma_t(const double2* x) const {  // Sigma^T x, x [nr][N]
    const MeshDev& d = op->mesh->d;
    SymvInput in;
    in.mode = SymvInput::kSigmaT;
    in.p[0] = x;
    in.stride[0] = op->mesh->h.N;
    in.idx0 = d.cell_edge.as<int>();
    in.sgn = d.sgn.as<float>();
    return in;
  }
  SymvInput lambda_t(const double2* x) const {  // Lambda^T x, x [nr][N]
    const MeshDev& d = op->mesh->d;
    SymvInput in;
    in.mode = SymvInput::kLambdaT;
    in.p[0] = x;
    in.stride[0] = op->mesh->h.N;
    in.idx0 = d.ve_ptr.as<int>();
    in.idx1 = d.ve_idx.as<int>();
    in.sgn = d.ve_sgn.as<float>();
    return in;
  }
  SymvInput vin(const double2* x, const double2* s1, const double2* sg, double ka, double kb) const {
    SymvInput in;
    in.mode = SymvInput::kVin;
    in.p[0] = x; in.stride[0] = op->mesh->h.N;
    in.p[1] = s1; in.stride[1] = op->mesh->h.C;
    in.p[2] = sg; in.stride[2] = op->mesh->h.C;
    in.c[0] = ka; in.c[1] = kb;
    in.idx0 = op->mesh->d.edge_cell.as<int>();
    return in;
  }
  SymvInput middle_w(const double2* h, const double2* a, const double2* s2, const double2* s3, double ia2,
                     double ig, double ib2) const {
    SymvInput in;
    in.mode = SymvInput::kMiddleW;
    in.p[0] = h; in.stride[0] = op->mesh->h.V;
    in.p[1] = a; in.stride[1] = op->mesh->h.N;
    in.p[2] = s2; in.stride[2] = op->mesh->h.C;
    in.p[3] = s3; in.stride[3] = op->mesh->h.C;
    in.c[0] = ia2; in.c[1] = ig; in.c[2] = ib2;
    in.idx0 = op->mesh->d.edge_cell.as<int>();
    in.idx1 = op->mesh->d.edge_vtx.as<int>();
    return in;
  }
  SymvInput proj_lh(const double2* x, const double2* sl) const {  // x - Sigma sl
    SymvInput in;
    in.mode = SymvInput::kProjLH;
    in.p[0] = x; in.stride[0] = op->mesh->h.N;
    in.p[1] = sl; in.stride[1] = op->mesh->h.C;
    in.idx0 = op->mesh->d.edge_cell.as<int>();
    return in;
  }
};

bool use_gsigma(rfcmp_op op) { return op->opt.outer_star == 1; }

// Left half: y = sgn * P_o^H T^H w, with w = middle_w(v2, a, s2, s3) and
// Sig^T w_S (= (t4 - mean t4)/beta^2) in W.c[8].
rfcmp_status left_half(const Dense& D, const Work& W, const SymvInput& w_in, double2* y, int nr, double sgn) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C;
  const double k = op->k, al = op->alpha, be = op->beta;
  double2 *s4 = W.c[10], *vw = W.c[11], *t6 = W.c[12], *g6 = W.c[13];
  RF_TRY(D.pair(kTA, w_in, W.nD, kV, Dense::plain(W.c[8], C), vw, true, nr));  // zA, vw
  RF_TRY(D.prod(kLP, false, D.sigma_t(W.nD), s4, nr));
  RF_TRY(comb_mean(C, nullptr, -sgn * (k / be), s4, sgn / (k * be), vw, t6, 0.0, nullptr, nr, s));
  const double2* gsel = t6;
  if (use_gsigma(op)) {
    RF_TRY(D.prod(kGTP, false, t6, g6, nr));
    gsel = g6;
  }
  return left_y(d, N, C, sgn * k / al, W.nD, s4, gsel, y, nr, s);
}

// y = A x for nr <= W.R right-hand sides.
rfcmp_status apply_batch(const Dense& D, const Work& W, const double2* x, double2* y, int nr) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t C = h.C;
  const double k = op->k, al = op->alpha, be = op->beta, ga = op->gamma;
  double2 *s1 = W.c[1], *g1 = W.c[2], *s1g = W.c[3], *vphi = W.c[4], *s2 = W.c[6], *t4 = W.c[7], *sw = W.c[8],
          *s3 = W.c[9];
  const SymvInput sx = D.sigma_t(x);
  SymvInput sus = sx;      // Sig^T u_S
  const double2* s_us = s1;  // u_S = Sig s_us
  if (use_gsigma(op)) {
    RF_TRY(D.pair(kLP, sx, s1, kGTP, sx, g1, false, nr));
    RF_TRY(D.prod(kLP, false, g1, s1g, nr));
    sus = Dense::plain(g1, C);
    s_us = s1g;
  } else {
    RF_TRY(D.prod(kLP, false, sx, s1, nr));
  }
  // a = T_A((ik/alpha) u_L - (k/beta) u_S),  vphi = V Sig^T u_S
  RF_TRY(D.pair(kTA, D.vin(x, s1, s_us, k / al, k / be), W.nB, kV, sus, vphi, false, nr));
  // s2 = L^+ Sig^T a,  h = G_ll^-1 Lam^T a
  RF_TRY(D.pair(kLP, D.sigma_t(W.nB), s2, kGLL, D.lambda_t(W.nB), W.v2, false, nr));
  // t4 = A (s2 + (vphi - mean vphi)/(k beta)),  Sig^T w_S = (t4 - mean t4)/beta^2
  RF_TRY(comb_mean(C, d.area.as<double>(), 1.0, s2, 1.0 / (k * be), vphi, t4, 1.0 / (be * be), sw, nr, s));
  RF_TRY(D.prod(kLP, false, t4, s3, nr));
  return left_half(D, W, D.middle_w(W.v2, W.nB, s2, s3, 1.0 / (al * al), 1.0 / ga, 1.0 / (be * be)), y, nr,
                   1.0);
}

rfcmp_status rhs_batch(const Dense& D, const Work& W, const double2* e, double2* b, int nr) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t C = h.C;
  const double al = op->alpha, be = op->beta, ga = op->gamma;
  double2 *s2 = W.c[6], *t4 = W.c[7], *sw = W.c[8], *s3 = W.c[9];
  RF_TRY(D.pair(kLP, D.sigma_t(e), s2, kGLL, D.lambda_t(e), W.v2, false, nr));
  RF_TRY(comb_mean(C, d.area.as<double>(), 1.0, s2, 0.0, nullptr, t4, 1.0 / (be * be), sw, nr, s));
  RF_TRY(D.prod(kLP, false, t4, s3, nr));
  return left_half(D, W, D.middle_w(W.v2, e, s2, s3, 1.0 / (al * al), 1.0 / ga, 1.0 / (be * be)), b, nr, -1.0);
}

// b = -P_o^H T^H P_m e for the split excitation e = Sigma sv + e1: the static
// part lies in the range of Sigma, where P_mL vanishes and
// P_mS Sigma sv = Sigma L^+ A (sv - mean sv)/beta^2 (L^+ L = I - 1 1^T/C), so
// the O(1) static part never meets the O(k) loop part of e1:
//   s2 = L^+ Sigma^T e1, h = G_ll^-1 Lambda^T e1,
//   t4 = A (s2 + sv - mean sv), s3 = L^+ t4,
//   w  = Lambda h/alpha^2 + (e1 - Sigma s2)/gamma + Sigma s3/beta^2.
rfcmp_status rhs_batch_split(const Dense& D, const Work& W, const double2* sv, const double2* e1, double2* b,
                             int nr) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t C = h.C;
  const double al = op->alpha, be = op->beta, ga = op->gamma;
  double2 *s2 = W.c[6], *t4 = W.c[7], *sw = W.c[8], *s3 = W.c[9];
  RF_TRY(D.pair(kLP, D.sigma_t(e1), s2, kGLL, D.lambda_t(e1), W.v2, false, nr));
  RF_TRY(comb_mean(C, d.area.as<double>(), 1.0, s2, 1.0, sv, t4, 1.0 / (be * be), sw, nr, s));
  RF_TRY(D.prod(kLP, false, t4, s3, nr));
  return left_half(D, W, D.middle_w(W.v2, e1, s2, s3, 1.0 / (al * al), 1.0 / ga, 1.0 / (be * be)), b, nr, -1.0);
}

// j = P_o x (recover_batch); with js != nullptr, j receives the loop part
// P_LH x/alpha and js the star part i P_s x/beta.
rfcmp_status recover_batch(const Dense& D, const Work& W, const double2* x, double2* j, int nr,
                           double2* js = nullptr);
rfcmp_status recover_batch(const Dense& D, const Work& W, const double2* x, double2* j, int nr, double2* js) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C;
  const SymvInput sx = D.sigma_t(x);
  const double2* sg = W.c[1];
  if (use_gsigma(op)) {
    RF_TRY(D.pair(kLP, sx, W.c[1], kGTP, sx, W.c[2], false, nr));
    RF_TRY(D.prod(kLP, false, W.c[2], W.c[3], nr));
    sg = W.c[3];
  } else {
    RF_TRY(D.prod(kLP, false, sx, W.c[1], nr));
  }
  if (js) return recover_j_split(d, N, C, 1.0 / op->alpha, 1.0 / op->beta, x, W.c[1], sg, j, js, nr, s);
  return recover_j(d, N, C, 1.0 / op->alpha, 1.0 / op->beta, x, W.c[1], sg, j, nr, s);
}

// Run f over chunks of at most W.R right-hand sides.
template <class F>
rfcmp_status batched(int nrhs, int R, int64_t nin, int64_t nout, const double2* x, double2* y, F f) {
  for (int r0 = 0; r0 < nrhs; r0 += R) {
    const int nr = std::min(R, nrhs - r0);
    RF_TRY(f(x + (int64_t)r0 * nin, y + (int64_t)r0 * nout, nr));
  }
  return RFCMP_OK;
}

// One power-iteration application of the three scaling operators to the
// normalised rows of W.pv ([3][N]: alpha, gamma, beta); the results,
// normalised, replace them, with their squared norms in W.dout.
//   O_alpha v = P_LH conj(T_A) Lam G_ll^-1 Lam^T T_A P_LH v
//   O_gamma v = P_LH conj(T_A) P_LH T_A P_LH v
//   O_beta  v = P_Sigma T_Phi^H P_mS_hat T_Phi P_Sigma v
//             = Sig conj(V) (I - J) diag(A) (I - J) V Sig^T v
// project_in: apply P_LH to the alpha and gamma inputs.  Only the random
// start vector needs it: every later input is the normalised output of the
// previous step, which ends in P_LH, and P_LH is idempotent (Sigma^T P_LH = 0).
rfcmp_status power_apply(const Dense& D, const Work& W, bool project_in) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C, V = h.V;
  double2* va = W.pv;
  double2* vb = W.pv + 2 * N;
  // The beta chain's two V products ride along with the two-column T_A
  // passes of alpha and gamma, with one column of their own.
  const SymvInput sb = D.sigma_t(vb);
  if (project_in) RF_TRY(D.prod(kLP, false, D.sigma_t(va), W.c[1], 2));
  const SymvInput ta_in = project_in ? D.proj_lh(va, W.c[1]) : Dense::plain(va, N);
  RF_TRY(D.pair(kTA, ta_in, W.nB, kV, sb, W.c[7], false, 2, 1));                    // T_A P_LH v | V Sig^T v
  RF_TRY(D.pair(kLP, D.sigma_t(W.nB + N), W.c[3], kGLL, D.lambda_t(W.nB), W.v2, false, 1));
  RF_TRY(comb_mean(C, d.area.as<double>(), 0.0, nullptr, 1.0, W.c[7], W.c[8], 1.0, W.c[9], 1, s));
  RF_TRY(power_branch(d, N, V, C, W.v2, W.nB, W.c[3], W.nC, s));                // alpha | gamma branch
  RF_TRY(D.pair(kTA, Dense::plain(W.nC, N), W.nD, kV, Dense::plain(W.c[9], C), W.c[10], true, 2, 1));
  RF_TRY(D.prod(kLP, false, D.sigma_t(W.nD), W.c[5], 2));
  return power_next(d, N, C, W.nD, W.c[5], W.c[10], W.pv, W.dout, s);
}

// alpha, beta, gamma from the three power-iteration norms (rows alpha,
// gamma, beta of W.dout), reading 3 of the Sec. 4 norms
struct Scalings {
  double a, b, g;
};
Scalings scalings_of(double k, const double2 (&nr2)[3]) {
  const double la = std::sqrt(nr2[0].x), lg = std::sqrt(nr2[1].x), lb = std::sqrt(nr2[2].x);
  const double a = std::pow(k * k * la, 0.25);
  return {a, std::pow(lb / (k * k), 0.25), k * k * lg / (a * a)};
}

// The three power iterations side by side, at most `steps` steps.  With
// tol > 0 the scalings are read every kPowerCheck steps, and the iteration
// stops at the first check from 2 kPowerCheck steps on where each of alpha,
// beta, gamma moved by less than tol (relative) since the previous check.
constexpr int kPowerCheck = 5;
rfcmp_status power_scalings(rfcmp_op op, const double2* start, int steps, double tol, hipStream_t s) {
  const int64_t N = op->mesh->h.N;
  RF_TRY(ensure_work(op, 4));
  const Work W = carve(op);
  const Dense D{op, s, false, &W};
  for (int r = 0; r < 3; ++r)
    RF_HIP(hipMemcpyAsync(W.pw + r * N, start, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
  RF_TRY(normalize_rows(N, W.pw, W.pv, W.dout, 3, s));
  // each application ends with the next normalised vectors in W.pv and the
  // squared norms of the raw ones in W.dout
  double2* hn = reinterpret_cast<double2*>(op->host_scal);  // pinned
  const double k = op->k;
  Scalings prev{0.0, 0.0, 0.0};
  int done = 0;
  for (int it = 0; it < steps; ++it) {
    RF_TRY(power_apply(D, W, it == 0));
    done = it + 1;
    if (tol > 0 && done % kPowerCheck == 0 && done < steps) {
      RF_HIP(hipMemcpyAsync(hn, W.dout, sizeof(double2) * 3, hipMemcpyDeviceToHost, s));
      RF_HIP(hipStreamSynchronize(s));
      const double2 nr2[3] = {hn[0], hn[1], hn[2]};
      const Scalings cur = scalings_of(k, nr2);
      const bool conv = done >= 2 * kPowerCheck && std::fabs(cur.a - prev.a) <= tol * cur.a &&
                        std::fabs(cur.b - prev.b) <= tol * cur.b && std::fabs(cur.g - prev.g) <= tol * cur.g;
      prev = cur;
      if (conv) break;
    }
  }
  RF_HIP(hipMemcpyAsync(hn, W.dout, sizeof(double2) * 3, hipMemcpyDeviceToHost, s));
  RF_HIP(hipStreamSynchronize(s));
  const double2 nr2[3] = {hn[0], hn[1], hn[2]};
  const double la = std::sqrt(nr2[0].x), lg = std::sqrt(nr2[1].x), lb = std::sqrt(nr2[2].x);
  if (!(la > 0) || !(lb > 0) || !(lg > 0) || !std::isfinite(la + lb + lg)) {
    set_error("power iteration produced a non-positive norm (%g, %g, %g)", la, lb, lg);
    return RFCMP_E_STATE;
  }
  const Scalings sc = scalings_of(k, nr2);
  op->lam[0] = la;
  op->lam[1] = lb;
  op->lam[2] = lg;
  op->alpha = sc.a;
  op->beta = sc.b;
  op->gamma = sc.g;
  op->power_steps = done;
  return RFCMP_OK;
}

// ------------------------------------------------------------------ CG
// Extreme eigenvalues of the CG Lanczos tridiagonal (Sec. 3.4: the iteration
// count is governed by cond(A)).  With step lengths a_i and b_i = rho_{i+1}/rho_i
// the tridiagonal has diagonal 1/a_1, 1/a_i + b_{i-1}/a_{i-1} and off-diagonal
// sqrt(b_i)/a_i; its eigenvalues are found by Sturm-sequence bisection.
double lanczos_cond(const std::vector<double>& a, const std::vector<double>& b) {
  const size_t m = a.size();
  if (m < 2) return 0.0;
  std::vector<double> d(m), e(m, 0.0);
  for (size_t i = 0; i < m; ++i) {
    d[i] = 1.0 / a[i] + (i ? b[i - 1] / a[i - 1] : 0.0);
    if (i + 1 < m) e[i] = std::sqrt(b[i]) / a[i];
  }
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < m; ++i) {
    const double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {  // number of eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (size_t i = 1; i < m; ++i) {
      const double qq = (q == 0.0) ? 1e-300 : q;
      q = d[i] - x - e[i - 1] * e[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int k) {  // k-th smallest (0-based)
    double a0 = lo, b0 = hi;
    for (int it = 0; it < 200 && b0 - a0 > 1e-13 * std::max(std::fabs(a0), std::fabs(b0)); ++it) {
      const double mid = 0.5 * (a0 + b0);
      if (count_below(mid) > k) b0 = mid; else a0 = mid;
    }
    return 0.5 * (a0 + b0);
  };
  const double lmin = kth(0), lmax = kth((int)m - 1);
  return lmin > 0 ? lmax / lmin : 0.0;
}

// Block of nr independent complex CGs on the HPD system (Sec. 3.4) sharing
// the operator passes: solves A x = W.b from x = 0 (x in W.x), stopping
// right-hand side r once its recursive residual norm is <= target[r] (it is
// then frozen: step length 0), or after maxit iterations.  The CG scalars
// stay on the device; the host examines iteration i while iteration i+1 runs
// (pinned copies and events), so the GPU never waits for the test.  iters[r]
// counts the iterations in which r was still active.
rfcmp_status block_cg(const Dense& D, const Work& W, int nr, const double* target, int maxit, int* iters,
                      double* cond = nullptr) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const int64_t N = op->mesh->h.N;
  const int64_t NR = (int64_t)nr * N;
  double* hs = op->host_scal;  // per parity p: rho_new at 4Rp, pq at 4Rp + R; active flags at 6R
  double* hs_dev = op->host_scal_dev;  // the same memory as the device addresses it
  const int R = W.R;
  std::vector<int> act(nr, 1);
  for (int r = 0; r < nr; ++r) iters[r] = 0;
  RF_HIP(hipMemsetAsync(W.x, 0, sizeof(double2) * NR, s));
  RF_HIP(hipMemcpyAsync(W.r, W.b, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  RF_HIP(hipMemcpyAsync(W.p, W.b, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  RF_TRY(set_active(W.active, 1, nr, s));
  RF_TRY(dot(N, W.r, W.r, W.part, W.dout, nr, s));
  RF_TRY(take_real_n(W.dout, W.rho, nr, s));  // rho[0][r]
  std::vector<double> rho_prev(nr);
  RF_HIP(hipMemcpyAsync(hs, W.rho, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
  RF_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nr; ++r) rho_prev[r] = hs[r];
  std::vector<std::vector<double>> la(nr), lb(nr);
  hipEvent_t ev[2];
  RF_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  RF_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  // The iterations run on the operator's internal stream when they are
  // replayed as graphs (a stream that can be captured: the caller's may be the
  // null stream), after the set-up above on s; s waits for them at the end.
  const bool use_graphs = op->opt.graphs == 1 && !profiling_enabled();
  hipStream_t cs = s;
  if (use_graphs) {
    if (!op->cg_stream) RF_HIP(hipStreamCreateWithFlags(&op->cg_stream, hipStreamNonBlocking));
    cs = op->cg_stream;
    RF_HIP(hipEventRecord(ev[0], s));
    RF_HIP(hipStreamWaitEvent(cs, ev[0], 0));
  }
  Dense Dc = D;
  Dc.s = cs;
  // one iteration of parity c (the recurrence scalars at rho + c R, the host
  // copies in slot c), without the event that publishes them
  auto iteration = [&](int c) -> rfcmp_status {
    RF_TRY(apply_batch(Dc, W, W.p, W.q, nr));
    // the dot kernels also store the real parts for the host, straight into
    // the mapped pinned buffer; the event recorded after the iteration
    // publishes them
    RF_TRY(dot(N, W.p, W.q, W.part, W.dout, nr, cs, W.pq, hs_dev + c * 4 * R + R));
    RF_TRY(cg_xr_blk(N, nr, W.rho + c * R, W.pq, W.active, W.x, W.r, W.p, W.q, cs));
    RF_TRY(dot(N, W.r, W.r, W.part, W.dout, nr, cs, W.rho + (1 - c) * R, hs_dev + c * 4 * R));
    return cg_p_blk(N, nr, W.rho + (1 - c) * R, W.rho + c * R, W.active, W.r, W.p, cs);
  };
  // every kernel argument of an iteration, apart from the parity
  uint64_t key = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
  if (use_graphs) {
    double sc[3] = {op->alpha, op->beta, op->gamma};
    uint64_t bits[3];
    std::memcpy(bits, sc, sizeof(bits));
    for (uint64_t b : bits) mix(b);
    mix((uint64_t)nr);
    mix((uint64_t)D.bf16);
    mix((uint64_t)(uintptr_t)op->work.p);
    mix((uint64_t)op->work_nrhs);
    mix((uint64_t)(uintptr_t)op->sp_scratch.p);
    mix((uint64_t)(uintptr_t)op->symv_scratch.p);
    mix((uint64_t)(uintptr_t)op->gemm_scratch.p);
    mix((uint64_t)(uintptr_t)op->z_scratch.p);
    mix((uint64_t)(uintptr_t)hs_dev);
  }
  auto graph_for = [&](int c) -> rfcmp_status {
    if (op->cg_exec[c] && op->cg_key[c] == key) return RFCMP_OK;
    if (op->cg_exec[c]) RF_HIP(hipGraphExecDestroy(op->cg_exec[c]));
    op->cg_exec[c] = nullptr;
    RF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const rfcmp_status st = iteration(c);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (st < 0) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess || !g) {
      set_error("capture of a CG iteration failed: %s", hipGetErrorString(ec));
      return RFCMP_E_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&op->cg_exec[c], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      op->cg_exec[c] = nullptr;
      set_error("instantiating a CG iteration graph failed: %s", hipGetErrorString(ei));
      return RFCMP_E_HIP;
    }
    op->cg_key[c] = key;
    return RFCMP_OK;
  };
  int cur = 0, it = 0, last_checked = -1, nactive = nr;
  while (true) {
    bool issued = false;
    if (it < maxit && nactive > 0) {
      const int slot = it & 1;
      if (use_graphs && it >= 2) {
        RF_TRY(graph_for(cur));
        RF_HIP(hipGraphLaunch(op->cg_exec[cur], cs));
      } else {
        RF_TRY(iteration(cur));
      }
      RF_HIP(hipEventRecord(ev[slot], cs));
      const int nxt = 1 - cur;
      cur = nxt;
      ++it;
      for (int r = 0; r < nr; ++r) iters[r] += act[r];
      issued = true;
    }
    const int look = issued ? it - 2 : it - 1;
    if (look <= last_checked) {
      if (!issued) break;
      continue;
    }
    RF_HIP(hipEventSynchronize(ev[look & 1]));
    last_checked = look;
    const double* h = hs + (look & 1) * 4 * R;
    bool changed = false;
    for (int r = 0; r < nr; ++r) {
      if (!act[r]) continue;
      const double rho = h[r], pq = h[R + r];
      if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rho)) {
        set_error("CG breakdown at iteration %d (rhs %d): p^H A p = %g", look + 1, r, pq);
        return RFCMP_E_BREAKDOWN;
      }
      la[r].push_back(rho_prev[r] / pq);
      lb[r].push_back(rho / rho_prev[r]);
      rho_prev[r] = rho;
      if (std::sqrt(rho) <= target[r]) {
        act[r] = 0;
        --nactive;
        changed = true;
      }
    }
    if (changed) {
      // freeze converged right-hand sides from the next enqueued iteration on
      int* ha = reinterpret_cast<int*>(hs + 6 * R);
      for (int r = 0; r < nr; ++r) ha[r] = act[r];
      RF_HIP(hipMemcpyAsync(W.active, ha, sizeof(int) * nr, hipMemcpyHostToDevice, cs));
      RF_HIP(hipStreamSynchronize(cs));  // ha is reused by the next change
    }
    if (nactive == 0 || !issued) break;
  }
  if (cs != s) {
    RF_HIP(hipEventRecord(ev[0], cs));
    RF_HIP(hipStreamWaitEvent(s, ev[0], 0));
  }
  if (cond)
    for (int r = 0; r < nr; ++r) cond[r] = lanczos_cond(la[r], lb[r]);
  return RFCMP_OK;
}

// Solve for nr <= W.R right-hand sides e (device) into j:
//   precision 0: block CG on the complex64/FP64 operator to |r| <= tol |b|,
//                restarted from the true residual until that meets tol too;
//   precision 1: iterative refinement: inner block CG on the BF16x3 operator
//                to kInnerReduction of the current residual (not below
//                kFinalTarget tol), i += d, true residual
//                r = b - A i with the complex64/FP64 operator, until
//                |r| <= tol |b|.
// system: e is the system's own right-hand side b and j receives the iterate
// i (no excitation mapping, no recovery).
// sv != nullptr: the excitation is split, e = Sigma sv + e (rhs_batch_split);
// js != nullptr: j receives the loop part of the solution and js its star part.
// ------------------------------------------------------------------ block CG
// CG on the nr right-hand sides with one shared Krylov space (block CG,
// O'Leary 1980, with orthonormalised search blocks): solves A X = W.b from
// X = 0 (X in W.x), iterating
//   Q = A P,  M = P^H Q,  alpha = M^-1 P^H R,  X += P alpha,  R -= Q alpha,
//   Y = R - P M^-1 Q^H R  (A-orthogonal to P),  P = Y S,
// where S comes from a pivoted Cholesky factorisation of Y^H Y (columns whose
// remaining norm falls below 1e-7 of the largest are dropped, so a block that
// loses rank -- right-hand sides converged, or dependent -- keeps going on
// the rest) and makes P orthonormal.  The block search space holds every
// right-hand side's Krylov space, so each converges in at most the
// iterations of its own CG, usually fewer.  The small matrices are formed by
// tall-skinny Gram products on the device and factored on the host in FP64;
// it stops when every column of R is below its target.
typedef std::complex<double> cplx;
// Products of the small matrices in plain real arithmetic: the operators of
// std::complex follow the C rules for infinities (a library call per
// product), which the finite Gram matrices here never need.
inline cplx cmul(cplx a, cplx b) {
  return cplx(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}
inline cplx cmulc(cplx a, cplx b) {  // conj(a) b
  return cplx(a.real() * b.real() + a.imag() * b.imag(), a.real() * b.imag() - a.imag() * b.real());
}
// options.block_cg = -1 takes the shared block Krylov space from this many
// right-hand sides on (on the level-5 sphere with 64 waves: 14 iterations
// against 21, 190 against 173 solves per second)
constexpr int kBlockAutoRhs = 8;

// Pivoted Cholesky of the Hermitian positive semidefinite G (n x n,
// row-major): G[pi][pi] = R^H R over the kept columns.  Fills S (n x q,
// row-major) with Pi[:, kept] R^-1, so that Y S is orthonormal when G = Y^H Y.
int orth_transform(const std::vector<cplx>& G0, int n, double rel, std::vector<cplx>& S) {
  std::vector<cplx> A = G0;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  double d0 = 0.0;
  for (int i = 0; i < n; ++i) d0 = std::max(d0, A[i * n + i].real());
  std::vector<cplx> R(n * n, cplx(0.0, 0.0));
  int q = 0;
  if (d0 > 0.0)
    for (; q < n; ++q) {
      int p = q;
      for (int i = q + 1; i < n; ++i)
        if (A[i * n + i].real() > A[p * n + p].real()) p = i;
      if (!(A[p * n + p].real() > rel * d0)) break;
      if (p != q) {
        for (int i = 0; i < n; ++i) std::swap(A[q * n + i], A[p * n + i]);
        for (int i = 0; i < n; ++i) std::swap(A[i * n + q], A[i * n + p]);
        for (int i = 0; i < q; ++i) std::swap(R[i * n + q], R[i * n + p]);
        std::swap(perm[q], perm[p]);
      }
      const double rqq = std::sqrt(A[q * n + q].real());
      R[q * n + q] = rqq;
      for (int j = q + 1; j < n; ++j) R[q * n + j] = A[q * n + j] / rqq;
      for (int i = q + 1; i < n; ++i)
        for (int j = q + 1; j < n; ++j) A[i * n + j] -= cmulc(R[q * n + i], R[q * n + j]);
    }
  // R^-1 (upper triangular, q x q, real positive diagonal), by columns;
  // column c kept contiguous (Rt[c q + k] = (R^-1)_kc)
  std::vector<cplx> Rt(q * q, cplx(0.0, 0.0));
  for (int c = 0; c < q; ++c) {
    cplx* col = &Rt[(size_t)c * q];
    col[c] = 1.0 / R[c * n + c].real();
    for (int i = c - 1; i >= 0; --i) {
      cplx acc(0.0, 0.0);
      for (int k = i + 1; k <= c; ++k) acc += cmul(R[i * n + k], col[k]);
      col[i] = -acc / R[i * n + i].real();
    }
  }
  S.assign((size_t)n * q, cplx(0.0, 0.0));
  for (int k = 0; k < q; ++k)
    for (int c = 0; c < q; ++c) S[(size_t)perm[k] * q + c] = Rt[(size_t)c * q + k];
  return q;
}

// Cholesky factor L (p x p, row-major) of M; false if M is not numerically
// positive definite.
bool hpd_factor(const std::vector<cplx>& M, int p, std::vector<cplx>& L) {
  L.assign((size_t)p * p, cplx(0.0, 0.0));
  for (int j = 0; j < p; ++j) {
    cplx d = M[j * p + j];
    for (int k = 0; k < j; ++k) d -= cmulc(L[j * p + k], L[j * p + k]);
    if (!(d.real() > 0.0)) return false;
    const double ljj = std::sqrt(d.real());
    L[j * p + j] = ljj;
    for (int i = j + 1; i < p; ++i) {
      cplx v = M[i * p + j];
      for (int k = 0; k < j; ++k) v -= cmulc(L[j * p + k], L[i * p + k]);
      L[i * p + j] = v / ljj;
    }
  }
  return true;
}

// Z = M^-1 C from the factor of hpd_factor, C p x m row-major: the
// substitutions by rows, all columns of C at once (each entry takes its
// terms in the order of k, as a column-by-column sweep would).
void hpd_subst(const std::vector<cplx>& L, int p, const std::vector<cplx>& C, int m, std::vector<cplx>& Z) {
  Z = C;
  for (int i = 0; i < p; ++i) {  // L y = c
    cplx* zi = &Z[(size_t)i * m];
    for (int k = 0; k < i; ++k) {
      const cplx l = L[i * p + k];
      const cplx* zk = &Z[(size_t)k * m];
      for (int c = 0; c < m; ++c) zi[c] -= cmul(l, zk[c]);
    }
    const double d = L[i * p + i].real();
    for (int c = 0; c < m; ++c) zi[c] /= d;
  }
  for (int i = p - 1; i >= 0; --i) {  // L^H z = y
    cplx* zi = &Z[(size_t)i * m];
    for (int k = i + 1; k < p; ++k) {
      const cplx l = L[k * p + i];
      const cplx* zk = &Z[(size_t)k * m];
      for (int c = 0; c < m; ++c) zi[c] -= cmulc(l, zk[c]);
    }
    const double d = L[i * p + i].real();
    for (int c = 0; c < m; ++c) zi[c] /= d;
  }
}

rfcmp_status block_cg_shared(const Dense& D, const Work& W, int nr, const double* target, int maxit, int* iters) {
  rfcmp_op op = D.op;
  hipStream_t s = D.s;
  const int64_t N = op->mesh->h.N;
  const int64_t NR = (int64_t)nr * N;
  for (int r = 0; r < nr; ++r) iters[r] = 0;
  constexpr size_t kSm = (size_t)kBlockMax * kBlockMax;  // entries of one small matrix
  const size_t need = 3 * sizeof(double2) * kSm + gram_scratch_bytes(N);
  if (op->bcg_scratch.bytes < need) RF_TRY(op->bcg_scratch.alloc(need));
  double2* dS = op->bcg_scratch.as<double2>();  // small matrices of the updates, one per use
  double2* dT = dS + kSm;
  double2* dU = dT + kSm;
  void* gscr = dU + kSm;
  const size_t gbytes = op->bcg_scratch.bytes - 3 * sizeof(double2) * kSm;
  // Host side of an iteration: three waits on the stream.  The Gram results
  // and the norms are written by the device straight into mapped pinned
  // memory (slots 0-2, norms after slot 5); the small matrices go up by
  // asynchronous copies from pinned slots 3-5, each slot rewritten only after
  // a later wait, when its copy has completed.
  if (!op->bcg_host) {
    RF_HIP(hipHostMalloc((void**)&op->bcg_host, sizeof(double2) * (6 * kSm + kBlockMax), hipHostMallocMapped));
    RF_HIP(hipHostGetDevicePointer((void**)&op->bcg_host_dev, op->bcg_host, 0));
  }
  double2* hslot[6];
  double2* dslot[6];
  for (int q = 0; q < 6; ++q) {
    hslot[q] = op->bcg_host + q * kSm;
    dslot[q] = op->bcg_host_dev + q * kSm;
  }
  const double* hrn = reinterpret_cast<const double*>(op->bcg_host + 6 * kSm);
  double* drn = reinterpret_cast<double*>(op->bcg_host_dev + 6 * kSm);
  auto wait = [&]() -> rfcmp_status {
    RF_HIP(hipStreamSynchronize(s));
    return RFCMP_OK;
  };
  auto read = [&](int slot, int cnt, std::vector<cplx>& h) {
    h.resize(cnt);
    for (int i = 0; i < cnt; ++i) h[i] = cplx(hslot[slot][i].x, hslot[slot][i].y);
  };
  auto upload = [&](const std::vector<cplx>& h, int slot, double2* d) -> rfcmp_status {
    double2* t = hslot[slot];
    for (size_t i = 0; i < h.size(); ++i) t[i] = make_double2(h[i].real(), h[i].imag());
    RF_HIP(hipMemcpyAsync(d, t, sizeof(double2) * h.size(), hipMemcpyHostToDevice, s));
    return RFCMP_OK;
  };
  std::vector<double> rn(nr);
  auto take_norms = [&]() {
    for (int r = 0; r < nr; ++r) rn[r] = std::sqrt(std::max(hrn[r], 0.0));
  };
  auto done = [&]() {
    for (int r = 0; r < nr; ++r)
      if (!(rn[r] <= target[r])) return false;
    return true;
  };
  constexpr double kDrop = 1e-14;  // pivots below this fraction of the largest diagonal (norms below 1e-7)
  RF_HIP(hipMemsetAsync(W.x, 0, sizeof(double2) * NR, s));
  RF_HIP(hipMemcpyAsync(W.r, W.b, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  // P = R S: orthonormal basis of the residuals
  RF_TRY(dot(N, W.r, W.r, W.part, W.dout, nr, s, nullptr, drn));
  RF_TRY(gram_c128(W.r, nr, W.r, nr, N, dslot[0], gscr, gbytes, s));
  RF_TRY(wait());
  take_norms();
  if (done()) return RFCMP_OK;
  std::vector<cplx> G, S, M, Lm, C2, C3, A1, T;
  read(0, nr * nr, G);
  int p = orth_transform(G, nr, kDrop, S);
  if (p == 0) return RFCMP_OK;
  RF_TRY(upload(S, 5, dU));
  RF_TRY(tsmm_c128(W.r, nr, dU, p, N, W.p, 1.0, false, s));
  int it = 0;
  while (it < maxit) {
    RF_TRY(apply_batch(D, W, W.p, W.q, p));   // Q = A P
    ++it;
    RF_TRY(gram_c128(W.p, p, W.q, p, N, dslot[0], gscr, gbytes, s));
    RF_TRY(gram_c128(W.p, p, W.r, nr, N, dslot[1], gscr, gbytes, s));
    RF_TRY(wait());
    read(0, p * p, M);
    for (int i = 0; i < p; ++i)  // Hermitian part (the products are Hermitian to rounding)
      for (int j = 0; j <= i; ++j) {
        const cplx h = 0.5 * (M[i * p + j] + std::conj(M[j * p + i]));
        M[i * p + j] = h;
        M[j * p + i] = std::conj(h);
      }
    read(1, p * nr, C2);
    if (!hpd_factor(M, p, Lm)) {
      set_error("block CG breakdown at iteration %d: P^H A P not positive definite", it);
      return RFCMP_E_BREAKDOWN;
    }
    hpd_subst(Lm, p, C2, nr, A1);
    RF_TRY(upload(A1, 3, dS));
    RF_TRY(tsmm_c128(W.p, p, dS, nr, N, W.x, 1.0, true, s));    // X += P alpha
    RF_TRY(tsmm_c128(W.q, p, dS, nr, N, W.r, -1.0, true, s));   // R -= Q alpha
    RF_TRY(dot(N, W.r, W.r, W.part, W.dout, nr, s, nullptr, drn));
    RF_TRY(gram_c128(W.q, p, W.r, nr, N, dslot[2], gscr, gbytes, s));
    RF_TRY(wait());
    take_norms();
    for (int r = 0; r < nr; ++r) iters[r] = it;
    if (done() || it >= maxit) break;
    // Y = R - P M^-1 Q^H R into W.q (Q is not needed any more)
    read(2, p * nr, C3);
    hpd_subst(Lm, p, C3, nr, T);
    RF_TRY(upload(T, 4, dT));
    RF_HIP(hipMemcpyAsync(W.q, W.r, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
    RF_TRY(tsmm_c128(W.p, p, dT, nr, N, W.q, -1.0, true, s));
    // P = Y S, orthonormal
    RF_TRY(gram_c128(W.q, nr, W.q, nr, N, dslot[0], gscr, gbytes, s));
    RF_TRY(wait());
    read(0, nr * nr, G);
    p = orth_transform(G, nr, kDrop, S);
    if (p == 0) break;
    RF_TRY(upload(S, 5, dU));
    RF_TRY(tsmm_c128(W.q, nr, dU, p, N, W.p, 1.0, false, s));
  }
  return RFCMP_OK;
}

// Reduction the inner BF16x3 solve aims for in one round.  Deeper inner
// solves (down to the products' own accuracy, about 1e-7) cost more Krylov
// iterations than the FP64 residual and restart they save: on the level-5
// sphere with 64 waves, 26 iterations against 21 in two rounds.
constexpr double kInnerReduction = 1e-4;
// The round that can finish aims at this fraction of the tolerance: the gap
// between the inner solve's recursive residual and the true one is the
// BF16x3 product error times that round's correction (about 1e-4 of the
// first round's), and the measured true residuals stay below 0.7 of the
// target (level-4 and level-5 spheres, the 96 x 48 torus; at 0.9 the torus
// ended at 0.9 of the tolerance).
constexpr double kFinalTarget = 0.75;

rfcmp_status solve_batch(rfcmp_op op, const double2* e, double2* j, int nr, double tol, int maxit, hipStream_t s,
                         rfcmp_info* info, bool system = false, const double2* sv = nullptr,
                         double2* js = nullptr) {
  const int64_t N = op->mesh->h.N;
  const int64_t NR = (int64_t)nr * N;
  const Work W = carve(op);
  const Dense D64{op, s, false, &W};
  const Dense D16{op, s, true, &W};
  const bool split = op->opt.precision == 1;
  if (system)
    RF_HIP(hipMemcpyAsync(W.b0, e, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  else if (sv)
    RF_TRY(rhs_batch_split(D64, W, sv, e, W.b0, nr));
  else
    RF_TRY(rhs_batch(D64, W, e, W.b0, nr));
  RF_HIP(hipMemcpyAsync(W.b, W.b0, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  RF_HIP(hipMemsetAsync(W.d, 0, sizeof(double2) * NR, s));  // accumulated solution
  RF_TRY(dot(N, W.b, W.b, W.part, W.dout, nr, s));
  std::vector<double2> hd(nr);
  RF_HIP(hipMemcpyAsync(hd.data(), W.dout, sizeof(double2) * nr, hipMemcpyDeviceToHost, s));
  RF_HIP(hipStreamSynchronize(s));
  std::vector<double> bn(nr), res(nr), target(nr), rel(nr, 1.0);
  for (int r = 0; r < nr; ++r) res[r] = bn[r] = std::sqrt(hd[r].x);
  std::vector<int> its(nr, 0), tot(nr, 0), rst(nr, -1);
  std::vector<double> cond(nr, 0.0);
  rfcmp_status st = RFCMP_OK;
  bool zero = true;
  for (int r = 0; r < nr; ++r) zero &= !(bn[r] > 0);
  for (int round = 0; round < 40 && !zero; ++round) {
    for (int r = 0; r < nr; ++r)
      target[r] = split ? std::max(kInnerReduction * res[r], kFinalTarget * tol * bn[r]) : tol * bn[r];
    int budget = maxit;
    for (int r = 0; r < nr; ++r) budget = std::min(budget, maxit - tot[r]);
    if (budget <= 0) {
      st = RFCMP_W_NOT_CONVERGED;
      break;
    }
    if ((op->opt.block_cg == 1 && nr > 1) || (op->opt.block_cg == -1 && nr >= kBlockAutoRhs))
      RF_TRY(block_cg_shared(split ? D16 : D64, W, nr, target.data(), budget, its.data()));
    else
      RF_TRY(block_cg(split ? D16 : D64, W, nr, target.data(), budget, its.data(),
                      round == 0 ? cond.data() : nullptr));
    for (int r = 0; r < nr; ++r) {
      tot[r] += its[r];
      rst[r] += 1;
    }
    RF_TRY(vadd_to(NR, W.x, W.d, s));
    // true residual of the stored operator, FP64-accumulated
    RF_TRY(apply_batch(D64, W, W.d, W.q, nr));
    RF_TRY(vsub(NR, W.b0, W.q, W.b, s));
    RF_TRY(dot(N, W.b, W.b, W.part, W.dout, nr, s));
    RF_HIP(hipMemcpyAsync(hd.data(), W.dout, sizeof(double2) * nr, hipMemcpyDeviceToHost, s));
    RF_HIP(hipStreamSynchronize(s));
    bool all = true, exhausted = false;
    for (int r = 0; r < nr; ++r) {
      res[r] = std::sqrt(hd[r].x);
      rel[r] = bn[r] > 0 ? res[r] / bn[r] : 0.0;
      if (!(rel[r] <= tol)) {
        all = false;
        exhausted |= tot[r] >= maxit;
      }
    }
    if (all) break;
    if (exhausted || round == 39) {
      st = RFCMP_W_NOT_CONVERGED;
      break;
    }
  }
  if (info)
    for (int r = 0; r < nr; ++r) {
      info[r].iters = tot[r];
      info[r].restarts = std::max(rst[r], 0);
      info[r].rel_residual = zero ? 0.0 : rel[r];
      info[r].cond_estimate = cond[r];
    }
  if (system)
    RF_HIP(hipMemcpyAsync(j, W.d, sizeof(double2) * NR, hipMemcpyDeviceToDevice, s));
  else
    RF_TRY(recover_batch(D64, W, W.d, j, nr, js));
  return st;
}

// The mesh arrays on the device, and for the dense projectors (projector
// option 1) their inverses, enqueued on internal streams.  The sparse
// factors are joined and uploaded by mesh_sparse_projectors once the caller
// has queued its own work.
rfcmp_status ensure_mesh_device(rfcmp_mesh m, bool need_gtp, bool dense, hipStream_t s) {
  if (!m->d.uploaded) {
    RF_TRY(mesh_upload(m, s));
    m->d.uploaded = true;
  }
  if (!dense) return RFCMP_OK;
  if (!m->d.ready) {
    RF_TRY(mesh_projectors(m, need_gtp, s));
    m->d.ready = true;
  } else if (need_gtp && !m->d.has_gtp) {
    RF_TRY(mesh_projectors(m, true, s));
  }
  return RFCMP_OK;
}

// Everything the operator's projectors need before its first product on s.
rfcmp_status ready_projectors(rfcmp_op op, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  if (op->opt.projector == kProjSparse) {
    RF_TRY(mesh_sparse_projectors(m, op->opt.outer_star == 1));
    RF_TRY(ensure_sp_scratch(op));
  }
  return wait_projectors(m, s);
}

// BF16x3 planes of the operator's blocks (the projector matrices stay FP64;
// rfcmp_matvec builds their planes on demand).
rfcmp_status ensure_split(rfcmp_op op, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  const MeshHost& h = m->h;
  if (!op->TA16) {
    op->TA16 = std::make_unique<SplitMatrix>();
    RF_TRY(op->TA16->from_c64(op->TA.as<float2>(), h.N, op->ldA, kTriBlock, s));
    op->V16 = std::make_unique<SplitMatrix>();
    RF_TRY(op->V16->from_c64(op->Vb.as<float2>(), h.C, op->ldV, 0, s));
  }
  const size_t need = gemm_scratch_bytes(std::max(h.N, std::max(h.C, h.V)), 64);
  if (op->gemm_scratch.bytes < need) RF_TRY(op->gemm_scratch.alloc(need));
  return RFCMP_OK;
}

bool unit(const double* v) {
  const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  return std::fabs(n - 1.0) <= 1e-12;
}

}  // namespace
}  // namespace rfcmp

namespace rfcmp {
namespace {
struct ProfState {
  std::mutex mu;  // calls on different operators may run on several host threads
  bool on = false;
  std::vector<std::string> only;  // empty: every tag
  std::vector<hipEvent_t> pool;  // all events ever created (reused)
  size_t next = 0;
  std::vector<std::tuple<std::string, hipEvent_t, hipEvent_t>> rec;
};
ProfState& prof() {
  static ProfState p;
  return p;
}
}  // namespace
bool profiling_enabled() { return prof().on; }
const char* profile_tag_suffix(const char* tag, int k) {
  static std::mutex mu;
  static std::set<std::string> names;
  std::lock_guard<std::mutex> g(mu);
  return names.insert(std::string(tag) + "_nr" + std::to_string(k)).first->c_str();
}
bool profiling_selected(const char* tag) {
  const ProfState& p = prof();
  if (p.only.empty()) return true;
  for (const auto& t : p.only)
    if (t == tag) return true;
  return false;
}
hipEvent_t profile_event() {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (p.next == p.pool.size()) {
    hipEvent_t e;
    // timing only: no system-scope fence (cache write-back) at each record,
    // which would stall the stream around every timed launch
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    p.pool.push_back(e);
  }
  return p.pool[p.next++];
}
void profile_record(const char* tag, hipEvent_t a, hipEvent_t b) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.rec.emplace_back(tag, a, b);
}

// Concurrent work of rfcmp_batch_solve and rfcmp_op_create_many: at most one
// stream per hardware queue HIP gives a process by default.
constexpr int kBatchStreams = 4;

// job(q, stream) for every q of `order`, on up to max_streams internal
// streams (non-blocking, default priority), each driven by a host thread of
// its own that takes the next q when its job returns.  The streams start
// after the work queued on s, and s waits for them.  status[q] and msg[q]
// receive each job's status and error text; the return value reports the
// streams' own set-up.  Jobs must not share mutable state.
template <class F>
rfcmp_status run_concurrent(const std::vector<int>& order, int max_streams, hipStream_t s, F job,
                            std::vector<rfcmp_status>& status, std::vector<std::string>& msg) {
  const int count = (int)order.size();
  status.assign(count, RFCMP_OK);
  msg.assign(count, std::string());
  if (count == 0) return RFCMP_OK;
  int dev = 0;
  RF_HIP(hipGetDevice(&dev));
  const int nw = std::max(1, std::min({count, max_streams, kBatchStreams}));
  struct Streams {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> ev;
    ~Streams() {
      for (hipStream_t x : s) (void)hipStreamDestroy(x);
      for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    }
  } W;
  for (int w = 0; w <= nw; ++w) {
    hipEvent_t ev = nullptr;
    RF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    W.ev.push_back(ev);
  }
  for (int w = 0; w < nw; ++w) {
    hipStream_t x = nullptr;
    RF_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    W.s.push_back(x);
  }
  RF_HIP(hipEventRecord(W.ev[nw], s));
  for (int w = 0; w < nw; ++w) RF_HIP(hipStreamWaitEvent(W.s[w], W.ev[nw], 0));
  std::atomic<int> next{0};
  auto worker = [&](int w) {
    const bool on_device = hipSetDevice(dev) == hipSuccess;
    for (int t; (t = next.fetch_add(1)) < count;) {
      const int q = order[t];
      if (!on_device) {
        status[q] = RFCMP_E_HIP;
        msg[q] = "hipSetDevice failed on a worker thread";
        continue;
      }
      status[q] = job(q, W.s[w]);
      if (status[q] < 0) msg[q] = last_error();
    }
  };
  std::vector<std::thread> threads;
  for (int w = 1; w < nw; ++w) threads.emplace_back(worker, w);
  worker(0);
  for (std::thread& t : threads) t.join();
  for (int w = 0; w < nw; ++w) {
    RF_HIP(hipEventRecord(W.ev[w], W.s[w]));
    RF_HIP(hipStreamWaitEvent(s, W.ev[w], 0));
  }
  return RFCMP_OK;
}
}  // namespace rfcmp

using namespace rfcmp;

#define RF_ARG(cond, msg)              \
  do {                                 \
    if (!(cond)) {                     \
      set_error("%s", msg);            \
      return RFCMP_E_ARG;              \
    }                                  \
  } while (0)

extern "C" {

const char* rfcmp_last_error(void) { return rfcmp::last_error(); }
const char* rfcmp_version(void) { return "rfcmp 0.1 (gfx950)"; }

rfcmp_status rfcmp_profile_enable(int32_t on) {
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (auto& r : p.rec) (void)hipEventSynchronize(std::get<2>(r));
  p.rec.clear();
  p.next = 0;
  p.on = on != 0;
  return RFCMP_OK;
}

rfcmp_status rfcmp_profile_select(const char* tags) {
  ProfState& p = prof();
  p.only.clear();
  if (!tags) return RFCMP_OK;
  std::string cur;
  for (const char* c = tags;; ++c) {
    if (*c == ',' || *c == 0) {
      if (!cur.empty()) p.only.push_back(cur);
      cur.clear();
      if (*c == 0) break;
    } else {
      cur += *c;
    }
  }
  return RFCMP_OK;
}

rfcmp_status rfcmp_profile_read(const char* tag, double* total_ms, int64_t* launches) {
  RF_ARG(tag && total_ms && launches, "NULL argument");
  double t = 0.0;
  int64_t n = 0;
  ProfState& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (auto& r : p.rec) {
    if (std::get<0>(r) != tag) continue;
    RF_HIP(hipEventSynchronize(std::get<2>(r)));
    float ms = 0.f;
    RF_HIP(hipEventElapsedTime(&ms, std::get<1>(r), std::get<2>(r)));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return RFCMP_OK;
}

rfcmp_status rfcmp_mesh_create(const double* xyz, int64_t nv, const int32_t* tri, int64_t nc, rfcmp_mesh* out) {
  RF_ARG(out, "out is NULL");
  *out = nullptr;
  auto m = std::make_unique<rfcmp_mesh_s>();
  RF_TRY(build_mesh_host(xyz, nv, tri, nc, m->h));
  // the near-pair list of the default factor, on a host thread beside
  // whatever the caller does next (the projector builds, at the latest)
  rfcmp_options o;
  rfcmp_options_default(&o);
  try {
    const MeshHost* hp = &m->h;
    const double f = o.near_factor;
    m->near_async = std::async(std::launch::async, [hp, f]() {
      NearData v;
      near_data(*hp, f, v);
      return v;
    });
    m->near_async_factor = f;
  } catch (const std::exception&) {
    m->near_async_factor = -1.0;  // computed when first needed
  }
  // the sparse factors of L and G_ll on two more host threads (joined when
  // an operator first needs them), where the automatic projector choice
  // takes them; for smaller meshes they are factored on the calling thread
  // if an operator asks for them, so that the host threads of a batch of
  // small meshes do not compete with the threads that drive its solves
  if (m->h.C > kAutoSparseCells) {
    try {
      const MeshHost* hp = &m->h;
      for (int q = 0; q < 2; ++q)
        m->fac_async[q] = std::async(std::launch::async, [hp, q]() { return factor_mesh_matrix(*hp, q); });
    } catch (const std::exception&) {
      // factored on the calling thread when first needed
    }
  }
  *out = m.release();
  return RFCMP_OK;
}

rfcmp_status rfcmp_mesh_sizes(rfcmp_mesh m, int64_t* N, int64_t* V, int64_t* C, int32_t* genus) {
  RF_ARG(m, "mesh is NULL");
  if (N) *N = m->h.N;
  if (V) *V = m->h.V;
  if (C) *C = m->h.C;
  if (genus) *genus = m->h.genus;
  return RFCMP_OK;
}

rfcmp_status rfcmp_mesh_edges(rfcmp_mesh m, int32_t* ev, int32_t* ec, int32_t* el) {
  RF_ARG(m, "mesh is NULL");
  const size_t n = 2 * size_t(m->h.N);
  if (ev) std::memcpy(ev, m->h.edge_vtx.data(), n * sizeof(int32_t));
  if (ec) std::memcpy(ec, m->h.edge_cell.data(), n * sizeof(int32_t));
  if (el) std::memcpy(el, m->h.edge_local.data(), n * sizeof(int32_t));
  return RFCMP_OK;
}

rfcmp_status rfcmp_mesh_near_pairs(rfcmp_mesh m, double f, int64_t* count, int32_t* pairs) {
  RF_ARG(m && count, "mesh or count is NULL");
  RF_ARG(std::isfinite(f) && f > 0, "near_factor must be > 0");
  std::vector<int32_t> p;
  near_pairs(m->h, f, p);
  *count = int64_t(p.size() / 2);
  if (pairs) std::memcpy(pairs, p.data(), p.size() * sizeof(int32_t));
  return RFCMP_OK;
}

rfcmp_status rfcmp_mesh_factor_info(rfcmp_mesh m, int32_t which, int64_t* n, int32_t* supernodes, int32_t* levels,
                                    int64_t* stored, double* seconds) {
  RF_ARG(m && which >= 0 && which <= 2, "NULL mesh or which outside 0..2");
  const SpDevice* F = m->d.sp[which].get();
  if (!F) {
    set_error("sparse factor %d has not been built for this mesh", which);
    return RFCMP_E_STATE;
  }
  if (n) *n = F->n;
  if (supernodes) *supernodes = F->nsn;
  if (levels) *levels = F->ntop + (F->nsub > 0 ? 1 : 0);
  if (stored) *stored = F->nnz;
  if (seconds) *seconds = F->seconds;
  return RFCMP_OK;
}

void rfcmp_mesh_destroy(rfcmp_mesh m) { delete m; }

rfcmp_status rfcmp_options_default(rfcmp_options* o) {
  RF_ARG(o, "options is NULL");
  o->near_factor = 2.0;
  o->outer_star = 0;
  o->scaling = 0;
  o->power_iters = 30;
  o->precision = 0;
  o->power_tol = 1e-2;
  o->streams = kBatchStreams;
  o->projector = 0;
  o->graphs = 0;
  o->aca_tol = 0.0;
  o->block_cg = -1;
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_create(rfcmp_mesh m, double k, const rfcmp_options* opt, const void* power_start,
                             void* stream, rfcmp_op* out) {
  RF_ARG(out, "out is NULL");
  *out = nullptr;
  return rfcmp_op_create_many(m, &k, 1, opt, power_start, stream, out);
}

rfcmp_status rfcmp_op_create_many(rfcmp_mesh m, const double* k, int32_t nk, const rfcmp_options* opt,
                                  const void* power_start, void* stream, rfcmp_op* out) {
  RF_ARG(out, "out is NULL");
  RF_ARG(k && nk > 0 && nk <= 1024, "need 1 to 1024 wavenumbers");
  for (int32_t i = 0; i < nk; ++i) out[i] = nullptr;
  RF_ARG(m, "mesh is NULL");
  for (int32_t i = 0; i < nk; ++i) RF_ARG(std::isfinite(k[i]) && k[i] > 0, "wavenumber must be finite and > 0");
  rfcmp_options o;
  rfcmp_options_default(&o);
  if (opt) o = *opt;
  RF_ARG(std::isfinite(o.near_factor) && o.near_factor > 0, "near_factor must be > 0");
  RF_ARG(o.outer_star == 0 || o.outer_star == 1, "outer_star must be 0 or 1");
  RF_ARG(o.scaling == 0 || o.scaling == 1, "scaling must be 0 or 1");
  RF_ARG(o.precision == 0 || o.precision == 1, "precision must be 0 or 1");
  RF_ARG(o.scaling == 1 || (o.power_iters > 0 && power_start), "power scalings need power_iters > 0 and power_start");
  RF_ARG(std::isfinite(o.power_tol) && o.power_tol >= 0, "power_tol must be >= 0");
  RF_ARG(o.streams >= 1 && o.streams <= kBatchStreams, "streams must be 1..4");
  RF_ARG(o.projector >= 0 && o.projector <= 2, "projector must be 0, 1 or 2");
  RF_ARG(o.graphs == 0 || o.graphs == 1, "graphs must be 0 or 1");
  RF_ARG(std::isfinite(o.aca_tol) && o.aca_tol >= 0 && o.aca_tol < 1, "aca_tol must be in [0, 1)");
  RF_ARG(o.aca_tol == 0 || o.precision == 0, "compressed blocks (aca_tol > 0) need precision 0");
  RF_ARG(o.block_cg >= -1 && o.block_cg <= 1, "block_cg must be -1, 0 or 1");
  if (o.projector == kProjAuto) o.projector = m->h.C > kAutoSparseCells ? kProjSparse : kProjDense;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  RF_HIP(hipGetDevice(&dev));
  if (m->device >= 0 && m->device != dev) {
    set_error("mesh device data live on device %d, current device is %d", m->device, dev);
    return RFCMP_E_STATE;
  }
  RF_TRY(ensure_mesh_device(m, o.outer_star == 1, o.projector == kProjDense, s));
  m->device = dev;
  const int64_t N = m->h.N, C = m->h.C, V = m->h.V;
  std::vector<std::unique_ptr<rfcmp_op_s>> ops(nk);
  // Every operator's blocks first: their assembly runs beside the projector
  // builds of a new mesh, which the scalings then wait for.
  for (int32_t i = 0; i < nk; ++i) {
    auto& op = ops[i];
    op = std::make_unique<rfcmp_op_s>();
    op->mesh = m;
    op->k = k[i];
    op->opt = o;
    op->ldA = (int64_t)round_up(N, 64);
    op->ldV = (int64_t)round_up(C, 64);
    if (o.aca_tol > 0) {
      RF_TRY(hm_mesh_setup(m, s));
      op->hm = std::make_unique<HmOp>();
      op->hm->tol = o.aca_tol;
    } else {
      RF_TRY(op->TA.alloc(sizeof(float2) * N * op->ldA));
      RF_TRY(op->Vb.alloc(sizeof(float2) * C * op->ldV));
    }
    RF_TRY(ensure_work(op.get(), 4));
    RF_TRY(op->symv_scratch.alloc(symv_scratch_bytes(N, 4) + symv_scratch_bytes(C, 4) + symv_scratch_bytes(V, 4)));
    RF_TRY(assemble_blocks(op.get(), s));
  }
  for (int32_t i = 0; i < nk; ++i) RF_TRY(ready_projectors(ops[i].get(), s));
  for (int32_t i = 0; i < nk; ++i) {
    rfcmp_op op = ops[i].get();
    op->alpha = std::sqrt(k[i]);
    op->beta = 1.0 / std::sqrt(k[i]);
    op->gamma = k[i];
    if (o.precision == 1) RF_TRY(ensure_split(op, s));
  }
  // The power iterations of several wavenumbers run concurrently (each
  // operator's own workspace; the mesh's matrices are only read), the
  // highest wavenumber, which takes the most steps, first.
  const double2* start = static_cast<const double2*>(power_start);
  if (o.scaling == 0 && (nk == 1 || o.streams == 1)) {
    for (int i = 0; i < nk; ++i) RF_TRY(power_scalings(ops[i].get(), start, o.power_iters, o.power_tol, s));
  } else if (o.scaling == 0) {
    std::vector<int> order(nk);
    for (int i = 0; i < nk; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return k[a] > k[b]; });
    std::vector<rfcmp_status> status;
    std::vector<std::string> msg;
    RF_TRY(run_concurrent(
        order, o.streams, s,
        [&](int q, hipStream_t ws) { return power_scalings(ops[q].get(), start, o.power_iters, o.power_tol, ws); },
        status, msg));
    for (int i = 0; i < nk; ++i)
      if (status[i] < 0) {
        set_error("wavenumber %d: %s", i, msg[i].c_str());
        return status[i];
      }
  }
  RF_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i < nk; ++i) out[i] = ops[i].release();
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_scalings(rfcmp_op op, double* a, double* b, double* g, double* lam) {
  RF_ARG(op, "op is NULL");
  if (a) *a = op->alpha;
  if (b) *b = op->beta;
  if (g) *g = op->gamma;
  if (lam)
    for (int i = 0; i < 3; ++i) lam[i] = op->lam[i];
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_power_steps(rfcmp_op op, int32_t* steps) {
  RF_ARG(op && steps, "NULL argument");
  *steps = op->power_steps;
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_set_scalings(rfcmp_op op, double a, double b, double g) {
  RF_ARG(op, "op is NULL");
  RF_ARG(std::isfinite(a) && std::isfinite(b) && std::isfinite(g) && a > 0 && b > 0 && g > 0,
         "scalings must be finite and > 0");
  op->alpha = a;
  op->beta = b;
  op->gamma = g;
  return RFCMP_OK;
}

// D [n][n] = the symmetric M stored as the upper triangle of tri-wide
// blocks (entries with k < tri floor(i / tri) read transposed).
__global__ void k_export_tri(const float2* __restrict__ M, long n, long ld, long tri, float2* __restrict__ D) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const long i = t / n, k = t % n;
  D[t] = k < (i / tri) * tri ? M[k * ld + i] : M[i * ld + k];
}

rfcmp_status rfcmp_op_export(rfcmp_op op, void* TA, void* V, void* stream) {
  RF_ARG(op, "op is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = op->mesh->h.N, C = op->mesh->h.C;
  if (op->hm) return hm_export(op, static_cast<float2*>(TA), static_cast<float2*>(V), s);
  if (TA && N > 0) {
    const long tot = (long)N * N;
    hipLaunchKernelGGL(k_export_tri, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, op->TA.as<float2>(),
                       (long)N, (long)op->ldA, (long)kTriBlock, static_cast<float2*>(TA));
    RF_HIP(hipGetLastError());
  }
  if (V)
    RF_HIP(hipMemcpy2DAsync(V, sizeof(float2) * C, op->Vb.p, sizeof(float2) * op->ldV, sizeof(float2) * C, C,
                            hipMemcpyDeviceToDevice, s));
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_compression(rfcmp_op op, int64_t* dense_entries, int64_t* lowrank_entries,
                                  int32_t* lowrank_blocks, int32_t* max_rank, double* mean_rank) {
  RF_ARG(op, "op is NULL");
  if (!op->hm) {
    set_error("operator blocks are dense (options.aca_tol = 0)");
    return RFCMP_E_STATE;
  }
  const HmOp& P = *op->hm;
  int mx = 0;
  double sum = 0.0;
  for (int r : P.hrankA) mx = std::max(mx, r), sum += r;
  for (int r : P.hrankV) mx = std::max(mx, r), sum += r;
  const size_t nb = P.hrankA.size() + P.hrankV.size();
  for (int q = 0; q < 2; ++q) {
    if (dense_entries) dense_entries[q] = P.dense_entries[q];
    if (lowrank_entries) lowrank_entries[q] = P.lr_entries[q];
  }
  if (lowrank_blocks) *lowrank_blocks = (int32_t)P.hrankA.size();
  if (max_rank) *max_rank = mx;
  if (mean_rank) *mean_rank = nb ? sum / (double)nb : 0.0;
  return RFCMP_OK;
}

void rfcmp_op_destroy(rfcmp_op op) { delete op; }

rfcmp_status rfcmp_rhs_planewave(rfcmp_op op, const double* khat, const double* pol, int32_t nrhs, void* e,
                                 void* stream) {
  RF_ARG(op && khat && pol && e, "NULL argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  for (int r = 0; r < nrhs; ++r) {
    RF_ARG(unit(khat + 3 * r) && unit(pol + 3 * r), "khat and pol must be unit vectors (1e-12)");
    const double dp = khat[3 * r] * pol[3 * r] + khat[3 * r + 1] * pol[3 * r + 1] + khat[3 * r + 2] * pol[3 * r + 2];
    RF_ARG(std::fabs(dp) <= 1e-12, "pol must be orthogonal to khat (1e-12)");
  }
  return rhs_planewave(op, khat, pol, nrhs, static_cast<double2*>(e), static_cast<hipStream_t>(stream));
}

rfcmp_status rfcmp_rhs_planewave_split(rfcmp_op op, const double* khat, const double* pol, int32_t nrhs, void* s,
                                       void* e1, void* stream) {
  RF_ARG(op && khat && pol && s && e1 && s != e1, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  for (int r = 0; r < nrhs; ++r) {
    RF_ARG(unit(khat + 3 * r) && unit(pol + 3 * r), "khat and pol must be unit vectors (1e-12)");
    const double dp = khat[3 * r] * pol[3 * r] + khat[3 * r + 1] * pol[3 * r + 1] + khat[3 * r + 2] * pol[3 * r + 2];
    RF_ARG(std::fabs(dp) <= 1e-12, "pol must be orthogonal to khat (1e-12)");
  }
  return rhs_planewave(op, khat, pol, nrhs, static_cast<double2*>(e1), static_cast<hipStream_t>(stream),
                       static_cast<double2*>(s));
}

rfcmp_status rfcmp_rhs_planewave_noalloc(rfcmp_op op, const double* khat, const double* pol, int32_t nrhs,
                                         void* e, void* stream) {
  RF_ARG(op && khat && pol && e, "NULL argument");
  RF_ARG(nrhs > 0 && nrhs <= RFCMP_RHS_NOALLOC_MAX, "nrhs must be in [1, RFCMP_RHS_NOALLOC_MAX]");
  for (int r = 0; r < nrhs; ++r) {
    RF_ARG(unit(khat + 3 * r) && unit(pol + 3 * r), "khat and pol must be unit vectors (1e-12)");
    const double dp = khat[3 * r] * pol[3 * r] + khat[3 * r + 1] * pol[3 * r + 1] + khat[3 * r + 2] * pol[3 * r + 2];
    RF_ARG(std::fabs(dp) <= 1e-12, "pol must be orthogonal to khat (1e-12)");
  }
  return rhs_planewave_noalloc(op, khat, pol, nrhs, static_cast<double2*>(e), static_cast<hipStream_t>(stream));
}

rfcmp_status rfcmp_rhs_gap(rfcmp_mesh m, const int32_t* edges, const void* volts, int32_t ngap, int32_t nrhs,
                           void* e, void* stream) {
  RF_ARG(m && e, "NULL argument");
  RF_ARG(nrhs > 0 && nrhs <= 65535 && ngap >= 0 && ngap <= (1 << 20), "nrhs must be in [1, 65535], ngap in [0, 2^20]");
  RF_ARG(ngap == 0 || (edges && volts), "NULL edges or volts");
  RF_ARG((int64_t)ngap * nrhs <= (int64_t)1 << 26, "at most 2^26 gaps in all");
  for (int64_t t = 0; t < (int64_t)ngap * nrhs; ++t)
    RF_ARG(edges[t] >= 0 && edges[t] < m->h.N, "gap edge index out of range");
  return rhs_gap(m, edges, static_cast<const double2*>(volts), ngap, nrhs, static_cast<double2*>(e),
                 static_cast<hipStream_t>(stream));
}

rfcmp_status rfcmp_farfield(rfcmp_op op, const void* j, int32_t nrhs, const double* dirs, int32_t ndir, void* F,
                            void* rcs, void* stream) {
  RF_ARG(op && j && dirs && F, "NULL argument");
  RF_ARG(nrhs > 0 && ndir > 0 && nrhs <= 65535 && ndir <= (1 << 30), "nrhs and ndir must be > 0");
  for (int d = 0; d < ndir; ++d) RF_ARG(unit(dirs + 3 * d), "directions must be unit vectors (1e-12)");
  return far_field(op, static_cast<const double2*>(j), nullptr, nrhs, dirs, ndir, static_cast<double2*>(F),
                   static_cast<double*>(rcs), static_cast<hipStream_t>(stream));
}

rfcmp_status rfcmp_farfield_split(rfcmp_op op, const void* j_loop, const void* j_star, int32_t nrhs,
                                  const double* dirs, int32_t ndir, void* F, void* rcs, void* stream) {
  RF_ARG(op && j_loop && j_star && dirs && F, "NULL argument");
  RF_ARG(nrhs > 0 && ndir > 0 && nrhs <= 65535 && ndir <= (1 << 30), "nrhs and ndir must be > 0");
  for (int d = 0; d < ndir; ++d) RF_ARG(unit(dirs + 3 * d), "directions must be unit vectors (1e-12)");
  return far_field(op, static_cast<const double2*>(j_loop), static_cast<const double2*>(j_star), nrhs, dirs, ndir,
                   static_cast<double2*>(F), static_cast<double*>(rcs), static_cast<hipStream_t>(stream));
}

rfcmp_status rfcmp_precond_rhs(rfcmp_op op, const void* e, void* b, int32_t nrhs, void* stream) {
  RF_ARG(op && e && b && e != b, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RF_TRY(ensure_work(op, std::min(nrhs, 64)));
  const Work W = carve(op);
  const Dense D{op, s, false, &W};
  return batched(nrhs, W.R, N, N, static_cast<const double2*>(e), static_cast<double2*>(b),
                 [&](const double2* x, double2* y, int nr) { return rhs_batch(D, W, x, y, nr); });
}

rfcmp_status rfcmp_apply(rfcmp_op op, const void* x, void* y, int32_t nrhs, void* stream) {
  RF_ARG(op && x && y && x != y, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RF_TRY(ensure_work(op, std::min(nrhs, 64)));
  const Work W = carve(op);
  const Dense D{op, s, false, &W};
  return batched(nrhs, W.R, N, N, static_cast<const double2*>(x), static_cast<double2*>(y),
                 [&](const double2* a, double2* b, int nr) { return apply_batch(D, W, a, b, nr); });
}

rfcmp_status rfcmp_recover(rfcmp_op op, const void* i, void* j, int32_t nrhs, void* stream) {
  RF_ARG(op && i && j && i != j, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RF_TRY(ensure_work(op, std::min(nrhs, 64)));
  const Work W = carve(op);
  const Dense D{op, s, false, &W};
  return batched(nrhs, W.R, N, N, static_cast<const double2*>(i), static_cast<double2*>(j),
                 [&](const double2* a, double2* b, int nr) { return recover_batch(D, W, a, b, nr); });
}

rfcmp_status rfcmp_project(rfcmp_op op, int32_t which, const void* xv, void* yv, int32_t nrhs, void* stream) {
  RF_ARG(op && xv && yv && xv != yv, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  RF_ARG(which >= 0 && which <= 6, "unknown projector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rfcmp_mesh m = op->mesh;
  if (which == RFCMP_PROJ_GSIGMA) {
    RF_TRY(ensure_mesh_device(m, true, op->opt.projector == kProjDense, s));
    if (op->opt.projector == kProjSparse) RF_TRY(mesh_sparse_projectors(m, true));
    RF_TRY(wait_projectors(m, s));
  }
  RF_TRY(ensure_sp_scratch(op));
  const MeshDev& d = m->d;
  const int64_t N = m->h.N, C = m->h.C, V = m->h.V;
  const int64_t nin = (which == RFCMP_PROJ_LPINV) ? C : (which == RFCMP_PROJ_GLL_INV ? V : N);
  const int64_t nout = (which <= RFCMP_PROJ_GSIGMA) ? N : (which == RFCMP_PROJ_LAMBDA_T || which == RFCMP_PROJ_GLL_INV ? V : C);
  RF_TRY(ensure_work(op, std::min(nrhs, 64)));
  const Work W = carve(op);
  const Dense D{op, s, false, &W};
  return batched(nrhs, W.R, nin, nout, static_cast<const double2*>(xv), static_cast<double2*>(yv),
                 [&](const double2* x, double2* y, int nr) -> rfcmp_status {
                   switch (which) {
                     case RFCMP_PROJ_SIGMA:
                     case RFCMP_PROJ_LH:
                       RF_TRY(D.prod(kLP, false, D.sigma_t(x), W.c[1], nr));
                       return which == RFCMP_PROJ_SIGMA
                                  ? axpy_sigma(d, N, C, 0.0, false, nullptr, 1.0, W.c[1], y, nr, s)
                                  : axpy_sigma(d, N, C, 1.0, false, x, -1.0, W.c[1], y, nr, s);
                     case RFCMP_PROJ_GSIGMA:
                       RF_TRY(D.prod(kGTP, false, D.sigma_t(x), W.c[2], nr));
                       RF_TRY(D.prod(kLP, false, W.c[2], W.c[1], nr));
                       return axpy_sigma(d, N, C, 0.0, false, nullptr, 1.0, W.c[1], y, nr, s);
                     case RFCMP_PROJ_LPINV:
                       return D.prod(kLP, false, x, y, nr);
                     case RFCMP_PROJ_GLL_INV:
                       return D.prod(kGLL, false, x, y, nr);
                     case RFCMP_PROJ_SIGMA_T:
                       return sigma_t(d, C, N, x, y, nr, s);
                     default:
                       return lambda_t(d, V, N, x, y, nr, s);
                   }
                 });
}

rfcmp_status rfcmp_matvec(rfcmp_op op, int32_t which, int32_t conj, const void* x, void* y, int32_t nrhs,
                          void* stream) {
  RF_ARG(op && x && y && x != y, "NULL or aliased argument");
  RF_ARG(nrhs > 0 && which >= 0 && which <= 5, "bad which/nrhs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double2* xx = static_cast<const double2*>(x);
  double2* yy = static_cast<double2*>(y);
  if (op->hm) {
    if (which > 1) {
      set_error("operator with compressed blocks: BF16x3 products (which 2-5) are not available");
      return RFCMP_E_STATE;
    }
    return hm_matvec(op, which, conj != 0, xx, yy, nrhs, s);
  }
  if (which <= 1 && nrhs >= kZgemmMinRhs) {
    RF_TRY(ensure_z_scratch(op));
    return which == 0 ? zgemm_c64(op->TA.as<float2>(), op->mesh->h.N, op->ldA, conj != 0, xx, yy, nrhs,
                                  op->z_scratch.p, op->z_scratch.bytes, s, "zgemm_ta")
                      : zgemm_c64(op->Vb.as<float2>(), op->mesh->h.C, op->ldV, conj != 0, xx, yy, nrhs,
                                  op->z_scratch.p, op->z_scratch.bytes, s, "zgemm_v");
  }
  if (which == 0)
    return csymv(op->TA.as<float2>(), op->mesh->h.N, op->ldA, conj != 0, xx, yy, nrhs, op->symv_scratch.p,
                 op->symv_scratch.bytes, s, "cmatvec_ta");
  if (which == 1)
    return csymv(op->Vb.as<float2>(), op->mesh->h.C, op->ldV, conj != 0, xx, yy, nrhs, op->symv_scratch.p,
                 op->symv_scratch.bytes, s, "cmatvec_v");
  RF_TRY(ensure_split(op, s));
  RF_TRY(ensure_work(op, 4));
  const Work W = carve(op);
  const Dense D{op, s, true, &W};
  switch (which) {
    case 2: return D.prod(kTA, conj != 0, xx, yy, nrhs);
    case 3: return D.prod(kV, conj != 0, xx, yy, nrhs);
    default: break;
  }
  // BF16x3 products of the dense inverses: built for this mesh on first use
  // when the operator applies the sparse factors
  rfcmp_mesh m = op->mesh;
  RF_TRY(ensure_mesh_device(m, false, true, s));
  RF_TRY(wait_projectors(m, s));
  MeshDev& d = m->d;
  if (!d.Lp16) {
    d.Lp16 = std::make_unique<SplitMatrix>();
    RF_TRY(d.Lp16->from_f64(d.Lp.as<double>(), m->h.C, d.ldL, s));
    d.Gll16 = std::make_unique<SplitMatrix>();
    RF_TRY(d.Gll16->from_f64(d.Gll_inv.as<double>(), m->h.V, d.ldG, s));
  }
  return gemm_bf16x3(which == 4 ? *d.Lp16 : *d.Gll16, false, xx, yy, nrhs, op->gemm_scratch.p,
                     op->gemm_scratch.bytes, s, which == 4 ? "gemm_lp" : "gemm_gll");
}

static rfcmp_status solve_common(rfcmp_op op, const void* e, void* j, int32_t nrhs, double tol, int32_t maxit,
                                 void* stream, rfcmp_info* info, bool system, const void* sv = nullptr,
                                 void* js = nullptr) {
  RF_ARG(op && e && j && e != j, "NULL or aliased argument");
  RF_ARG(!js || (js != j && js != e && js != sv), "aliased argument");
  RF_ARG(nrhs > 0 && maxit > 0 && std::isfinite(tol) && tol > 0, "bad nrhs/maxit/tol");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = op->mesh->h.N;
  const auto t0 = std::chrono::steady_clock::now();
  RF_TRY(ensure_work(op, std::min(nrhs, 64)));
  if (op->opt.precision == 1) RF_TRY(ensure_split(op, s));
  rfcmp_status worst = RFCMP_OK;
  const int R = op->work_nrhs;
  for (int r0 = 0; r0 < nrhs; r0 += R) {
    const int nr = std::min(R, nrhs - r0);
    const int64_t C = op->mesh->h.C;
    rfcmp_status st = solve_batch(op, static_cast<const double2*>(e) + (int64_t)r0 * N,
                                  static_cast<double2*>(j) + (int64_t)r0 * N, nr, tol, maxit, s,
                                  info ? info + r0 : nullptr, system,
                                  sv ? static_cast<const double2*>(sv) + (int64_t)r0 * C : nullptr,
                                  js ? static_cast<double2*>(js) + (int64_t)r0 * N : nullptr);
    if (st < 0) return st;
    if (st > worst) worst = st;
  }
  RF_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info)
    for (int r = 0; r < nrhs; ++r) info[r].ms_solve = ms;
  return worst;
}

rfcmp_status rfcmp_solve(rfcmp_op op, const void* e, void* j, int32_t nrhs, double tol, int32_t maxit,
                         void* stream, rfcmp_info* info) {
  return solve_common(op, e, j, nrhs, tol, maxit, stream, info, false);
}

rfcmp_status rfcmp_solve_split(rfcmp_op op, const void* s, const void* e1, void* j_loop, void* j_star,
                               int32_t nrhs, double tol, int32_t maxit, void* stream, rfcmp_info* info) {
  RF_ARG(s && j_star, "NULL argument");
  return solve_common(op, e1, j_loop, nrhs, tol, maxit, stream, info, false, s, j_star);
}

rfcmp_status rfcmp_solve_system(rfcmp_op op, const void* b, void* i, int32_t nrhs, double tol, int32_t maxit,
                                void* stream, rfcmp_info* info) {
  return solve_common(op, b, i, nrhs, tol, maxit, stream, info, true);
}

// Several operators' solves at once.  Each is solve_common unchanged, on an
// internal stream of its own driven by a host thread of its own: a CG
// iteration of a small operator is bounded by launch and read-back latency
// rather than by the device, and the solves of the other operators fill
// those gaps.  Largest operators first (at equal size the higher wavenumber),
// so that the last to start are short.
rfcmp_status rfcmp_batch_solve(const rfcmp_op* ops, int32_t nops, const void* const* e, void* const* j,
                               const int32_t* nrhs, double tol, int32_t maxit, void* stream, rfcmp_info* info) {
  RF_ARG(ops && e && j && nrhs && nops > 0, "NULL argument or nops <= 0");
  RF_ARG(maxit > 0 && std::isfinite(tol) && tol > 0, "bad maxit/tol");
  std::vector<int64_t> off(nops + 1, 0);
  for (int q = 0; q < nops; ++q) {
    if (!(ops[q] && e[q] && j[q] && e[q] != j[q] && nrhs[q] > 0)) {
      set_error("operator %d: NULL or aliased argument, or nrhs <= 0", q);
      return RFCMP_E_ARG;
    }
    off[q + 1] = off[q] + nrhs[q];
  }
  {
    std::vector<rfcmp_op> sorted(ops, ops + nops);
    std::sort(sorted.begin(), sorted.end());
    RF_ARG(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(), "an operator appears twice");
  }
  int dev = 0;
  RF_HIP(hipGetDevice(&dev));
  for (int q = 0; q < nops; ++q)
    if (ops[q]->mesh->device != dev) {
      set_error("operator %d lives on device %d, current device is %d", q, ops[q]->mesh->device, dev);
      return RFCMP_E_ARG;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // Workspaces and BF16x3 planes first, on the caller's stream and thread:
  // growing a workspace synchronises the device, and the planes of a mesh
  // that several operators share are built once.  The solves then allocate
  // nothing.
  for (int q = 0; q < nops; ++q) {
    RF_TRY(ensure_work(ops[q], std::min(nrhs[q], 64)));
    if (ops[q]->opt.precision == 1) RF_TRY(ensure_split(ops[q], s));
  }
  std::vector<int> order(nops);
  for (int q = 0; q < nops; ++q) order[q] = q;
  // at equal size the higher wavenumber first: CG takes more iterations there
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int64_t sa = ops[a]->mesh->h.N * nrhs[a], sb = ops[b]->mesh->h.N * nrhs[b];
    return sa != sb ? sa > sb : ops[a]->k > ops[b]->k;
  });
  std::vector<rfcmp_status> status;
  std::vector<std::string> msg;
  RF_TRY(run_concurrent(
      order, kBatchStreams, s,
      [&](int q, hipStream_t ws) {
        return solve_common(ops[q], e[q], j[q], nrhs[q], tol, maxit, ws, info ? info + off[q] : nullptr, false);
      },
      status, msg));
  rfcmp_status worst = RFCMP_OK;
  for (int q = 0; q < nops; ++q) {
    if (status[q] < 0) {
      set_error("operator %d: %s", q, msg[q].c_str());
      return status[q];
    }
    worst = std::max(worst, status[q]);
  }
  return worst;
}

}  // extern "C"
