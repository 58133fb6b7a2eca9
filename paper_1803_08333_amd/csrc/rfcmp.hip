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
#include <chrono>
#include <cmath>
#include <cstring>
#include <tuple>

#include "vecops.h"

namespace rfcmp {
const char* last_error();

namespace {

constexpr int kR = 4;  // right-hand sides per batched operator pass

struct Work {
  double2 *nA, *nB, *nC, *nD;                  // [kR][N]
  double2* c[14];                              // [kR][C]
  double2 *v1, *v2;                            // [kR][V]
  double2 *m1, *m2, *m3;                       // [kR] means
  double2 *part, *dout;                        // reductions
  double2 *cx, *cr, *cp, *cq, *cb;             // CG [N]
  double2 *pv, *pw;                            // power iteration [3][N]
};

size_t work_bytes(int64_t N, int64_t C, int64_t V) {
  const size_t z = sizeof(double2);
  return z * (4 * kR * N + 14 * kR * C + 2 * kR * V + 3 * kR + (dot_partials() + 1) * kR + 5 * N + 6 * N) + 4096;
}

Work carve(rfcmp_op op) {
  const MeshHost& h = op->mesh->h;
  const int64_t N = h.N, C = h.C, V = h.V;
  double2* p = op->work.as<double2>();
  Work w;
  auto take = [&](int64_t n) {
    double2* q = p;
    p += n;
    return q;
  };
  w.nA = take(kR * N); w.nB = take(kR * N); w.nC = take(kR * N); w.nD = take(kR * N);
  for (auto& c : w.c) c = take(kR * C);
  w.v1 = take(kR * V); w.v2 = take(kR * V);
  w.m1 = take(kR); w.m2 = take(kR); w.m3 = take(kR);
  w.part = take((int64_t)dot_partials() * kR);
  w.dout = take(kR);
  w.cx = take(N); w.cr = take(N); w.cp = take(N); w.cq = take(N); w.cb = take(N);
  w.pv = take(3 * N); w.pw = take(3 * N);
  return w;
}

bool use_gsigma(rfcmp_op op) { return op->opt.outer_star == 1; }

// Left half: y = sgn * P_o^H T^H w for w in W.nC with Sig^T w_S in W.c[8].
rfcmp_status left_half(rfcmp_op op, const Work& W, double2* y, int nr, double sgn, hipStream_t s) {
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C;
  const double k = op->k, al = op->alpha, be = op->beta;
  double2 *t5 = W.c[9], *s4 = W.c[10], *vw = W.c[11], *t6 = W.c[12], *g6 = W.c[13];
  RF_TRY(cmatvec(op->TA.as<float2>(), N, op->ldA, true, W.nC, W.nD, nr, s, "cmatvec_ta"));      // zA
  RF_TRY(cmatvec(op->Vb.as<float2>(), C, op->ldV, true, W.c[8], vw, nr, s, "cmatvec_v"));      // vw
  RF_TRY(sigma_t(d, C, N, W.nD, t5, nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t5, s4, nr, s, "dmatvec_lp"));
  RF_TRY(mean(C, vw, W.m3, nr, s));
  RF_TRY(comb_c(C, nullptr, -sgn * (k / be), s4, sgn / (k * be), vw, W.m3, t6, nr, s));
  const double2* gsel = t6;
  if (use_gsigma(op)) {
    RF_TRY(dmatvec(d.Gtp_inv.as<double>(), C, d.ldT, t6, g6, nr, s, "dmatvec_gtp"));
    gsel = g6;
  }
  RF_TRY(left_y(d, N, C, sgn * k / al, W.nD, s4, gsel, y, nr, s));
  return RFCMP_OK;
}

// y = A x for nr <= kR right-hand sides.
rfcmp_status apply_batch(rfcmp_op op, const double2* x, double2* y, int nr, hipStream_t s) {
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C, V = h.V;
  const double k = op->k, al = op->alpha, be = op->beta, ga = op->gamma;
  const Work W = carve(op);
  double2 *t1 = W.c[0], *s1 = W.c[1], *g1 = W.c[2], *s1g = W.c[3], *vphi = W.c[4], *t2 = W.c[5],
          *s2 = W.c[6], *t4 = W.c[7], *sw = W.c[8], *s3 = W.c[9];
  RF_TRY(sigma_t(d, C, N, x, t1, nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t1, s1, nr, s, "dmatvec_lp"));
  const double2* sus = t1;   // Sig^T u_S
  const double2* s_us = s1;  // u_S = Sig s_us
  if (use_gsigma(op)) {
    RF_TRY(dmatvec(d.Gtp_inv.as<double>(), C, d.ldT, t1, g1, nr, s, "dmatvec_gtp"));
    RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, g1, s1g, nr, s, "dmatvec_lp"));
    sus = g1;
    s_us = s1g;
  }
  RF_TRY(vin(d, N, C, k / al, k / be, x, s1, s_us, W.nA, nr, s));
  RF_TRY(cmatvec(op->TA.as<float2>(), N, op->ldA, false, W.nA, W.nB, nr, s, "cmatvec_ta"));   // a
  RF_TRY(cmatvec(op->Vb.as<float2>(), C, op->ldV, false, sus, vphi, nr, s, "cmatvec_v"));     // vphi
  RF_TRY(sigma_t(d, C, N, W.nB, t2, nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t2, s2, nr, s, "dmatvec_lp"));
  RF_TRY(lambda_t(d, V, N, W.nB, W.v1, nr, s));
  RF_TRY(dmatvec(d.Gll_inv.as<double>(), V, d.ldG, W.v1, W.v2, nr, s, "dmatvec_gll"));
  RF_TRY(mean(C, vphi, W.m1, nr, s));
  RF_TRY(comb_c(C, d.area.as<double>(), 1.0, s2, 1.0 / (k * be), vphi, W.m1, t4, nr, s));
  // s3 lives in c[9]: written before left_half reuses that slot as t5
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t4, s3, nr, s, "dmatvec_lp"));
  RF_TRY(middle_w(d, N, C, V, 1.0 / (al * al), 1.0 / ga, 1.0 / (be * be), W.v2, W.nB, s2, s3, W.nC, nr, s));
  RF_TRY(mean(C, t4, W.m2, nr, s));
  RF_TRY(comb_c(C, nullptr, 0.0, nullptr, 1.0 / (be * be), t4, W.m2, sw, nr, s));
  return left_half(op, W, y, nr, 1.0, s);
}

rfcmp_status rhs_batch(rfcmp_op op, const double2* e, double2* b, int nr, hipStream_t s) {
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C, V = h.V;
  const double al = op->alpha, be = op->beta, ga = op->gamma;
  const Work W = carve(op);
  double2 *t2 = W.c[5], *s2 = W.c[6], *t4 = W.c[7], *sw = W.c[8], *s3 = W.c[9];
  RF_TRY(sigma_t(d, C, N, e, t2, nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t2, s2, nr, s, "dmatvec_lp"));
  RF_TRY(lambda_t(d, V, N, e, W.v1, nr, s));
  RF_TRY(dmatvec(d.Gll_inv.as<double>(), V, d.ldG, W.v1, W.v2, nr, s, "dmatvec_gll"));
  RF_TRY(comb_c(C, d.area.as<double>(), 1.0, s2, 0.0, nullptr, nullptr, t4, nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, t4, s3, nr, s, "dmatvec_lp"));
  RF_TRY(middle_w(d, N, C, V, 1.0 / (al * al), 1.0 / ga, 1.0 / (be * be), W.v2, e, s2, s3, W.nC, nr, s));
  RF_TRY(mean(C, t4, W.m2, nr, s));
  RF_TRY(comb_c(C, nullptr, 0.0, nullptr, 1.0 / (be * be), t4, W.m2, sw, nr, s));
  return left_half(op, W, b, nr, -1.0, s);
}

rfcmp_status recover_batch(rfcmp_op op, const double2* x, double2* j, int nr, hipStream_t s) {
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C;
  const Work W = carve(op);
  RF_TRY(sigma_t(d, C, N, x, W.c[0], nr, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[0], W.c[1], nr, s, "dmatvec_lp"));
  const double2* sg = W.c[1];
  if (use_gsigma(op)) {
    RF_TRY(dmatvec(d.Gtp_inv.as<double>(), C, d.ldT, W.c[0], W.c[2], nr, s, "dmatvec_gtp"));
    RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[2], W.c[3], nr, s, "dmatvec_lp"));
    sg = W.c[3];
  }
  return recover_j(d, N, C, 1.0 / op->alpha, 1.0 / op->beta, x, W.c[1], sg, j, nr, s);
}

template <class F>
rfcmp_status batched(int nrhs, int64_t nin, int64_t nout, const double2* x, double2* y, F f) {
  for (int r0 = 0; r0 < nrhs; r0 += kR) {
    const int nr = std::min(kR, nrhs - r0);
    RF_TRY(f(x + (int64_t)r0 * nin, y + (int64_t)r0 * nout, nr));
  }
  return RFCMP_OK;
}

// One power-iteration application of the three scaling operators to the
// normalised rows of W.pv ([3][N]: alpha, gamma, beta), result in W.pw.
//   O_alpha v = P_LH conj(T_A) Lam G_ll^-1 Lam^T T_A P_LH v
//   O_gamma v = P_LH conj(T_A) P_LH T_A P_LH v
//   O_beta  v = P_Sigma T_Phi^H P_mS_hat T_Phi P_Sigma v
//             = Sig conj(V) (I - J) diag(A) (I - J) V Sig^T v
rfcmp_status power_apply(rfcmp_op op, const Work& W, hipStream_t s) {
  const MeshHost& h = op->mesh->h;
  const MeshDev& d = op->mesh->d;
  const int64_t N = h.N, C = h.C, V = h.V;
  double2* va = W.pv;
  double2* vb = W.pv + 2 * N;
  RF_TRY(sigma_t(d, C, N, va, W.c[0], 2, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[0], W.c[1], 2, s, "dmatvec_lp"));
  RF_TRY(axpy_sigma(d, N, C, 1.0, false, va, -1.0, W.c[1], W.nA, 2, s));          // P_LH v
  RF_TRY(cmatvec(op->TA.as<float2>(), N, op->ldA, false, W.nA, W.nB, 2, s, "cmatvec_ta"));
  RF_TRY(lambda_t(d, V, N, W.nB, W.v1, 1, s));
  RF_TRY(dmatvec(d.Gll_inv.as<double>(), V, d.ldG, W.v1, W.v2, 1, s, "dmatvec_gll"));
  RF_TRY(lambda_n(d, N, V, W.v2, W.nC, 1, s));                                   // alpha branch
  RF_TRY(sigma_t(d, C, N, W.nB + N, W.c[2], 1, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[2], W.c[3], 1, s, "dmatvec_lp"));
  RF_TRY(axpy_sigma(d, N, C, 1.0, false, W.nB + N, -1.0, W.c[3], W.nC + N, 1, s));  // gamma branch
  RF_TRY(cmatvec(op->TA.as<float2>(), N, op->ldA, true, W.nC, W.nD, 2, s, "cmatvec_ta"));
  RF_TRY(sigma_t(d, C, N, W.nD, W.c[4], 2, s));
  RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[4], W.c[5], 2, s, "dmatvec_lp"));
  RF_TRY(axpy_sigma(d, N, C, 1.0, false, W.nD, -1.0, W.c[5], W.pw, 2, s));
  // beta
  RF_TRY(sigma_t(d, C, N, vb, W.c[6], 1, s));
  RF_TRY(cmatvec(op->Vb.as<float2>(), C, op->ldV, false, W.c[6], W.c[7], 1, s, "cmatvec_v"));
  RF_TRY(mean(C, W.c[7], W.m1, 1, s));
  RF_TRY(comb_c(C, d.area.as<double>(), 0.0, nullptr, 1.0, W.c[7], W.m1, W.c[8], 1, s));
  RF_TRY(mean(C, W.c[8], W.m2, 1, s));
  RF_TRY(comb_c(C, nullptr, 0.0, nullptr, 1.0, W.c[8], W.m2, W.c[9], 1, s));
  RF_TRY(cmatvec(op->Vb.as<float2>(), C, op->ldV, true, W.c[9], W.c[10], 1, s, "cmatvec_v"));
  RF_TRY(axpy_sigma(d, N, C, 0.0, false, nullptr, 1.0, W.c[10], W.pw + 2 * N, 1, s));
  return RFCMP_OK;
}

rfcmp_status power_scalings(rfcmp_op op, const double2* start, int steps, hipStream_t s) {
  const int64_t N = op->mesh->h.N;
  const Work W = carve(op);
  for (int r = 0; r < 3; ++r)
    RF_HIP(hipMemcpyAsync(W.pw + r * N, start, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
  for (int it = 0; it < steps; ++it) {
    RF_TRY(dot(N, W.pw, W.pw, W.part, W.dout, 3, s));
    RF_HIP(hipMemcpyAsync(W.pv, W.pw, sizeof(double2) * 3 * N, hipMemcpyDeviceToDevice, s));
    RF_TRY(normalize(N, W.dout, W.pv, 3, s));
    RF_TRY(power_apply(op, W, s));
  }
  RF_TRY(dot(N, W.pw, W.pw, W.part, W.dout, 3, s));
  double2 nr2[3];
  RF_HIP(hipMemcpyAsync(nr2, W.dout, sizeof nr2, hipMemcpyDeviceToHost, s));
  RF_HIP(hipStreamSynchronize(s));
  const double la = std::sqrt(nr2[0].x), lg = std::sqrt(nr2[1].x), lb = std::sqrt(nr2[2].x);
  if (!(la > 0) || !(lb > 0) || !(lg > 0) || !std::isfinite(la + lb + lg)) {
    set_error("power iteration produced a non-positive norm (%g, %g, %g)", la, lb, lg);
    return RFCMP_E_STATE;
  }
  const double k = op->k;
  op->lam[0] = la;
  op->lam[1] = lb;
  op->lam[2] = lg;
  op->alpha = std::pow(k * k * la, 0.25);
  op->beta = std::pow(lb / (k * k), 0.25);
  op->gamma = k * k * lg / (op->alpha * op->alpha);
  return RFCMP_OK;
}

// Complex CG on the HPD system for one right-hand side.
rfcmp_status cg_one(rfcmp_op op, const double2* e, double2* j, double tol, int maxit, hipStream_t s,
                    rfcmp_info* info) {
  const int64_t N = op->mesh->h.N;
  const Work W = carve(op);
  double* sc = op->scal.as<double>();  // slots: 0/1 rho ping-pong, 2 pq
  double* hs = op->host_scal;
  RF_TRY(rhs_batch(op, e, W.cb, 1, s));
  RF_TRY(dot(N, W.cb, W.cb, W.part, W.dout, 1, s));
  RF_HIP(hipMemcpyAsync(hs, W.dout, sizeof(double2), hipMemcpyDeviceToHost, s));
  RF_HIP(hipStreamSynchronize(s));
  const double bn = std::sqrt(hs[0]);
  RF_HIP(hipMemsetAsync(W.cx, 0, sizeof(double2) * N, s));
  if (!(bn > 0)) {
    RF_HIP(hipMemsetAsync(j, 0, sizeof(double2) * N, s));
    if (info) *info = rfcmp_info{0, 0, 0.0, 0.0};
    return RFCMP_OK;
  }
  RF_HIP(hipMemcpyAsync(W.cr, W.cb, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
  int it = 0, restarts = -1;
  double rel = 1.0;
  rfcmp_status st = RFCMP_OK;
  while (true) {
    ++restarts;
    RF_HIP(hipMemcpyAsync(W.cp, W.cr, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
    RF_TRY(dot(N, W.cr, W.cr, W.part, W.dout, 1, s));
    RF_TRY(take_real(W.dout, sc, 0, s));
    int cur = 0;
    while (it < maxit) {
      RF_TRY(apply_batch(op, W.cp, W.cq, 1, s));
      RF_TRY(dot(N, W.cp, W.cq, W.part, W.dout, 1, s));
      RF_TRY(take_real(W.dout, sc, 2, s));
      RF_TRY(cg_xr(N, sc, cur, W.cx, W.cr, W.cp, W.cq, s));
      const int nxt = 1 - cur;
      RF_TRY(dot(N, W.cr, W.cr, W.part, W.dout, 1, s));
      RF_TRY(take_real(W.dout, sc, nxt, s));
      RF_HIP(hipMemcpyAsync(hs, sc, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
      RF_HIP(hipStreamSynchronize(s));
      ++it;
      const double pq = hs[2], rho = hs[nxt];
      if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rho)) {
        set_error("CG breakdown at iteration %d: p^H A p = %g", it, pq);
        st = RFCMP_E_BREAKDOWN;
        break;
      }
      if (std::sqrt(rho) / bn <= tol) break;
      RF_TRY(cg_p(N, sc, cur, nxt, W.cr, W.cp, s));
      cur = nxt;
    }
    if (st < 0) break;
    // true residual of the (stored) operator, FP64-accumulated
    RF_TRY(apply_batch(op, W.cx, W.cq, 1, s));
    RF_TRY(vsub(N, W.cb, W.cq, W.cr, s));
    RF_TRY(dot(N, W.cr, W.cr, W.part, W.dout, 1, s));
    RF_HIP(hipMemcpyAsync(hs, W.dout, sizeof(double2), hipMemcpyDeviceToHost, s));
    RF_HIP(hipStreamSynchronize(s));
    rel = std::sqrt(hs[0]) / bn;
    if (rel <= tol) break;
    if (it >= maxit || restarts >= 20) {
      st = RFCMP_W_NOT_CONVERGED;
      break;
    }
  }
  if (info) {
    info->iters = it;
    info->restarts = restarts;
    info->rel_residual = rel;
  }
  if (st < 0) return st;
  RF_TRY(recover_batch(op, W.cx, j, 1, s));
  return st;
}

rfcmp_status ensure_mesh_device(rfcmp_mesh m, bool need_gtp, hipStream_t s) {
  if (!m->d.ready) {
    RF_TRY(mesh_upload(m, s));
    RF_TRY(mesh_projectors(m, need_gtp, s));
    m->d.ready = true;
  } else if (need_gtp && !m->d.has_gtp) {
    RF_TRY(mesh_projectors(m, true, s));
  }
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
  bool on = false;
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
hipEvent_t profile_event() {
  ProfState& p = prof();
  if (p.next == p.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.pool.push_back(e);
  }
  return p.pool[p.next++];
}
void profile_record(const char* tag, hipEvent_t a, hipEvent_t b) { prof().rec.emplace_back(tag, a, b); }
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
  for (auto& r : p.rec) (void)hipEventSynchronize(std::get<2>(r));
  p.rec.clear();
  p.next = 0;
  p.on = on != 0;
  return RFCMP_OK;
}

rfcmp_status rfcmp_profile_read(const char* tag, double* total_ms, int64_t* launches) {
  RF_ARG(tag && total_ms && launches, "NULL argument");
  double t = 0.0;
  int64_t n = 0;
  for (auto& r : prof().rec) {
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

void rfcmp_mesh_destroy(rfcmp_mesh m) { delete m; }

rfcmp_status rfcmp_options_default(rfcmp_options* o) {
  RF_ARG(o, "options is NULL");
  o->near_factor = 2.0;
  o->outer_star = 0;
  o->scaling = 0;
  o->power_iters = 30;
  o->precision = 0;
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_create(rfcmp_mesh m, double k, const rfcmp_options* opt, const void* power_start,
                             void* stream, rfcmp_op* out) {
  RF_ARG(out, "out is NULL");
  *out = nullptr;
  RF_ARG(m, "mesh is NULL");
  RF_ARG(std::isfinite(k) && k > 0, "wavenumber must be finite and > 0");
  rfcmp_options o;
  rfcmp_options_default(&o);
  if (opt) o = *opt;
  RF_ARG(std::isfinite(o.near_factor) && o.near_factor > 0, "near_factor must be > 0");
  RF_ARG(o.outer_star == 0 || o.outer_star == 1, "outer_star must be 0 or 1");
  RF_ARG(o.scaling == 0 || o.scaling == 1, "scaling must be 0 or 1");
  RF_ARG(o.precision == 0 || o.precision == 1, "precision must be 0 or 1");
  RF_ARG(o.scaling == 1 || (o.power_iters > 0 && power_start), "power scalings need power_iters > 0 and power_start");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  RF_HIP(hipGetDevice(&dev));
  if (m->device >= 0 && m->device != dev) {
    set_error("mesh device data live on device %d, current device is %d", m->device, dev);
    return RFCMP_E_STATE;
  }
  RF_TRY(ensure_mesh_device(m, o.outer_star == 1, s));
  m->device = dev;
  auto op = std::make_unique<rfcmp_op_s>();
  op->mesh = m;
  op->k = k;
  op->opt = o;
  const int64_t N = m->h.N, C = m->h.C, V = m->h.V;
  op->ldA = (int64_t)round_up(N, 64);
  op->ldV = (int64_t)round_up(C, 64);
  RF_TRY(op->TA.alloc(sizeof(float2) * N * op->ldA));
  RF_TRY(op->Vb.alloc(sizeof(float2) * C * op->ldV));
  RF_TRY(op->work.alloc(work_bytes(N, C, V)));
  RF_TRY(op->scal.alloc(sizeof(double) * 8));
  RF_HIP(hipHostMalloc((void**)&op->host_scal, sizeof(double) * 8, hipHostMallocDefault));
  RF_TRY(assemble_blocks(op.get(), s));
  op->alpha = std::sqrt(k);
  op->beta = 1.0 / std::sqrt(k);
  op->gamma = k;
  if (o.scaling == 0) RF_TRY(power_scalings(op.get(), static_cast<const double2*>(power_start), o.power_iters, s));
  *out = op.release();
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

rfcmp_status rfcmp_op_set_scalings(rfcmp_op op, double a, double b, double g) {
  RF_ARG(op, "op is NULL");
  RF_ARG(std::isfinite(a) && std::isfinite(b) && std::isfinite(g) && a > 0 && b > 0 && g > 0,
         "scalings must be finite and > 0");
  op->alpha = a;
  op->beta = b;
  op->gamma = g;
  return RFCMP_OK;
}

rfcmp_status rfcmp_op_export(rfcmp_op op, void* TA, void* V, void* stream) {
  RF_ARG(op, "op is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = op->mesh->h.N, C = op->mesh->h.C;
  if (TA)
    RF_HIP(hipMemcpy2DAsync(TA, sizeof(float2) * N, op->TA.p, sizeof(float2) * op->ldA, sizeof(float2) * N, N,
                            hipMemcpyDeviceToDevice, s));
  if (V)
    RF_HIP(hipMemcpy2DAsync(V, sizeof(float2) * C, op->Vb.p, sizeof(float2) * op->ldV, sizeof(float2) * C, C,
                            hipMemcpyDeviceToDevice, s));
  return RFCMP_OK;
}

void rfcmp_op_destroy(rfcmp_op op) {
  if (!op) return;
  if (op->host_scal) (void)hipHostFree(op->host_scal);
  delete op;
}

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

rfcmp_status rfcmp_precond_rhs(rfcmp_op op, const void* e, void* b, int32_t nrhs, void* stream) {
  RF_ARG(op && e && b && e != b, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return batched(nrhs, N, N, static_cast<const double2*>(e), static_cast<double2*>(b),
                 [&](const double2* x, double2* y, int nr) { return rhs_batch(op, x, y, nr, s); });
}

rfcmp_status rfcmp_apply(rfcmp_op op, const void* x, void* y, int32_t nrhs, void* stream) {
  RF_ARG(op && x && y && x != y, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return batched(nrhs, N, N, static_cast<const double2*>(x), static_cast<double2*>(y),
                 [&](const double2* a, double2* b, int nr) { return apply_batch(op, a, b, nr, s); });
}

rfcmp_status rfcmp_recover(rfcmp_op op, const void* i, void* j, int32_t nrhs, void* stream) {
  RF_ARG(op && i && j && i != j, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  const int64_t N = op->mesh->h.N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return batched(nrhs, N, N, static_cast<const double2*>(i), static_cast<double2*>(j),
                 [&](const double2* a, double2* b, int nr) { return recover_batch(op, a, b, nr, s); });
}

rfcmp_status rfcmp_project(rfcmp_op op, int32_t which, const void* xv, void* yv, int32_t nrhs, void* stream) {
  RF_ARG(op && xv && yv && xv != yv, "NULL or aliased argument");
  RF_ARG(nrhs > 0, "nrhs must be > 0");
  RF_ARG(which >= 0 && which <= 6, "unknown projector");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rfcmp_mesh m = op->mesh;
  if (which == RFCMP_PROJ_GSIGMA) RF_TRY(ensure_mesh_device(m, true, s));
  const MeshDev& d = m->d;
  const int64_t N = m->h.N, C = m->h.C, V = m->h.V;
  const int64_t nin = (which == RFCMP_PROJ_LPINV) ? C : (which == RFCMP_PROJ_GLL_INV ? V : N);
  const int64_t nout = (which <= RFCMP_PROJ_GSIGMA) ? N : (which == RFCMP_PROJ_LAMBDA_T || which == RFCMP_PROJ_GLL_INV ? V : C);
  return batched(nrhs, nin, nout, static_cast<const double2*>(xv), static_cast<double2*>(yv),
                 [&](const double2* x, double2* y, int nr) -> rfcmp_status {
                   const Work W = carve(op);
                   switch (which) {
                     case RFCMP_PROJ_SIGMA:
                     case RFCMP_PROJ_LH:
                       RF_TRY(sigma_t(d, C, N, x, W.c[0], nr, s));
                       RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[0], W.c[1], nr, s, "dmatvec_lp"));
                       return which == RFCMP_PROJ_SIGMA
                                  ? axpy_sigma(d, N, C, 0.0, false, nullptr, 1.0, W.c[1], y, nr, s)
                                  : axpy_sigma(d, N, C, 1.0, false, x, -1.0, W.c[1], y, nr, s);
                     case RFCMP_PROJ_GSIGMA:
                       RF_TRY(sigma_t(d, C, N, x, W.c[0], nr, s));
                       RF_TRY(dmatvec(d.Gtp_inv.as<double>(), C, d.ldT, W.c[0], W.c[2], nr, s, "dmatvec_gtp"));
                       RF_TRY(dmatvec(d.Lp.as<double>(), C, d.ldL, W.c[2], W.c[1], nr, s, "dmatvec_lp"));
                       return axpy_sigma(d, N, C, 0.0, false, nullptr, 1.0, W.c[1], y, nr, s);
                     case RFCMP_PROJ_LPINV:
                       return dmatvec(d.Lp.as<double>(), C, d.ldL, x, y, nr, s);
                     case RFCMP_PROJ_GLL_INV:
                       return dmatvec(d.Gll_inv.as<double>(), V, d.ldG, x, y, nr, s);
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
  RF_ARG(nrhs > 0 && (which == 0 || which == 1), "bad which/nrhs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (which == 0)
    return cmatvec(op->TA.as<float2>(), op->mesh->h.N, op->ldA, conj != 0, static_cast<const double2*>(x),
                   static_cast<double2*>(y), nrhs, s);
  return cmatvec(op->Vb.as<float2>(), op->mesh->h.C, op->ldV, conj != 0, static_cast<const double2*>(x),
                 static_cast<double2*>(y), nrhs, s);
}

rfcmp_status rfcmp_solve(rfcmp_op op, const void* e, void* j, int32_t nrhs, double tol, int32_t maxit,
                         void* stream, rfcmp_info* info) {
  RF_ARG(op && e && j && e != j, "NULL or aliased argument");
  RF_ARG(nrhs > 0 && maxit > 0 && std::isfinite(tol) && tol > 0, "bad nrhs/maxit/tol");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = op->mesh->h.N;
  const auto t0 = std::chrono::steady_clock::now();
  rfcmp_status worst = RFCMP_OK;
  for (int r = 0; r < nrhs; ++r) {
    rfcmp_info one{};
    rfcmp_status st = cg_one(op, static_cast<const double2*>(e) + r * N, static_cast<double2*>(j) + r * N, tol,
                             maxit, s, &one);
    if (st < 0) return st;
    if (st > worst) worst = st;
    if (info) info[r] = one;
  }
  RF_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info)
    for (int r = 0; r < nrhs; ++r) info[r].ms_solve = ms;
  return worst;
}

}  // extern "C"
