// Galerkin assembly of the EFIE blocks (Sec. 2 of the paper):
//   T_A[m,n] = int int f_m(r).f_n(r') G_k dS dS',
//   V[c,c']  = (A_c A_c')^-1 int_c int_c' G_k,     G_k = exp(ikR)/(4 pi R),
// with RWG pieces f_m|_c = sigma (r - r_m^c)/(2 A_c) (eq. RWGdef).
//
// Cell-pair formulation.  For the 3 x 3 local edges (i of c, j of c') the
// pair contributes
//   B[(c,i),(c',j)] = sigma_i sigma_j / (4 A_c A_c') int int (r - r_i).(r' - r_j) G_k,
// and T_A[m,n] sums the four B entries of the cell slots of m and n.
//
// Far pairs (FP32, 7 x 7 points): with r = x_c + rho, r' = x_c' + rho' and
// q_i = r_i - x_c (all O(h)), the block is
//   B = sigma sigma'/4 (I_rr' - q_i.I_r' - q'_j.I_r + q_i.q'_j I_0)
// over the normalised moments I_0 = sum w w' G, I_r = sum w w' rho G,
// I_r' = sum w w' rho' G, I_rr' = sum w w' rho.rho' G.  The centroid offset is
// formed in FP64 and every other length is O(h), so FP32 keeps its relative
// precision instead of losing (1/h)^2 to cancellation of O(1) coordinates.
//
// Near pairs (FP64): singular extraction G = 1/(4 pi R) + (exp(ikR) - 1)/(4 pi R);
// the 1/R part is integrated over the inner cell in closed form (Wilton et al.,
// IEEE TAP 1984; Graglia, IEEE TAP 1993), the bounded rest with 7 x 7 points,
// the outer cell is the lower-indexed one and self blocks are symmetrised.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rfcmp {

namespace {

constexpr int kQ = 7;
constexpr int kTile = 16;

// Radon's 7-point degree-5 rule (Stroud T2:5-1): centroid and two orbits.
struct Rule {
  double bary[kQ][3];
  double w[kQ];
};
Rule make_rule() {
  Rule r;
  const double s = std::sqrt(15.0);
  const double a1 = (6.0 - s) / 21.0, b1 = (9.0 + 2.0 * s) / 21.0;
  const double a2 = (6.0 + s) / 21.0, b2 = (9.0 - 2.0 * s) / 21.0;
  const double w0 = 9.0 / 40.0, w1 = (155.0 - s) / 1200.0, w2 = (155.0 + s) / 1200.0;
  const double P[kQ][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
                           {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
  const double W[kQ] = {w0, w1, w1, w1, w2, w2, w2};
  for (int q = 0; q < kQ; ++q) {
    for (int d = 0; d < 3; ++d) r.bary[q][d] = P[q][d];
    r.w[q] = W[q];
  }
  return r;
}

struct RuleArgs {
  float wf[kQ];
  double wd[kQ];
  double bary[kQ][3];
};

// ---------------------------------------------------------------- far pairs
// sin and cos of a moderate argument in FP32: Cody-Waite reduction by pi/2
// (two-term split of pi/2, one rounding per step) to |r| <= pi/4, then the
// Taylor series of sin to r^9 and of cos to r^8 (truncation below 3e-8), and
// the quadrant rotation.  Keeps full relative accuracy as x -> 0, which the
// imaginary part of G_k needs at low frequency.
constexpr float kPio2Hi = (float)1.57079632679489661923;
constexpr float kPio2Lo = (float)(1.57079632679489661923 - (double)kPio2Hi);
constexpr float k2OverPi = (float)0.63661977236758134308;

__device__ inline void sincos_moderate(float x, float& sn, float& cs) {
  const float n = rintf(x * k2OverPi);
  float r = fmaf(-n, kPio2Hi, x);
  r = fmaf(-n, kPio2Lo, r);
  const float r2 = r * r;
  float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(r2, ps, 1.0f / 120.0f);
  ps = fmaf(r2, ps, -1.0f / 6.0f);
  const float s = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, 1.0f / 40320.0f, -1.0f / 720.0f);
  pc = fmaf(r2, pc, 1.0f / 24.0f);
  pc = fmaf(r2, pc, -0.5f);
  const float c = fmaf(r2, pc, 1.0f);
  const int q = ((int)n) & 3;
  const float s1 = (q & 1) ? c : s;
  const float c1 = (q & 1) ? s : c;
  sn = (q & 2) ? -s1 : s1;
  cs = ((q + 1) & 2) ? -c1 : c1;
}

// sin and cos of kR come from the polynomial above, or, when kR <= 2 over the
// whole mesh (HW), from the transcendental unit (v_sin_f32 / v_cos_f32 take
// the argument in revolutions).  Measured on the device against double
// precision for |x| < 2: sin within 1e-6 relative (also as x -> 0), cos
// within 2.1e-7 absolute; beyond 2 the revolution product loses absolute
// accuracy (7e-7 up to 10), so larger kR keeps the reduced polynomial.
// Upper-triangular tile (I <= J) of kTile x kTile cell pairs per block, one
// pair per thread.  Pairs c >= c' of diagonal tiles are left to their mirror
// (c == c' to the near kernel).  Every pair writes B(c,c') and B(c',c) =
// B(c,c')^T from the same registers, so B is exactly symmetric.
template <bool HW>
__global__ __launch_bounds__(256) void k_far_pairs(int C, long ntiles, const double* __restrict__ cen,
                                                   const float4* __restrict__ qoff,
                                                   const float4* __restrict__ fvoff,
                                                   const float* __restrict__ sgn, float kk,
                                                   RuleArgs rule, float2* __restrict__ B, long ldB,
                                                   float2* __restrict__ Vm, long ldV) {
  const long t = blockIdx.x;
  if (t >= ntiles) return;
  // t -> (I, J) with I <= J, t = J(J+1)/2 + I
  long J = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (J * (J + 1) / 2 > t) --J;
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  const long I = t - J * (J + 1) / 2;

  __shared__ float4 sq_t[kTile][kQ], sq_s[kTile][kQ];
  __shared__ double sc_t[kTile][3], sc_s[kTile][3];
  for (int e = threadIdx.x; e < kTile * kQ; e += 256) {
    const int cc = e / kQ, q = e % kQ;
    const long ct = I * kTile + cc, cs = J * kTile + cc;
    sq_t[cc][q] = ct < C ? qoff[ct * kQ + q] : make_float4(0, 0, 0, 0);
    sq_s[cc][q] = cs < C ? qoff[cs * kQ + q] : make_float4(0, 0, 0, 0);
  }
  for (int e = threadIdx.x; e < kTile * 3; e += 256) {
    const int cc = e / 3, d = e % 3;
    const long ct = I * kTile + cc, cs = J * kTile + cc;
    sc_t[cc][d] = ct < C ? cen[ct * 3 + d] : 0.0;
    sc_s[cc][d] = cs < C ? cen[cs * 3 + d] : 0.0;
  }
  __syncthreads();

  const int ti = threadIdx.x / kTile, tj = threadIdx.x % kTile;
  const long c = I * kTile + ti, cp = J * kTile + tj;
  if (c >= C || cp >= C) return;
  if (I == J && ti >= tj) return;

  const float dx = (float)(sc_t[ti][0] - sc_s[tj][0]);
  const float dy = (float)(sc_t[ti][1] - sc_s[tj][1]);
  const float dz = (float)(sc_t[ti][2] - sc_s[tj][2]);
  float bq[kQ][3], wq[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const float4 b = sq_s[tj][q];
    bq[q][0] = b.x; bq[q][1] = b.y; bq[q][2] = b.z;
    wq[q] = rule.wf[q];
  }

  float i0r = 0, i0i = 0;                       // I_0
  float irr[3] = {0, 0, 0}, iri[3] = {0, 0, 0};   // I_r
  float jrr[3] = {0, 0, 0}, jri[3] = {0, 0, 0};   // I_r'
  float kr = 0, ki = 0;                         // I_rr'
#pragma unroll 1
  for (int p = 0; p < kQ; ++p) {
    const float4 a = sq_t[ti][p];
    const float bx = dx + a.x, by = dy + a.y, bz = dz + a.z;
    float s0r = 0, s0i = 0, s1r[3] = {0, 0, 0}, s1i[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const float rx = bx - bq[q][0], ry = by - bq[q][1], rz = bz - bq[q][2];
      const float R2 = rx * rx + ry * ry + rz * rz;
      const float rinv = __frsqrt_rn(R2);
      const float R = R2 * rinv;
      float sn, cs;
      if (HW) {  // the transcendental unit, argument in revolutions (kR <= 2 here)
        const float rev = kk * R * 0.159154943091895336f;
        sn = __builtin_amdgcn_sinf(rev);
        cs = __builtin_amdgcn_cosf(rev);
      } else {
        sincos_moderate(kk * R, sn, cs);
      }
      const float g = wq[q] * rinv;
      const float gr = cs * g, gi = sn * g;
      s0r += gr;
      s0i += gi;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s1r[d] += bq[q][d] * gr;
        s1i[d] += bq[q][d] * gi;
      }
    }
    const float wp = rule.wf[p];
    i0r += wp * s0r;
    i0i += wp * s0i;
    irr[0] += wp * a.x * s0r; iri[0] += wp * a.x * s0i;
    irr[1] += wp * a.y * s0r; iri[1] += wp * a.y * s0i;
    irr[2] += wp * a.z * s0r; iri[2] += wp * a.z * s0i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      jrr[d] += wp * s1r[d];
      jri[d] += wp * s1i[d];
    }
    kr += wp * (a.x * s1r[0] + a.y * s1r[1] + a.z * s1r[2]);
    ki += wp * (a.x * s1i[0] + a.y * s1i[1] + a.z * s1i[2]);
  }
  const float inv4pi = 0.0795774715459476679f;  // 1/(4 pi)
  i0r *= inv4pi; i0i *= inv4pi; kr *= inv4pi; ki *= inv4pi;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    irr[d] *= inv4pi; iri[d] *= inv4pi; jrr[d] *= inv4pi; jri[d] *= inv4pi;
  }
  Vm[c * ldV + cp] = make_float2(i0r, i0i);
  Vm[cp * ldV + c] = make_float2(i0r, i0i);

  float4 qt[3], qs[3];
  float st[3], ss[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    qt[i] = fvoff[c * 3 + i];
    qs[i] = fvoff[cp * 3 + i];
    st[i] = sgn[c * 3 + i];
    ss[i] = sgn[cp * 3 + i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // t_i = I_rr' - q_i.I_r',  u_i = I_r - q_i I_0
    const float tr = kr - (qt[i].x * jrr[0] + qt[i].y * jrr[1] + qt[i].z * jrr[2]);
    const float tim = ki - (qt[i].x * jri[0] + qt[i].y * jri[1] + qt[i].z * jri[2]);
    const float ur[3] = {irr[0] - qt[i].x * i0r, irr[1] - qt[i].y * i0r, irr[2] - qt[i].z * i0r};
    const float ui[3] = {iri[0] - qt[i].x * i0i, iri[1] - qt[i].y * i0i, iri[2] - qt[i].z * i0i};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float f = 0.25f * st[i] * ss[j];
      const float br = f * (tr - (qs[j].x * ur[0] + qs[j].y * ur[1] + qs[j].z * ur[2]));
      const float bi = f * (tim - (qs[j].x * ui[0] + qs[j].y * ui[1] + qs[j].z * ui[2]));
      B[(3 * c + i) * ldB + 3 * cp + j] = make_float2(br, bi);
      B[(3 * cp + j) * ldB + 3 * c + i] = make_float2(br, bi);
    }
  }
}

// ---------------------------------------------------------------- near pairs
struct Pot {
  double S;       // int 1/R
  double W[3];    // int (r' - r)/R
};

// Closed-form potentials of the flat triangle P (CCW about its normal) at r.
__device__ Pot tri_potentials(const double P[3][3], const double r[3]) {
  double u0[3], v0[3], nr[3];
  for (int d = 0; d < 3; ++d) {
    u0[d] = P[1][d] - P[0][d];
    v0[d] = P[2][d] - P[0][d];
  }
  nr[0] = u0[1] * v0[2] - u0[2] * v0[1];
  nr[1] = u0[2] * v0[0] - u0[0] * v0[2];
  nr[2] = u0[0] * v0[1] - u0[1] * v0[0];
  const double nl = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
  for (int d = 0; d < 3; ++d) nr[d] /= nl;
  const double h = (r[0] - P[0][0]) * nr[0] + (r[1] - P[0][1]) * nr[1] + (r[2] - P[0][2]) * nr[2];
  const double ah = fabs(h);
  double rho[3];
  for (int d = 0; d < 3; ++d) rho[d] = r[d] - h * nr[d];
  Pot out{0.0, {0.0, 0.0, 0.0}};
  for (int e = 0; e < 3; ++e) {
    const double* a = P[e];
    const double* b = P[(e + 1) % 3];
    double lv[3];
    for (int d = 0; d < 3; ++d) lv[d] = b[d] - a[d];
    const double L = sqrt(lv[0] * lv[0] + lv[1] * lv[1] + lv[2] * lv[2]);
    for (int d = 0; d < 3; ++d) lv[d] /= L;
    // outward in-plane edge normal u = l x n
    const double uu[3] = {lv[1] * nr[2] - lv[2] * nr[1], lv[2] * nr[0] - lv[0] * nr[2],
                          lv[0] * nr[1] - lv[1] * nr[0]};
    double ta = 0, lm = 0, lp = 0, Rm2 = 0, Rp2 = 0;
    for (int d = 0; d < 3; ++d) {
      ta += (a[d] - rho[d]) * uu[d];
      lm += (a[d] - rho[d]) * lv[d];
      lp += (b[d] - rho[d]) * lv[d];
      Rm2 += (r[d] - a[d]) * (r[d] - a[d]);
      Rp2 += (r[d] - b[d]) * (r[d] - b[d]);
    }
    const double Rm = sqrt(Rm2), Rp = sqrt(Rp2);
    const double R02 = ta * ta + h * h;
    double f = 0.0;
    if (R02 > 1e-30 * L * L) {
      // ln((R+ + l+)/(R- + l-)) = ln((R- - l-)/(R+ - l+)); pick the form without cancellation
      f = (lp + lm >= 0.0) ? log((Rp + lp) / (Rm + lm)) : log((Rm - lm) / (Rp - lp));
    }
    double at = 0.0;
    if (ah > 0.0) at = atan(ta * lp / (R02 + ah * Rp)) - atan(ta * lm / (R02 + ah * Rm));
    out.S += ta * f - ah * at;
    const double wcoef = 0.5 * (R02 * f + lp * Rp - lm * Rm);
    for (int d = 0; d < 3; ++d) out.W[d] += wcoef * uu[d];
  }
  for (int d = 0; d < 3; ++d) out.W[d] -= h * out.S * nr[d];
  return out;
}

// One thread per near pair (c <= c'): outer cell c, inner cell c'.
__global__ __launch_bounds__(128) void k_near_pairs(long npairs, const int* __restrict__ pairs,
                                                    const double* __restrict__ vtx,
                                                    const double* __restrict__ area,
                                                    const float* __restrict__ sgn, double kk,
                                                    RuleArgs rule, float2* __restrict__ B, long ldB,
                                                    float2* __restrict__ Vm, long ldV) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npairs) return;
  const int c = pairs[2 * t], cp = pairs[2 * t + 1];
  double Po[3][3], Pi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) {
      Po[i][d] = vtx[(long)c * 9 + 3 * i + d];
      Pi[i][d] = vtx[(long)cp * 9 + 3 * i + d];
    }
  const double Ain = area[cp];
  double xo[kQ][3], xi[kQ][3];
  for (int q = 0; q < kQ; ++q)
    for (int d = 0; d < 3; ++d) {
      xo[q][d] = rule.bary[q][0] * Po[0][d] + rule.bary[q][1] * Po[1][d] + rule.bary[q][2] * Po[2][d];
      xi[q][d] = rule.bary[q][0] * Pi[0][d] + rule.bary[q][1] * Pi[1][d] + rule.bary[q][2] * Pi[2][d];
    }
  double vr = 0.0, vi = 0.0;
  double br[3][3] = {}, bi[3][3] = {};
  for (int p = 0; p < kQ; ++p) {
    const Pot pot = tri_potentials(Pi, xo[p]);
    const double wp = rule.wd[p];
    // singular part: int_c' (r' - r_j)/R = W + (x_p - r_j) S
    vr += wp * pot.S / Ain;
    double arm[3][3];  // x_p - r_i (outer)
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) arm[i][d] = xo[p][d] - Po[i][d];
    for (int j = 0; j < 3; ++j) {
      double inner[3];
      for (int d = 0; d < 3; ++d) inner[d] = pot.W[d] + (xo[p][d] - Pi[j][d]) * pot.S;
      for (int i = 0; i < 3; ++i)
        br[i][j] += wp * (arm[i][0] * inner[0] + arm[i][1] * inner[1] + arm[i][2] * inner[2]) / Ain;
    }
    // bounded part: (exp(ikR) - 1)/R = (-2 sin^2(kR/2) + i sin(kR))/R, ik at R = 0
    for (int q = 0; q < kQ; ++q) {
      double rr[3];
      for (int d = 0; d < 3; ++d) rr[d] = xo[p][d] - xi[q][d];
      const double R = sqrt(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
      double gr, gi;
      if (R > 0.0) {
        const double sh = sin(0.5 * kk * R);
        gr = -2.0 * sh * sh / R;
        gi = sin(kk * R) / R;
      } else {
        gr = 0.0;
        gi = kk;
      }
      const double ww = wp * rule.wd[q];
      vr += ww * gr;
      vi += ww * gi;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double dot = 0.0;
          for (int d = 0; d < 3; ++d) dot += (xo[p][d] - Po[i][d]) * (xi[q][d] - Pi[j][d]);
          br[i][j] += ww * dot * gr;
          bi[i][j] += ww * dot * gi;
        }
    }
  }
  const double inv4pi = 0.25 / M_PI;
  vr *= inv4pi;
  vi *= inv4pi;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double f = 0.25 * sgn[c * 3 + i] * sgn[cp * 3 + j] * inv4pi;
      br[i][j] *= f;
      bi[i][j] *= f;
    }
  if (c == cp) {
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) {
        const double mr = 0.5 * (br[i][j] + br[j][i]), mi = 0.5 * (bi[i][j] + bi[j][i]);
        br[i][j] = br[j][i] = mr;
        bi[i][j] = bi[j][i] = mi;
      }
  }
  const float2 v = make_float2((float)vr, (float)vi);
  Vm[(long)c * ldV + cp] = v;
  Vm[(long)cp * ldV + c] = v;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const float2 b = make_float2((float)br[i][j], (float)bi[i][j]);
      B[(long)(3 * c + i) * ldB + 3 * cp + j] = b;
      B[(long)(3 * cp + j) * ldB + 3 * c + i] = b;
    }
}

// ---------------------------------------------------------------- gather
// T_A[m,n] = (B[m+,n+] + B[m-,n-]) + (B[m+,n-] + B[m-,n+]) over the cell slots
// of the two edges; the fixed pairing keeps T_A exactly symmetric.  Only
// the entries with n >= kTriBlock floor(m / kTriBlock) are formed (the upper
// triangle of kTriBlock-wide blocks, all that the symmetric products read);
// the others are the transposed entries, bit for bit.
__global__ __launch_bounds__(256) void k_gather_ta(int N, const int* __restrict__ slot,
                                                   const float2* __restrict__ B, long ldB,
                                                   float2* __restrict__ TA, long ldA) {
  const int m = blockIdx.x;
  const int sp = slot[2 * m], sm = slot[2 * m + 1];
  const float2* bp = B + (long)sp * ldB;
  const float2* bm = B + (long)sm * ldB;
  for (int n = (m / kTriBlock) * kTriBlock + threadIdx.x; n < N; n += blockDim.x) {
    const int np = slot[2 * n], nm = slot[2 * n + 1];
    const float2 pp = bp[np], mm = bm[nm], pm = bp[nm], mp = bm[np];
    const float2 s1 = make_float2(pp.x + mm.x, pp.y + mm.y);
    const float2 s2 = make_float2(pm.x + mp.x, pm.y + mp.y);
    TA[(long)m * ldA + n] = make_float2(s1.x + s2.x, s1.y + s2.y);
  }
}

// ---------------------------------------------------------------- excitation
// e[r][m] = sum over the two cells of m: sigma/2 sum_q w_q (x_q - r_m).pol exp(ik khat.x_q).
// split = 1: e1 = e - Sigma s, the plane wave less its static part pol
// (whose excitation Sigma s, s_c = -pol . x_c, lies in the range of Sigma):
// exp(i t) - 1 = -2 sin^2(t/2) + i sin t keeps e1's O(k) loop part at any k.
__global__ void k_rhs(int N, int nrhs, const int* __restrict__ edge_cell, const int* __restrict__ edge_slot,
                      const double* __restrict__ vtx, double kk, const double* __restrict__ khat,
                      const double* __restrict__ pol, RuleArgs rule, double2* __restrict__ e, int split = 0) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)N * nrhs) return;
  const int r = int(t / N), m = int(t % N);
  const double kh[3] = {khat[3 * r], khat[3 * r + 1], khat[3 * r + 2]};
  const double po[3] = {pol[3 * r], pol[3 * r + 1], pol[3 * r + 2]};
  double sr = 0.0, si = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int c = edge_cell[2 * m + side], l = edge_slot[2 * m + side] - 3 * c;
    const double sg = side == 0 ? 0.5 : -0.5;
    const double* P = vtx + (long)c * 9;
    double accr = 0.0, acci = 0.0;
    for (int q = 0; q < kQ; ++q) {
      double x[3];
      for (int d = 0; d < 3; ++d)
        x[d] = rule.bary[q][0] * P[d] + rule.bary[q][1] * P[3 + d] + rule.bary[q][2] * P[6 + d];
      const double proj = (x[0] - P[3 * l]) * po[0] + (x[1] - P[3 * l + 1]) * po[1] + (x[2] - P[3 * l + 2]) * po[2];
      double sn, cs;
      const double ph = kk * (kh[0] * x[0] + kh[1] * x[1] + kh[2] * x[2]);
      sincos(ph, &sn, &cs);
      if (split) {
        const double h = sin(0.5 * ph);
        cs = -2.0 * h * h;
      }
      accr += rule.wd[q] * proj * cs;
      acci += rule.wd[q] * proj * sn;
    }
    sr += sg * accr;
    si += sg * acci;
  }
  e[t] = make_double2(sr, si);
}

// s[r][c] = -pol_r . x_c (x_c the centroid): the static part Sigma s of the
// plane-wave excitation (int f_m . pol = -int div(f_m) pol . r).
__global__ void k_rhs_static(int C, int nrhs, const double* __restrict__ cen, const double* __restrict__ pol,
                             double2* __restrict__ sv) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)C * nrhs) return;
  const int r = int(t / C), c = int(t % C);
  const double v = pol[3 * r] * cen[3 * c] + pol[3 * r + 1] * cen[3 * c + 1] + pol[3 * r + 2] * cen[3 * c + 2];
  sv[t] = make_double2(-v, 0.0);
}

// ---------------------------------------------------------------- far field
// F_r(d) = int j_r exp(-i k dhat_d . x) dS: on cell c the RWG current is
// sum_i j_m sigma_i (x - v_i)/(2 A_c) (v_i opposite local edge i) and the
// rule's weights sum to one, so F = sum_c sum_q w_q/2 sum_i sigma_i j_m
// (x_q - v_i) exp(-i k dhat . x_q).  sigma_r(d) = k^2/(4 pi) |F - dhat (dhat .
// F)|^2 (unit incident amplitude).  One workgroup per (direction, right-hand
// side): cells strided over the threads, then a fixed-order block sum (xor
// butterflies in each wave, the four wave sums in order).
// With js != nullptr, j is the loop (divergence-free) part of the current
// and js its star part: a loop current carries no net current, so its phase
// factor is taken as exp(-i t) - 1 = -2 sin^2(t/2) - i sin t, without
// cancellation at any k; js takes the plain phase.
__global__ __launch_bounds__(256) void k_farfield(int C, int N, int ndir, const int* __restrict__ cell_edge,
                                                  const float* __restrict__ sgn, const double* __restrict__ vtx,
                                                  double kk, const double* __restrict__ dirs, RuleArgs rule,
                                                  const double2* __restrict__ j, const double2* __restrict__ js,
                                                  double2* __restrict__ F, double* __restrict__ rcs) {
  __shared__ double red[4][6];
  const int d = blockIdx.x, r = blockIdx.y;
  const double dh[3] = {dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2]};
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // (re, im) of x, y, z
  for (int c = threadIdx.x; c < C; c += 256) {
    const double* P = vtx + (long)c * 9;
    double2 jc[3], jsc[3];
    double sg[3];
    for (int i = 0; i < 3; ++i) {
      jc[i] = j[(long)r * N + cell_edge[3 * c + i]];
      jsc[i] = js ? js[(long)r * N + cell_edge[3 * c + i]] : make_double2(0.0, 0.0);
      sg[i] = 0.5 * (double)sgn[3 * c + i];
    }
    for (int q = 0; q < kQ; ++q) {
      double x[3];
      for (int k = 0; k < 3; ++k)
        x[k] = rule.bary[q][0] * P[k] + rule.bary[q][1] * P[3 + k] + rule.bary[q][2] * P[6 + k];
      double sn, cs;
      const double ph = kk * (dh[0] * x[0] + dh[1] * x[1] + dh[2] * x[2]);
      sincos(ph, &sn, &cs);
      const double wr = rule.wd[q] * cs, wi = -rule.wd[q] * sn;  // w_q exp(-i k dhat . x_q)
      double lr = wr;                                            // the loop part's phase factor
      if (js) {
        const double h = sin(0.5 * ph);
        lr = -2.0 * rule.wd[q] * h * h;
      }
      for (int k = 0; k < 3; ++k) {
        double cr = 0.0, ci = 0.0;  // sum_i sigma_i / 2 j_m (x_q - v_i)_k
        double dr = 0.0, di = 0.0;  // the same for the star part
        for (int i = 0; i < 3; ++i) {
          const double arm = sg[i] * (x[k] - P[3 * i + k]);
          cr += arm * jc[i].x;
          ci += arm * jc[i].y;
          dr += arm * jsc[i].x;
          di += arm * jsc[i].y;
        }
        acc[2 * k] += (cr * lr - ci * wi) + (dr * wr - di * wi);
        acc[2 * k + 1] += (cr * wi + ci * lr) + (dr * wi + di * wr);
      }
    }
  }
  for (int q = 0; q < 6; ++q)
    for (int m = 32; m > 0; m >>= 1) acc[q] += __shfl_xor(acc[q], m);
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 6; ++q) red[threadIdx.x >> 6][q] = acc[q];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double f[6];
  for (int q = 0; q < 6; ++q) f[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
  double2* Fo = F + ((long)r * ndir + d) * 3;
  for (int k = 0; k < 3; ++k) Fo[k] = make_double2(f[2 * k], f[2 * k + 1]);
  if (rcs) {
    const double pr = dh[0] * f[0] + dh[1] * f[2] + dh[2] * f[4];  // dhat . F
    const double pi = dh[0] * f[1] + dh[1] * f[3] + dh[2] * f[5];
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double tr = f[2 * k] - dh[k] * pr, ti = f[2 * k + 1] - dh[k] * pi;
      s += tr * tr + ti * ti;
    }
    rcs[(long)r * ndir + d] = kk * kk / (4.0 * M_PI) * s;
  }
}

RuleArgs rule_args() {
  static const Rule r = make_rule();
  RuleArgs a;
  for (int q = 0; q < kQ; ++q) {
    a.wf[q] = (float)r.w[q];
    a.wd[q] = r.w[q];
    for (int d = 0; d < 3; ++d) a.bary[q][d] = r.bary[q][d];
  }
  return a;
}

}  // namespace

rfcmp_status mesh_upload(rfcmp_mesh m, hipStream_t s) {
  const MeshHost& h = m->h;
  MeshDev& d = m->d;
  const int64_t C = h.C, N = h.N, V = h.V;
  const Rule rule = make_rule();
  std::vector<double> vtx(9 * C);
  std::vector<float> qoff(4 * kQ * C), fvoff(12 * C), sg(3 * C);
  std::vector<int> slot(2 * N);
  for (int64_t c = 0; c < C; ++c) {
    const double* x = &h.centroid[3 * c];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) vtx[9 * c + 3 * i + k] = h.xyz[3 * h.tri[3 * c + i] + k];
    for (int q = 0; q < kQ; ++q)
      for (int k = 0; k < 3; ++k) {
        double p = 0.0;
        for (int i = 0; i < 3; ++i) p += rule.bary[q][i] * vtx[9 * c + 3 * i + k];
        qoff[4 * (kQ * c + q) + k] = (float)(p - x[k]);
      }
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) fvoff[12 * c + 4 * i + k] = (float)(vtx[9 * c + 3 * i + k] - x[k]);
      sg[3 * c + i] = (float)h.cell_sign[3 * c + i];
    }
  }
  for (int64_t n = 0; n < N; ++n) {
    slot[2 * n] = 3 * h.edge_cell[2 * n] + h.edge_local[2 * n];
    slot[2 * n + 1] = 3 * h.edge_cell[2 * n + 1] + h.edge_local[2 * n + 1];
  }
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> rfcmp_status {
    RF_TRY(b.alloc(bytes));
    RF_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return RFCMP_OK;
  };
  RF_TRY(up(d.cen, h.centroid.data(), sizeof(double) * 3 * C));
  RF_TRY(up(d.vtx, vtx.data(), sizeof(double) * 9 * C));
  RF_TRY(up(d.area, h.area.data(), sizeof(double) * C));
  RF_TRY(up(d.qoff, qoff.data(), sizeof(float) * qoff.size()));
  RF_TRY(up(d.fvoff, fvoff.data(), sizeof(float) * fvoff.size()));
  RF_TRY(up(d.sgn, sg.data(), sizeof(float) * sg.size()));
  RF_TRY(up(d.cell_edge, h.cell_edge.data(), sizeof(int) * 3 * C));
  RF_TRY(up(d.edge_cell, h.edge_cell.data(), sizeof(int) * 2 * N));
  RF_TRY(up(d.edge_slot, slot.data(), sizeof(int) * 2 * N));
  RF_TRY(up(d.edge_vtx, h.edge_vtx.data(), sizeof(int) * 2 * N));
  RF_TRY(up(d.ve_ptr, h.vtx_edge_ptr.data(), sizeof(int) * (V + 1)));
  RF_TRY(up(d.ve_idx, h.vtx_edge_idx.data(), sizeof(int) * 2 * N));
  std::vector<float> vs(h.vtx_edge_sgn.begin(), h.vtx_edge_sgn.end());
  RF_TRY(up(d.ve_sgn, vs.data(), sizeof(float) * 2 * N));
  RF_HIP(hipStreamSynchronize(s));  // host staging vectors die here
  return RFCMP_OK;
}

rfcmp_status assemble_blocks(rfcmp_op op, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  const MeshHost& h = m->h;
  MeshDev& d = m->d;
  const int64_t C = h.C, N = h.N;
  const RuleArgs ra = rule_args();

  const int64_t ldB = (int64_t)round_up(3 * C, 64);
  // scratch and near-pair list live with the mesh: reused by every wavenumber
  if (!d.pairB.p) RF_TRY(d.pairB.alloc(sizeof(float2) * ldB * 3 * C));
  DevBuf& B = d.pairB;
  RF_HIP(hipMemsetAsync(op->Vb.p, 0, op->Vb.bytes, s));

  // far pairs first: they do not need the near-pair list, which a new mesh
  // may still be computing on host threads
  const long nt = (long)((C + kTile - 1) / kTile);
  const long ntiles = nt * (nt + 1) / 2;
  {
  ProfScope prof("far_pairs", s);
  // largest kR between quadrature points: at most k times twice the largest
  // vertex distance from the bounding-box centre (the diameter of a sphere)
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  const size_t nv = h.xyz.size() / 3;
  for (size_t v = 0; v < nv; ++v)
    for (int q = 0; q < 3; ++q) {
      lo[q] = std::min(lo[q], h.xyz[3 * v + q]);
      hi[q] = std::max(hi[q], h.xyz[3 * v + q]);
    }
  double rad2 = 0.0;
  for (size_t v = 0; v < nv; ++v) {
    double r2 = 0.0;
    for (int q = 0; q < 3; ++q) {
      const double dq = h.xyz[3 * v + q] - 0.5 * (lo[q] + hi[q]);
      r2 += dq * dq;
    }
    rad2 = std::max(rad2, r2);
  }
  const double diag = 2.0 * std::sqrt(rad2);
  const bool hw = op->k * diag <= 2.0;
  hipLaunchKernelGGL(hw ? k_far_pairs<true> : k_far_pairs<false>, dim3((unsigned)ntiles), dim3(256), 0, s, (int)C, ntiles, d.cen.as<double>(),
                     d.qoff.as<float4>(), d.fvoff.as<float4>(), d.sgn.as<float>(), (float)op->k, ra,
                     B.as<float2>(), (long)ldB, op->Vb.as<float2>(), (long)op->ldV);
  }
  RF_HIP(hipGetLastError());
  if (d.near_factor != op->opt.near_factor) {
    std::vector<int32_t> pairs;
    if (m->near_async.valid() && m->near_async_factor == op->opt.near_factor)
      pairs = m->near_async.get();  // started at mesh creation
    else
      near_pairs(h, op->opt.near_factor, pairs);
    RF_TRY(d.near.alloc(sizeof(int) * std::max<size_t>(pairs.size(), 2)));
    d.near_host = std::move(pairs);  // the source stays alive with the mesh
    RF_HIP(hipMemcpyAsync(d.near.p, d.near_host.data(), sizeof(int) * d.near_host.size(), hipMemcpyHostToDevice,
                          s));
    d.npairs = (int64_t)d.near_host.size() / 2;
    d.near_factor = op->opt.near_factor;
  }
  const long npairs = (long)d.npairs;
  DevBuf& dp = d.near;
  if (npairs > 0) {
    ProfScope prof("near_pairs", s);
    hipLaunchKernelGGL(k_near_pairs, dim3((unsigned)((npairs + 127) / 128)), dim3(128), 0, s, npairs,
                       dp.as<int>(), d.vtx.as<double>(), d.area.as<double>(), d.sgn.as<float>(), op->k, ra,
                       B.as<float2>(), (long)ldB, op->Vb.as<float2>(), (long)op->ldV);
    RF_HIP(hipGetLastError());
  }
  {
  ProfScope prof("gather_ta", s);
  hipLaunchKernelGGL(k_gather_ta, dim3((unsigned)N), dim3(256), 0, s, (int)N, d.edge_slot.as<int>(),
                     B.as<float2>(), (long)ldB, op->TA.as<float2>(), (long)op->ldA);
  }
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

namespace {
// Voltage-gap excitation: element t = r N + m of e takes the summed gap
// voltage of flat index t from the sorted, duplicate-free list idx/val, found
// by binary search, else 0.
__global__ void k_rhs_gap(long total, const long* __restrict__ idx, const double2* __restrict__ val, int P,
                          double2* __restrict__ e) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = P;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (idx[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  e[t] = (lo < P && idx[lo] == t) ? val[lo] : make_double2(0.0, 0.0);
}
}  // namespace

rfcmp_status far_field(rfcmp_op op, const double2* j, const double2* js, int nrhs, const double* dirs, int ndir,
                       double2* F, double* rcs, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  DevBuf dd;
  RF_TRY(dd.alloc(sizeof(double) * 3 * ndir));
  RF_HIP(hipMemcpyAsync(dd.p, dirs, sizeof(double) * 3 * ndir, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_farfield, dim3((unsigned)ndir, (unsigned)nrhs), dim3(256), 0, s, (int)m->h.C, (int)m->h.N,
                     ndir, m->d.cell_edge.as<int>(), m->d.sgn.as<float>(), m->d.vtx.as<double>(), op->k,
                     dd.as<double>(), rule_args(), j, js, F, rcs);
  RF_HIP(hipGetLastError());
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

rfcmp_status rhs_planewave(rfcmp_op op, const double* khat, const double* pol, int nrhs, double2* e,
                           hipStream_t s, double2* sv) {
  rfcmp_mesh m = op->mesh;
  const int64_t N = m->h.N, C = m->h.C;
  DevBuf dk;
  RF_TRY(dk.alloc(sizeof(double) * 6 * nrhs));
  RF_HIP(hipMemcpyAsync(dk.p, khat, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, s));
  RF_HIP(hipMemcpyAsync(dk.as<double>() + 3 * nrhs, pol, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, s));
  const long total = (long)N * nrhs;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (int)N, nrhs,
                     m->d.edge_cell.as<int>(), m->d.edge_slot.as<int>(), m->d.vtx.as<double>(), op->k, dk.as<double>(),
                     dk.as<double>() + 3 * nrhs, rule_args(), e, sv ? 1 : 0);
  RF_HIP(hipGetLastError());
  if (sv) {
    const long tc = (long)C * nrhs;
    hipLaunchKernelGGL(k_rhs_static, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0, s, (int)C, nrhs,
                       m->d.cen.as<double>(), dk.as<double>() + 3 * nrhs, sv);
    RF_HIP(hipGetLastError());
  }
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

// Staging of rfcmp_rhs_planewave_noalloc: the directions and polarisations of
// at most RFCMP_RHS_NOALLOC_MAX plane waves (khat [nrhs][3], then pol
// [nrhs][3]), in a fixed array of each device instead of a buffer allocated
// per call.  Host code never uses the array's name as an address: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double rhs_stage[6 * RFCMP_RHS_NOALLOC_MAX];

namespace {
constexpr int kMaxDevices = 64;

rfcmp_status rhs_stage_address(double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  RF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the staging array is set up for", dev, kMaxDevices);
    return RFCMP_E_STATE;
  }
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    RF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(rhs_stage)));
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return RFCMP_OK;
}
}  // namespace

rfcmp_status rhs_planewave_noalloc(rfcmp_op op, const double* khat, const double* pol, int nrhs, double2* e,
                                   hipStream_t s) {
  if (nrhs > RFCMP_RHS_NOALLOC_MAX) {
    set_error("rfcmp_rhs_planewave_noalloc: %d plane waves, at most %d", nrhs, RFCMP_RHS_NOALLOC_MAX);
    return RFCMP_E_ARG;
  }
  rfcmp_mesh m = op->mesh;
  const int64_t N = m->h.N;
  double* stage = nullptr;
  RF_TRY(rhs_stage_address(&stage));
  RF_HIP(hipMemcpyAsync(stage, khat, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, s));
  RF_HIP(hipMemcpyAsync(stage + 3 * nrhs, pol, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, s));
  const long total = (long)N * nrhs;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (int)N, nrhs,
                     m->d.edge_cell.as<int>(), m->d.edge_slot.as<int>(), m->d.vtx.as<double>(), op->k, stage,
                     stage + 3 * nrhs, rule_args(), e);
  RF_HIP(hipGetLastError());
  // the next call on this device overwrites the stage
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

rfcmp_status rhs_gap(rfcmp_mesh m, const int32_t* edges, const double2* volts, int ngap, int nrhs, double2* e,
                     hipStream_t s) {
  const int64_t N = m->h.N;
  // Flat indices r N + m in order, gaps on one edge summed in the order given.
  std::vector<std::pair<long, double2>> g;
  g.reserve((size_t)ngap * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int q = 0; q < ngap; ++q) g.push_back({(long)r * N + edges[(long)r * ngap + q], volts[(long)r * ngap + q]});
  std::stable_sort(g.begin(), g.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  std::vector<long> idx;
  std::vector<double2> val;
  for (const auto& x : g) {
    if (!idx.empty() && idx.back() == x.first) {
      val.back().x += x.second.x;
      val.back().y += x.second.y;
    } else {
      idx.push_back(x.first);
      val.push_back(x.second);
    }
  }
  const int P = (int)idx.size();
  DevBuf di, dv;
  if (P) {
    RF_TRY(di.alloc(sizeof(long) * P));
    RF_TRY(dv.alloc(sizeof(double2) * P));
    RF_HIP(hipMemcpyAsync(di.p, idx.data(), sizeof(long) * P, hipMemcpyHostToDevice, s));
    RF_HIP(hipMemcpyAsync(dv.p, val.data(), sizeof(double2) * P, hipMemcpyHostToDevice, s));
  }
  const long total = (long)N * nrhs;
  hipLaunchKernelGGL(k_rhs_gap, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total,
                     P ? di.as<long>() : nullptr, P ? dv.as<double2>() : nullptr, P, e);
  RF_HIP(hipGetLastError());
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

}  // namespace rfcmp
