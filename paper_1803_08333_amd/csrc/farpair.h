// Far-pair quadrature shared by the assembly kernels (assemble.hip) and the
// compressed blocks (hmat.hip): the 7-point rule, the normalised moments of
// a far cell pair in FP32 and the block entries formed from them.
#pragma once

#include <cmath>

#include "internal.h"

namespace rfcmp {

constexpr int kQ = 7;

// Radon's 7-point degree-5 rule (Stroud T2:5-1): centroid and two orbits.
struct Rule {
  double bary[kQ][3];
  double w[kQ];
};
inline Rule make_rule() {
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
// Normalised moments of one far cell pair (c, c') (see above), scaled by
// 1/(4 pi): I_0, I_r (over c), I_r' (over c'), I_rr'.
struct Moments {
  float i0r, i0i, irr[3], iri[3], jrr[3], jri[3], kr, ki;
};

// qa: the 7 points of c minus its centroid, qb those of c'; (dx, dy, dz) =
// x_c - x_c' (formed in FP64 by the caller).
template <bool HW>
__device__ inline void far_moments(const float4* qa, const float4* qb, float dx, float dy, float dz,
                                   const RuleArgs& rule, float kk, Moments& M) {
  float bq[kQ][3], wq[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const float4 b = qb[q];
    bq[q][0] = b.x; bq[q][1] = b.y; bq[q][2] = b.z;
    wq[q] = rule.wf[q];
  }
  float i0r = 0, i0i = 0;
  float irr[3] = {0, 0, 0}, iri[3] = {0, 0, 0};
  float jrr[3] = {0, 0, 0}, jri[3] = {0, 0, 0};
  float kr = 0, ki = 0;
#pragma unroll 1
  for (int p = 0; p < kQ; ++p) {
    const float4 a = qa[p];
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
  M.i0r = i0r * inv4pi; M.i0i = i0i * inv4pi; M.kr = kr * inv4pi; M.ki = ki * inv4pi;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    M.irr[d] = irr[d] * inv4pi; M.iri[d] = iri[d] * inv4pi;
    M.jrr[d] = jrr[d] * inv4pi; M.jri[d] = jri[d] * inv4pi;
  }
}

// B[(c,i),(c',j)] = sigma_i sigma_j / 4 (I_rr' - q_i.I_r' - q'_j.(I_r - q_i I_0))
// with q_i = vertex i of c minus its centroid, q'_j the same for c'.
__device__ inline float2 b_entry(const Moments& M, float4 qi, float4 qj, float si, float sj) {
  const float tr = M.kr - (qi.x * M.jrr[0] + qi.y * M.jrr[1] + qi.z * M.jrr[2]);
  const float tim = M.ki - (qi.x * M.jri[0] + qi.y * M.jri[1] + qi.z * M.jri[2]);
  const float ur0 = M.irr[0] - qi.x * M.i0r, ur1 = M.irr[1] - qi.y * M.i0r, ur2 = M.irr[2] - qi.z * M.i0r;
  const float ui0 = M.iri[0] - qi.x * M.i0i, ui1 = M.iri[1] - qi.y * M.i0i, ui2 = M.iri[2] - qi.z * M.i0i;
  const float f = 0.25f * si * sj;
  return make_float2(f * (tr - (qj.x * ur0 + qj.y * ur1 + qj.z * ur2)),
                     f * (tim - (qj.x * ui0 + qj.y * ui1 + qj.z * ui2)));
}


// The rule as kernel arguments (weights in FP32 and FP64, points).
RuleArgs rule_args();

// V entry of a far cell pair: I_0 alone (see far_moments), scaled by 1/(4 pi).
template <bool HW>
__device__ inline float2 far_i0(const float4* qa, const float4* qb, float dx, float dy, float dz,
                                const RuleArgs& rule, float kk) {
  float i0r = 0, i0i = 0;
#pragma unroll 1
  for (int p = 0; p < kQ; ++p) {
    const float4 a = qa[p];
    const float bx = dx + a.x, by = dy + a.y, bz = dz + a.z;
    float s0r = 0, s0i = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const float4 b = qb[q];
      const float rx = bx - b.x, ry = by - b.y, rz = bz - b.z;
      const float R2 = rx * rx + ry * ry + rz * rz;
      const float rinv = __frsqrt_rn(R2);
      const float R = R2 * rinv;
      float sn, cs;
      if (HW) {
        const float rev = kk * R * 0.159154943091895336f;
        sn = __builtin_amdgcn_sinf(rev);
        cs = __builtin_amdgcn_cosf(rev);
      } else {
        sincos_moderate(kk * R, sn, cs);
      }
      const float g = rule.wf[q] * rinv;
      s0r += cs * g;
      s0i += sn * g;
    }
    i0r += rule.wf[p] * s0r;
    i0i += rule.wf[p] * s0i;
  }
  const float inv4pi = 0.0795774715459476679f;
  return make_float2(i0r * inv4pi, i0i * inv4pi);
}

}  // namespace rfcmp
