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
// sin and cos of x = kR on the transcendental unit (v_sin_f32, v_cos_f32 take
// the argument in revolutions).  The revolutions t = x / (2 pi) are formed as
// an unevaluated sum: the FP32 product by the FP32 value of 1/(2 pi), its
// rounding error by an FMA, and the product by the rest of 1/(2 pi); the
// integer part of the product is taken off exactly, so the unit sees an
// argument in [-1/2, 1/2] revolutions that is as accurate as x itself, for
// any x.  sin keeps full relative accuracy as x -> 0 (the reduction is the
// identity there), which the imaginary part of G_k needs at low frequency.
constexpr float kInv2PiHi = (float)0.15915494309189533577;
constexpr float kInv2PiLo = (float)(0.15915494309189533577 - (double)kInv2PiHi);

__device__ inline void sincos_kr(float x, float& sn, float& cs) {
  const float t = x * kInv2PiHi;
  const float te = fmaf(x, kInv2PiHi, -t) + x * kInv2PiLo;
  const float r = (t - rintf(t)) + te;
  sn = __builtin_amdgcn_sinf(r);
  cs = __builtin_amdgcn_cosf(r);
}

// Normalised moments of one far cell pair (c, c') (see above), scaled by
// 1/(4 pi): I_0, I_r (over c), I_r' (over c'), I_rr'.
struct Moments {
  float i0r, i0i, irr[3], iri[3], jrr[3], jri[3], kr, ki;
};

// qa: the 7 points of c minus its centroid, qb those of c'; (dx, dy, dz) =
// x_c - x_c' (formed in FP64 by the caller).
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
      sincos_kr(kk * R, sn, cs);
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
      sincos_kr(kk * R, sn, cs);
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
