// Device-side formation of a product input x[r][g] from a SymvInput (the
// fused gathers of the operator), shared by the dense symmetric products
// (symv.hip) and the sparse projector solves (spsolve.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "symv.h"

namespace rfcmp {

__device__ inline double2 csub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// x[r][g] of a SymvInput (g < n).
__device__ inline double2 input_entry(const SymvInput& in, int r, int g) {
  const double2* p0 = in.p[0] + r * in.stride[0];
  switch (in.mode) {
    case SymvInput::kSigmaT: {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double2 v = p0[in.idx0[3 * g + l]];
        const double sg = in.sgn[3 * g + l];
        sr = fma(sg, v.x, sr);
        si = fma(sg, v.y, si);
      }
      return make_double2(sr, si);
    }
    case SymvInput::kLambdaT: {
      double sr = 0.0, si = 0.0;
      for (int q = in.idx0[g]; q < in.idx0[g + 1]; ++q) {
        const double2 v = p0[in.idx1[q]];
        const double sg = in.sgn[q];
        sr = fma(sg, v.x, sr);
        si = fma(sg, v.y, si);
      }
      return make_double2(sr, si);
    }
    case SymvInput::kVin: {
      const int cp = in.idx0[2 * g], cm = in.idx0[2 * g + 1];
      const double2* p1 = in.p[1] + r * in.stride[1];
      const double2* p2 = in.p[2] + r * in.stride[2];
      const double2 ul = csub2(p0[g], csub2(p1[cp], p1[cm]));
      const double2 ug = csub2(p2[cp], p2[cm]);
      const double ka = in.c[0], kb = in.c[1];
      return make_double2(-ka * ul.y - kb * ug.x, ka * ul.x - kb * ug.y);
    }
    case SymvInput::kMiddleW: {
      const int cp = in.idx0[2 * g], cm = in.idx0[2 * g + 1];
      const double2* p1 = in.p[1] + r * in.stride[1];
      const double2* p2 = in.p[2] + r * in.stride[2];
      const double2* p3 = in.p[3] + r * in.stride[3];
      const double2 lh = csub2(p0[in.idx1[2 * g]], p0[in.idx1[2 * g + 1]]);
      const double2 pl = csub2(p1[g], csub2(p2[cp], p2[cm]));
      const double2 ss = csub2(p3[cp], p3[cm]);
      return make_double2(in.c[0] * lh.x + in.c[1] * pl.x + in.c[2] * ss.x,
                          in.c[0] * lh.y + in.c[1] * pl.y + in.c[2] * ss.y);
    }
    case SymvInput::kProjLH: {
      const int cp = in.idx0[2 * g], cm = in.idx0[2 * g + 1];
      const double2* p1 = in.p[1] + r * in.stride[1];
      return csub2(p0[g], csub2(p1[cp], p1[cm]));
    }
    default:
      return p0[g];
  }
}

}  // namespace rfcmp
