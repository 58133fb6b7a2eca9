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
#include <thread>
#include <vector>

#include "farpair.h"
#include "hmat.h"
#include "internal.h"

namespace rfcmp {

namespace {

// ---------------------------------------------------------------- T_A tiles
// One workgroup per pair of edge tiles (I <= J, kEdgeTile consecutive edges
// each) forms the T_A entries (m in I, n in J) straight from the cell pairs
// of the cells the two tiles touch: T_A[m,n] sums the four blocks
// B[(m+-), (n+-)], and each cell pair adds its B entries to the entries of
// its edges that lie in the tiles.  The sums run in LDS in a fixed order
// without atomics: t1 = B[m+,n+] + B[m-,n-], t2 = B[m+,n-] + B[m-,n+], the
// contributions whose row cell is c+ added in a first phase and those whose
// row cell is c- in a second (each entry of t1 or t2 has one contribution
// per phase), and T_A = t1 + t2 -- the same pairing whatever the order of
// the cell pairs.  A diagonal tile takes each unordered cell pair once and
// adds it to (m, n) and (n, m) from the same registers, and every other tile
// pair writes its transpose too: T_A is stored whole and exactly
// symmetric.  Near cell pairs (the self pairs among them)
// take their blocks from k_near_pairs (NB, FP64 singular extraction, run
// first) instead of the far rule: a tile pair that has near cell pairs
// (tile_near) looks each of its cell pairs up in the sorted near partners of
// its row cell.  V[c, c'] = I_0 of a far pair is written by the one
// workgroup whose tiles are the home tiles of c and c' (k_near_pairs writes
// the near ones).
constexpr int kAsmThreads = 1024;
struct CellL {
  float4 q[kQ];   // quadrature points minus centroid
  float4 fv[3];   // vertices minus centroid
  double cen[3];
  float sg[3];
  int rows;       // rows of the three local edges in this tile (8 bits each)
  int gid;        // cell index
  int home;       // home tile
};

__global__ __launch_bounds__(kAsmThreads) void k_assemble_ta(int N, const int* __restrict__ et_ptr,
                                                             const int* __restrict__ et_cell,
                                                             const int* __restrict__ et_rows,
                                                             const int* __restrict__ cell_home,
                                                             const double* __restrict__ cen,
                                                             const float4* __restrict__ qoff,
                                                             const float4* __restrict__ fvoff,
                                                             const float* __restrict__ sgn, float kk,
                                                             RuleArgs rule, const uint8_t* __restrict__ tile_near,
                                                             const int* __restrict__ np_ptr,
                                                             const int* __restrict__ np_other,
                                                             const int* __restrict__ np_code,
                                                             const float2* __restrict__ NB,
                                                             float2* __restrict__ TA, long ldA,
                                                             float2* __restrict__ Vm, long ldV,
                                                             const int2* __restrict__ lst,
                                                             const long* __restrict__ vdoff,
                                                             const int* __restrict__ cstart,
                                                             const int* __restrict__ ipc,
                                                             const float2* __restrict__ NV) {
  const long t = blockIdx.x;
  int I, Jt;
  if (lst) {  // list mode: the dense blocks of a compressed operator
    I = lst[t].x;
    Jt = lst[t].y;
  } else {
    long J = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > t) --J;
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    I = (int)(t - J * (J + 1) / 2);
    Jt = (int)J;
  }
  extern __shared__ __align__(16) unsigned char smem[];
  float2(*t1)[kEdgeTile] = reinterpret_cast<float2(*)[kEdgeTile]>(smem);
  float2(*t2)[kEdgeTile] = reinterpret_cast<float2(*)[kEdgeTile]>(smem + sizeof(float2) * kEdgeTile * kEdgeTile);
  CellL* cl = reinterpret_cast<CellL*>(smem + 2 * sizeof(float2) * kEdgeTile * kEdgeTile);
  const bool diag = I == Jt;
  const int i0 = et_ptr[I], nI = et_ptr[I + 1] - i0, j0 = et_ptr[Jt], nJ = et_ptr[Jt + 1] - j0;
  const int ncell = diag ? nI : nI + nJ;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * kEdgeTile * kEdgeTile; e += kAsmThreads)
    reinterpret_cast<float2*>(smem)[e] = make_float2(0.f, 0.f);
  for (int e = tid; e < ncell * kQ; e += kAsmThreads) {
    const int k = e / kQ, q = e % kQ;
    const int g = k < nI ? et_cell[i0 + k] : et_cell[j0 + k - nI];
    cl[k].q[q] = qoff[(long)g * kQ + q];
  }
  for (int k = tid; k < ncell; k += kAsmThreads) {
    const int g = k < nI ? et_cell[i0 + k] : et_cell[j0 + k - nI];
    CellL& c = cl[k];
    c.rows = k < nI ? et_rows[i0 + k] : et_rows[j0 + k - nI];
    c.gid = g;
    c.home = cell_home[g];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      c.fv[i] = fvoff[(long)g * 3 + i];
      c.sg[i] = sgn[(long)g * 3 + i];
      c.cen[i] = cen[(long)g * 3 + i];
    }
  }
  __syncthreads();
  const CellL* cI = cl;
  const CellL* cJ = diag ? cl : cl + nI;
  const bool any_near = lst ? true : tile_near[t] != 0;
  // list mode: V entries of the home cells of I and J, into the block's
  // own dense V block (rows the cells homed in I, columns those in J)
  const long vbase = lst ? vdoff[t] : 0;
  const int vcI = lst ? cstart[I] : 0, vcJ = lst ? cstart[Jt] : 0;
  const int vnJ = lst ? cstart[Jt + 1] - vcJ : 0;
  const int total = nI * nJ;
  for (int base = 0; base < total; base += kAsmThreads) {
    const int p = base + tid;
    const int a = p / nJ, b = p % nJ;
    // a diagonal tile takes each unordered pair once, the self pairs too
    const bool act = p < total && (!diag || a <= b);
    float2 bv[3][3];
    int ra = 0, rb = 0;
    float sa[3] = {0, 0, 0}, sb[3] = {0, 0, 0};
    bool self = false;
    if (act) {
      const CellL& A = cI[a];
      const CellL& Bc = cJ[b];
      self = A.gid == Bc.gid;
      int code = -1;
      if (any_near) {  // binary search of Bc among A's near partners
        int lo = np_ptr[A.gid], hi = np_ptr[A.gid + 1];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (np_other[mid] < Bc.gid)
            lo = mid + 1;
          else
            hi = mid;
        }
        if (lo < np_ptr[A.gid + 1] && np_other[lo] == Bc.gid) code = np_code[lo];
      }
      if (code >= 0) {
        // near: B[(A,i),(Bc,j)] of the pair stored as (A, Bc) (t = 0) or (Bc, A)
        const float2* nb = NB + (long)(code >> 1) * 9;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) bv[i][j] = nb[(code & 1) ? 3 * j + i : 3 * i + j];
        if (lst && A.home == I && Bc.home == Jt) {
          const float2 v = NV[code >> 1];
          const int la = ipc[A.gid] - vcI, lb = ipc[Bc.gid] - vcJ;
          Vm[vbase + (long)la * vnJ + lb] = v;
          if (diag) Vm[vbase + (long)lb * vnJ + la] = v;
        }
      } else {
        Moments M;
        far_moments(A.q, Bc.q, (float)(A.cen[0] - Bc.cen[0]), (float)(A.cen[1] - Bc.cen[1]),
                        (float)(A.cen[2] - Bc.cen[2]), rule, kk, M);
        if (A.home == I && Bc.home == Jt) {
          const float2 v = make_float2(M.i0r, M.i0i);
          if (lst) {
            const int la = ipc[A.gid] - vcI, lb = ipc[Bc.gid] - vcJ;
            Vm[vbase + (long)la * vnJ + lb] = v;
            if (diag) Vm[vbase + (long)lb * vnJ + la] = v;
          } else {
            Vm[(long)A.gid * ldV + Bc.gid] = v;
            Vm[(long)Bc.gid * ldV + A.gid] = v;
          }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) bv[i][j] = b_entry(M, A.fv[i], Bc.fv[j], A.sg[i], Bc.sg[j]);
      }
      ra = A.rows;
      rb = Bc.rows;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        sa[i] = A.sg[i];
        sb[i] = Bc.sg[i];
      }
    }
    // phase 0: contributions whose row cell is the edge's c+, phase 1: c-
#pragma unroll
    for (int phase = 0; phase < 2; ++phase) {
      if (act) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int r = (ra >> (8 * i)) & 0xFF;
          if (r == 0xFF) continue;
          const bool pa = sa[i] > 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const int c = (rb >> (8 * j)) & 0xFF;
            if (c == 0xFF) continue;
            const bool pb = sb[j] > 0.f;
            float2(*T)[kEdgeTile] = pa == pb ? t1 : t2;
            if ((phase == 0) == pa) {
              T[r][c].x += bv[i][j].x;
              T[r][c].y += bv[i][j].y;
            }
            if (diag && !self && (phase == 0) == pb) {
              T[c][r].x += bv[i][j].x;
              T[c][r].y += bv[i][j].y;
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (lst) {  // the tile as it is (both triangles for a diagonal tile; zero beyond N)
    float2* out = TA + t * (long)(kEdgeTile * kEdgeTile);
    for (int e = tid; e < kEdgeTile * kEdgeTile; e += kAsmThreads) {
      const int r = e / kEdgeTile, c = e % kEdgeTile;
      out[e] = make_float2(t1[r][c].x + t2[r][c].x, t1[r][c].y + t2[r][c].y);
    }
    return;
  }
  for (int e = tid; e < kEdgeTile * kEdgeTile; e += kAsmThreads) {
    const int r = e / kEdgeTile, c = e % kEdgeTile;
    const long m = (long)I * kEdgeTile + r, n = (long)Jt * kEdgeTile + c;
    if (m < N && n < N)
      TA[m * ldA + n] = make_float2(t1[r][c].x + t2[r][c].x, t1[r][c].y + t2[r][c].y);
  }
  if (!diag) {  // the transpose: T_A is stored whole
    for (int e = tid; e < kEdgeTile * kEdgeTile; e += kAsmThreads) {
      const int c = e / kEdgeTile, r = e % kEdgeTile;
      const long m = (long)I * kEdgeTile + r, n = (long)Jt * kEdgeTile + c;
      if (m < N && n < N)
        TA[n * ldA + m] = make_float2(t1[r][c].x + t2[r][c].x, t1[r][c].y + t2[r][c].y);
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
                                                    RuleArgs rule, float2* __restrict__ NB,
                                                    float2* __restrict__ Vm, long ldV,
                                                    float2* __restrict__ NV) {
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
  if (NV) {  // compressed operator: V of the pair, placed by the tile kernel
    NV[t] = v;
  } else {
    Vm[(long)c * ldV + cp] = v;
    Vm[(long)cp * ldV + c] = v;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) NB[t * 9 + 3 * i + j] = make_float2((float)br[i][j], (float)bi[i][j]);
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


}  // namespace

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
  std::vector<int> et_ptr, et_cell, et_rows, home;
  int cmax = 0;
  edge_tiles(h, et_ptr, et_cell, et_rows, home, cmax);
  d.etiles = (int64_t)et_ptr.size() - 1;
  d.et_cells_max = cmax;
  RF_TRY(up(d.et_ptr, et_ptr.data(), sizeof(int) * et_ptr.size()));
  RF_TRY(up(d.et_cell, et_cell.data(), sizeof(int) * et_cell.size()));
  RF_TRY(up(d.et_rows, et_rows.data(), sizeof(int) * et_rows.size()));
  RF_TRY(up(d.cell_home, home.data(), sizeof(int) * C));
  RF_HIP(hipStreamSynchronize(s));  // host staging vectors die here
  return RFCMP_OK;
}

rfcmp_status assemble_blocks(rfcmp_op op, hipStream_t s) {
  rfcmp_mesh m = op->mesh;
  const MeshHost& h = m->h;
  MeshDev& d = m->d;
  const int64_t N = h.N;
  const RuleArgs ra = rule_args();
  HmOp* hm = op->hm.get();
  if (!hm) RF_HIP(hipMemsetAsync(op->Vb.p, 0, op->Vb.bytes, s));

  const long nt = (long)d.etiles;
  const long npairs_t = nt * (nt + 1) / 2;
  // the near pairs (computed on a host thread from mesh creation on): their
  // blocks first, which the T_A tiles read
  if (d.near_factor != op->opt.near_factor) {
    NearData nd;
    if (m->near_async.valid() && m->near_async_factor == op->opt.near_factor)
      nd = m->near_async.get();
    else
      near_data(h, op->opt.near_factor, nd);
    const int64_t np = (int64_t)nd.pairs.size() / 2;
    RF_TRY(d.near.alloc(sizeof(int) * std::max<int64_t>(2 * np, 2)));
    RF_TRY(d.nearB.alloc(sizeof(float2) * 9 * std::max<int64_t>(np, 1)));
    RF_TRY(d.np_ptr.alloc(sizeof(int) * nd.ptr.size()));
    RF_TRY(d.np_other.alloc(sizeof(int) * std::max<size_t>(nd.other.size(), 1)));
    RF_TRY(d.np_code.alloc(sizeof(int) * std::max<size_t>(nd.code.size(), 1)));
    RF_TRY(d.tile_near.alloc(std::max<size_t>(nd.tile_near.size(), 1)));
    d.near_host = std::move(nd);  // the sources stay alive with the mesh
    const NearData& q = d.near_host;
    auto copy = [&](DevBuf& dst, const void* src, size_t bytes) -> rfcmp_status {
      if (bytes) RF_HIP(hipMemcpyAsync(dst.p, src, bytes, hipMemcpyHostToDevice, s));
      return RFCMP_OK;
    };
    RF_TRY(copy(d.near, q.pairs.data(), sizeof(int) * q.pairs.size()));
    RF_TRY(copy(d.np_ptr, q.ptr.data(), sizeof(int) * q.ptr.size()));
    RF_TRY(copy(d.np_other, q.other.data(), sizeof(int) * q.other.size()));
    RF_TRY(copy(d.np_code, q.code.data(), sizeof(int) * q.code.size()));
    RF_TRY(copy(d.tile_near, q.tile_near.data(), q.tile_near.size()));
    d.npairs = np;
    d.near_factor = op->opt.near_factor;
  }
  const long npairs = (long)d.npairs;
  if (hm) RF_TRY(hm->NV.alloc(sizeof(float2) * std::max<long>(npairs, 1)));
  if (npairs > 0) {
    ProfScope prof("near_pairs", s);
    hipLaunchKernelGGL(k_near_pairs, dim3((unsigned)((npairs + 127) / 128)), dim3(128), 0, s, npairs,
                       d.near.as<int>(), d.vtx.as<double>(), d.area.as<double>(), d.sgn.as<float>(), op->k, ra,
                       d.nearB.as<float2>(), hm ? nullptr : op->Vb.as<float2>(), (long)op->ldV,
                       hm ? hm->NV.as<float2>() : nullptr);
    RF_HIP(hipGetLastError());
  }
  if (hm) {
    // compressed: the dense blocks (pairs of tiles of the permuted order),
    // then ACA of the low-rank blocks
    const HmMesh& H = *m->hm;
    const int64_t nd = (int64_t)H.t.dense_I.size();
    RF_TRY(hm->TAd.alloc(sizeof(float2) * kEdgeTile * kEdgeTile * std::max<int64_t>(nd, 1)));
    RF_TRY(hm->Vd.alloc(sizeof(float2) * std::max<int64_t>(H.vd_total, 1)));
    RF_HIP(hipMemsetAsync(hm->Vd.p, 0, hm->Vd.bytes, s));
    if (nd > 0) {
      ProfScope prof("hm_dense", s);
      const size_t lds = 2 * sizeof(float2) * kEdgeTile * kEdgeTile + 2 * sizeof(CellL) * (size_t)H.t.et_cells_max;
      hipLaunchKernelGGL(k_assemble_ta, dim3((unsigned)nd), dim3(kAsmThreads),
                         lds, s, (int)N, H.et_ptr.as<int>(), H.et_cell.as<int>(), H.et_rows.as<int>(),
                         H.home.as<int>(), d.cen.as<double>(), d.qoff.as<float4>(), d.fvoff.as<float4>(),
                         d.sgn.as<float>(), (float)op->k, ra, (const uint8_t*)nullptr, d.np_ptr.as<int>(),
                         d.np_other.as<int>(), d.np_code.as<int>(), d.nearB.as<float2>(), hm->TAd.as<float2>(),
                         (long)kEdgeTile, hm->Vd.as<float2>(), 0L, H.dense_ij.as<int2>(), H.vd_off.as<long>(),
                         H.cell_start.as<int>(), H.iperm_c.as<int>(), hm->NV.as<float2>());
      RF_HIP(hipGetLastError());
    }
    hm->dense_entries[0] = nd * kEdgeTile * kEdgeTile;
    hm->dense_entries[1] = H.vd_total;
    return hm_aca(op, s);
  }
  {
    ProfScope prof("assemble_ta", s);
    const size_t lds = 2 * sizeof(float2) * kEdgeTile * kEdgeTile + 2 * sizeof(CellL) * (size_t)d.et_cells_max;
    hipLaunchKernelGGL(k_assemble_ta, dim3((unsigned)npairs_t), dim3(kAsmThreads),
                       lds, s, (int)N, d.et_ptr.as<int>(), d.et_cell.as<int>(), d.et_rows.as<int>(),
                       d.cell_home.as<int>(), d.cen.as<double>(), d.qoff.as<float4>(), d.fvoff.as<float4>(),
                       d.sgn.as<float>(), (float)op->k, ra, d.tile_near.as<uint8_t>(), d.np_ptr.as<int>(),
                       d.np_other.as<int>(), d.np_code.as<int>(), d.nearB.as<float2>(), op->TA.as<float2>(),
                       (long)op->ldA, op->Vb.as<float2>(), (long)op->ldV, (const int2*)nullptr,
                       (const long*)nullptr, (const int*)nullptr, (const int*)nullptr, (const float2*)nullptr);
  }
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

void edge_tiles(const MeshHost& h, std::vector<int>& ptr, std::vector<int>& cell, std::vector<int>& rows,
                std::vector<int>& home, int& cmax) {
  const int64_t N = h.N, C = h.C;
  const int64_t nt = (N + kEdgeTile - 1) / kEdgeTile;
  ptr.assign(nt + 1, 0);
  cell.clear();
  rows.clear();
  home.assign(C, 0);
  cmax = 0;
  std::vector<int> cells;
  for (int64_t t = 0; t < nt; ++t) {
    cells.clear();
    for (int64_t e = t * kEdgeTile; e < std::min<int64_t>(N, (t + 1) * kEdgeTile); ++e)
      for (int k = 0; k < 2; ++k) cells.push_back(h.edge_cell[2 * e + k]);
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    for (int c : cells) {
      int r3 = 0;
      for (int i = 0; i < 3; ++i) {
        const int64_t e = h.cell_edge[3 * c + i];
        const int r = (e / kEdgeTile == t) ? int(e % kEdgeTile) : 0xFF;
        r3 |= r << (8 * i);
      }
      cell.push_back(c);
      rows.push_back(r3);
    }
    ptr[t + 1] = (int)cell.size();
    cmax = std::max(cmax, (int)cells.size());
  }
  for (int64_t c = 0; c < C; ++c) home[c] = int(h.cell_edge[3 * c] / kEdgeTile);
}

void near_data(const MeshHost& h, double factor, NearData& out) {
  near_pairs(h, factor, out.pairs);
  const int64_t np = (int64_t)out.pairs.size() / 2, C = h.C, N = h.N;
  const int32_t* pr = out.pairs.data();
  const int64_t nt = (N + kEdgeTile - 1) / kEdgeTile;
  const size_t ntp = (size_t)(nt * (nt + 1) / 2);
  // Contiguous chunks of the pair list on a few threads.  Pass 1 counts each
  // chunk's occurrences of every cell; pass 2 places them, chunk by chunk in
  // list order (the offsets of a chunk follow the earlier chunks' counts), so
  // the result is the one of a single thread, and marks the chunk's tile
  // pairs in a map of its own (or-ed together afterwards).
  const int nthr = np >= 65536 ? (int)std::min<int64_t>(8, std::max(1u, std::thread::hardware_concurrency())) : 1;
  std::vector<std::vector<int32_t>> cnt(nthr, std::vector<int32_t>(C, 0));
  std::vector<std::vector<uint8_t>> tmap(nthr);
  auto chunk = [&](int t, int64_t& p0, int64_t& p1) {
    p0 = np * t / nthr;
    p1 = np * (t + 1) / nthr;
  };
  auto count = [&](int t) {
    int64_t p0, p1;
    chunk(t, p0, p1);
    std::vector<int32_t>& c = cnt[t];
    for (int64_t p = p0; p < p1; ++p) {
      ++c[pr[2 * p]];
      if (pr[2 * p] != pr[2 * p + 1]) ++c[pr[2 * p + 1]];
    }
  };
  auto place = [&](int t) {
    int64_t p0, p1;
    chunk(t, p0, p1);
    std::vector<int32_t>& fill = cnt[t];  // the chunk's offsets by now
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t a = pr[2 * p], b = pr[2 * p + 1];
      out.other[fill[a]] = b;
      out.code[fill[a]++] = int32_t(2 * p);
      if (a != b) {
        out.other[fill[b]] = a;
        out.code[fill[b]++] = int32_t(2 * p + 1);
      }
    }
    std::vector<uint8_t>& m = tmap[t];
    m.assign(ntp, 0);
    for (int64_t p = p0; p < p1; ++p) {
      int64_t ta[3], tb[3];
      for (int i = 0; i < 3; ++i) {
        ta[i] = h.cell_edge[3 * pr[2 * p] + i] / kEdgeTile;
        tb[i] = h.cell_edge[3 * pr[2 * p + 1] + i] / kEdgeTile;
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const int64_t I = std::min(ta[i], tb[j]), J = std::max(ta[i], tb[j]);
          m[(size_t)(J * (J + 1) / 2 + I)] = 1;
        }
    }
  };
  auto run = [&](auto&& fn) {
    std::vector<std::thread> pool;
    try {
      for (int t = 1; t < nthr; ++t) pool.emplace_back(fn, t);
    } catch (const std::system_error&) {
      for (int t = (int)pool.size() + 1; t < nthr; ++t) fn(t);  // no threads to be had: here
    }
    fn(0);
    for (auto& th : pool) th.join();
  };
  run(count);
  // the near partners of every cell, ascending, with 2 p + t.  The list runs
  // in order of its first cell, partners ascending, so placing in list order
  // puts cell c's partners a < c (from the pairs (a, c), in order of a)
  // before its own pairs (c, b), b >= c ascending: already sorted.
  out.ptr.assign(C + 1, 0);
  for (int64_t c = 0; c < C; ++c) {
    int32_t o = out.ptr[c];
    for (int t = 0; t < nthr; ++t) {
      const int32_t k = cnt[t][c];
      cnt[t][c] = o;
      o += k;
    }
    out.ptr[c + 1] = o;
  }
  out.other.resize(out.ptr[C]);
  out.code.resize(out.ptr[C]);
  run(place);
  // edge-tile pairs (I <= J) that hold a near cell pair
  out.tile_near.assign(ntp, 0);
  for (int t = 0; t < nthr; ++t)
    for (size_t q = 0; q < ntp; ++q) out.tile_near[q] |= tmap[t][q];
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
