// Solves with the sparse projector factors on the device (FP64), and the
// upload of a host factor.  See spchol.h.
//
// One workgroup per right-hand side (and factor of a pair).  The input is
// formed while it is permuted into the scratch (the operator's Sigma^T and
// Lambda^T gathers, as in the dense products); the dissection levels are
// then run as flat phases of independent row tasks (fronts, column tasks,
// struct tasks forward; two column phases backward), separated by workgroup
// barriers, and the result is permuted back.  For the grounded Laplacian
// factor the input and the output are made mean-free (L^+).  Every sum runs
// in a fixed order: the results do not depend on timing.
#include <algorithm>

#include "spchol.h"
#include "symv_input.h"

namespace rfcmp {
namespace {

struct SpArg {
  int n, nlev, grounded, nrhs;
  const int *perm, *iperm, *str;
  const int *fr_lvl, *fr_dest, *fr_xsrc, *fr_ptr, *fr_src;
  const int *col_lvl, *str_lvl;
  const int4* lanes;
  const int4* col_a;
  const long2* col_b;
  const int2* col_c;
  const int4* str_a;
  const long2* str_b;
  const int2* str_c;
  const double *l21, *l21t, *linv, *linvt;
  SymvInput in;
  double2* y;
  double2* scratch;
  long sstride;      // scratch entries per right-hand side
  long nstr_total;
};
struct SpArgs {
  SpArg a[2];
};

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cfma(double a, double2 v, double2 acc) {
  return make_double2(fma(a, v.x, acc.x), fma(a, v.y, acc.y));
}

// Sum over the workgroup, in a fixed order (lane sums, then wave sums in
// order); red: LDS space of one double2 per wave.
__device__ double2 block_sum(double2 v, double2* red) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  for (int w = 0; w < W; ++w) t = cadd(t, red[w]);
  return t;
}

constexpr int kSpThreads = 1024;

// Sum over the G lanes of a task's group (G a power of two <= 64, the group
// aligned in the wave), in a fixed order; every lane of the wave takes part.
__device__ inline double2 group_sum(double2 v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

__global__ void __launch_bounds__(kSpThreads) k_spsolve(const SpArgs args) {
  const SpArg& A = args.a[blockIdx.y];
  const int r = blockIdx.x;
  if (r >= A.nrhs) return;
  __shared__ double2 red[kSpThreads / 64];
  const int n = A.n;
  double2* x = A.scratch + (long)r * A.sstride;
  double2* z = x + n;
  double2* u = z + n;
  double2* fr = u + A.nstr_total;
  const int tid = threadIdx.x, nt = blockDim.x;

  // permuted input; mean-free for the Laplacian
  double2 s = make_double2(0.0, 0.0);
  for (int i = tid; i < n; i += nt) {
    const double2 v = input_entry(A.in, r, A.perm[i]);
    x[i] = v;
    s = cadd(s, v);
  }
  if (A.grounded) {
    const double2 t = block_sum(s, red);
    const double2 mean = make_double2(t.x / n, t.y / n);
    for (int i = tid; i < n; i += nt) x[i] = make_double2(x[i].x - mean.x, x[i].y - mean.y);
  }
  __syncthreads();

  // forward, heights up
  for (int h = 0; h < A.nlev; ++h) {
    // fronts: own entries plus the children's update vectors, in child order
    for (int k = A.fr_lvl[h] + tid; k < A.fr_lvl[h + 1]; k += nt) {
      const int xs = A.fr_xsrc[k];
      double2 v = xs >= 0 ? x[xs] : make_double2(0.0, 0.0);
      for (int q = A.fr_ptr[k]; q < A.fr_ptr[k + 1]; ++q) v = cadd(v, u[A.fr_src[q]]);
      fr[A.fr_dest[k]] = v;
    }
    __syncthreads();
    // y_i = (L_ss^-1 v)_i: row i of the inverse, columns j <= i
    {
      const int4 G4 = A.lanes[h];
      const int G = G4.x, per = nt / G, g = tid & (G - 1), slot = tid / G;
      for (int base = A.col_lvl[h]; base < A.col_lvl[h + 1]; base += per) {
        const int k = base + slot;
        double2 acc = make_double2(0.0, 0.0);
        if (k < A.col_lvl[h + 1]) {
          const int4 t = A.col_a[k];  // {c0, ncol, i, front}
          const double* L = A.linv + A.col_b[k].x + t.z;  // (i, j) at L[j * ncol]
          const double2* v = fr + t.w;
          double2 a1 = acc, a2 = acc, a3 = acc;
          int j = g;
          for (; j + 3 * G <= t.z; j += 4 * G) {
            const double l0 = L[(long)j * t.y], l1 = L[(long)(j + G) * t.y];
            const double l2 = L[(long)(j + 2 * G) * t.y], l3 = L[(long)(j + 3 * G) * t.y];
            acc = cfma(l0, v[j], acc);
            a1 = cfma(l1, v[j + G], a1);
            a2 = cfma(l2, v[j + 2 * G], a2);
            a3 = cfma(l3, v[j + 3 * G], a3);
          }
          for (; j <= t.z; j += G) acc = cfma(L[(long)j * t.y], v[j], acc);
          acc = cadd(cadd(acc, a1), cadd(a2, a3));
        }
        acc = group_sum(acc, G);
        if (k < A.col_lvl[h + 1] && g == 0) {
          const int4 t = A.col_a[k];
          x[t.x + t.z] = acc;
        }
      }
    }
    __syncthreads();
    // u_t = v_(ncol + t) - (L_21 y)_t
    {
      const int4 G4 = A.lanes[h];
      const int G = G4.y, per = nt / G, g = tid & (G - 1), slot = tid / G;
      for (int base = A.str_lvl[h]; base < A.str_lvl[h + 1]; base += per) {
        const int k = base + slot;
        double2 acc = make_double2(0.0, 0.0);
        if (k < A.str_lvl[h + 1]) {
          const int4 t = A.str_a[k];   // {c0, ncol, t, front}
          const long2 b = A.str_b[k];  // {L_21 offset + t, u index}
          const int nstr = A.str_c[k].x;
          const double* L = A.l21 + b.x;  // (t, j) at L[j * nstr]
          const double2* y = x + t.x;
          double2 a1 = acc, a2 = acc, a3 = acc;
          int j = g;
          for (; j + 3 * G < t.y; j += 4 * G) {
            const double l0 = L[(long)j * nstr], l1 = L[(long)(j + G) * nstr];
            const double l2 = L[(long)(j + 2 * G) * nstr], l3 = L[(long)(j + 3 * G) * nstr];
            acc = cfma(l0, y[j], acc);
            a1 = cfma(l1, y[j + G], a1);
            a2 = cfma(l2, y[j + 2 * G], a2);
            a3 = cfma(l3, y[j + 3 * G], a3);
          }
          for (; j < t.y; j += G) acc = cfma(L[(long)j * nstr], y[j], acc);
          acc = cadd(cadd(acc, a1), cadd(a2, a3));
        }
        acc = group_sum(acc, G);
        if (k < A.str_lvl[h + 1] && g == 0) {
          const int4 t = A.str_a[k];
          const double2 v = fr[t.w + t.y + t.z];
          u[A.str_b[k].y] = make_double2(v.x - acc.x, v.y - acc.y);
        }
      }
    }
    __syncthreads();
  }

  // backward, heights down
  for (int h = A.nlev - 1; h >= 0; --h) {
    // z_j = y_j - (L_21^T x_struct)_j
    {
      const int4 G4 = A.lanes[h];
      const int G = G4.z, per = nt / G, g = tid & (G - 1), slot = tid / G;
      for (int base = A.col_lvl[h]; base < A.col_lvl[h + 1]; base += per) {
        const int k = base + slot;
        double2 acc = make_double2(0.0, 0.0);
        if (k < A.col_lvl[h + 1]) {
          const int4 t = A.col_a[k];  // {c0, ncol, j, front}
          const int2 c = A.col_c[k];  // {so, nstr}
          const double* L = A.l21t + A.col_b[k].y + t.z;  // (q, j) at L[q * ncol]
          const int* srow = A.str + c.x;
          double2 a1 = acc, a2 = acc, a3 = acc;
          int q = g;
          for (; q + 3 * G < c.y; q += 4 * G) {
            const double l0 = L[(long)q * t.y], l1 = L[(long)(q + G) * t.y];
            const double l2 = L[(long)(q + 2 * G) * t.y], l3 = L[(long)(q + 3 * G) * t.y];
            const int r0 = srow[q], r1 = srow[q + G], r2 = srow[q + 2 * G], r3 = srow[q + 3 * G];
            acc = cfma(l0, x[r0], acc);
            a1 = cfma(l1, x[r1], a1);
            a2 = cfma(l2, x[r2], a2);
            a3 = cfma(l3, x[r3], a3);
          }
          for (; q < c.y; q += G) acc = cfma(L[(long)q * t.y], x[srow[q]], acc);
          acc = cadd(cadd(acc, a1), cadd(a2, a3));
        }
        acc = group_sum(acc, G);
        if (k < A.col_lvl[h + 1] && g == 0) {
          const int4 t = A.col_a[k];
          const double2 y = x[t.x + t.z];
          z[t.x + t.z] = make_double2(y.x - acc.x, y.y - acc.y);
        }
      }
    }
    __syncthreads();
    // x_i = (L_ss^-T z)_i: column i of the inverse, rows j >= i
    {
      const int4 G4 = A.lanes[h];
      const int G = G4.w, per = nt / G, g = tid & (G - 1), slot = tid / G;
      for (int base = A.col_lvl[h]; base < A.col_lvl[h + 1]; base += per) {
        const int k = base + slot;
        double2 acc = make_double2(0.0, 0.0);
        if (k < A.col_lvl[h + 1]) {
          const int4 t = A.col_a[k];
          const double* L = A.linvt + A.col_b[k].x + t.z;  // (j, i) of the inverse at L[j * ncol]
          const double2* zz = z + t.x;
          double2 a1 = acc, a2 = acc, a3 = acc;
          int j = t.z + g;
          for (; j + 3 * G < t.y; j += 4 * G) {
            const double l0 = L[(long)j * t.y], l1 = L[(long)(j + G) * t.y];
            const double l2 = L[(long)(j + 2 * G) * t.y], l3 = L[(long)(j + 3 * G) * t.y];
            acc = cfma(l0, zz[j], acc);
            a1 = cfma(l1, zz[j + G], a1);
            a2 = cfma(l2, zz[j + 2 * G], a2);
            a3 = cfma(l3, zz[j + 3 * G], a3);
          }
          for (; j < t.y; j += G) acc = cfma(L[(long)j * t.y], zz[j], acc);
          acc = cadd(cadd(acc, a1), cadd(a2, a3));
        }
        acc = group_sum(acc, G);
        if (k < A.col_lvl[h + 1] && g == 0) {
          const int4 t = A.col_a[k];
          x[t.x + t.z] = acc;
        }
      }
    }
    __syncthreads();
  }

  // back to the original order; mean-free for the Laplacian
  double2 mean = make_double2(0.0, 0.0);
  if (A.grounded) {
    double2 t = make_double2(0.0, 0.0);
    for (int i = tid; i < n; i += nt) t = cadd(t, x[i]);
    t = block_sum(t, red);
    mean = make_double2(t.x / n, t.y / n);
  }
  double2* yr = A.y + (long)r * n;
  for (int g = tid; g < n; g += nt) {
    const double2 v = x[A.iperm[g]];
    yr[g] = make_double2(v.x - mean.x, v.y - mean.y);
  }
}

}  // namespace

rfcmp_status spsolve_jobs(const SpSolveJob* jobs, int njobs, int nrhs, hipStream_t s, const char* tag) {
  if (njobs < 1 || njobs > 2 || nrhs <= 0) {
    set_error("spsolve: 1 or 2 jobs and nrhs > 0 required");
    return RFCMP_E_ARG;
  }
  SpArgs args{};
  for (int q = 0; q < njobs; ++q) {
    const SpDevice& F = *jobs[q].F;
    SpArg& a = args.a[q];
    a.n = F.n;
    a.nlev = F.nlev;
    a.grounded = F.grounded;
    a.perm = F.perm.as<int>();
    a.iperm = F.iperm.as<int>();
    a.str = F.str.as<int>();
    a.fr_lvl = F.fr_lvl.as<int>();
    a.fr_dest = F.fr_dest.as<int>();
    a.fr_xsrc = F.fr_xsrc.as<int>();
    a.fr_ptr = F.fr_ptr.as<int>();
    a.fr_src = F.fr_src.as<int>();
    a.col_lvl = F.col_lvl.as<int>();
    a.lanes = F.lanes.as<int4>();
    a.str_lvl = F.str_lvl.as<int>();
    a.col_a = F.col_a.as<int4>();
    a.col_b = F.col_b.as<long2>();
    a.col_c = F.col_c.as<int2>();
    a.str_a = F.str_a.as<int4>();
    a.str_b = F.str_b.as<long2>();
    a.str_c = F.str_c.as<int2>();
    a.l21 = F.l21.as<double>();
    a.l21t = F.l21t.as<double>();
    a.linv = F.linv.as<double>();
    a.linvt = F.linvt.as<double>();
    a.in = jobs[q].in;
    a.y = jobs[q].y;
    a.scratch = jobs[q].scratch;
    a.sstride = F.scratch_entries();
    a.nstr_total = F.nstr_total;
    a.nrhs = (q == 1 && jobs[1].nrhs > 0) ? std::min(jobs[1].nrhs, nrhs) : nrhs;
  }
  ProfScope prof(tag, s);
  hipLaunchKernelGGL(k_spsolve, dim3((unsigned)nrhs, (unsigned)njobs), dim3(kSpThreads), 0, s, args);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

void spchol_arrays(const SpFactor& F, SpArrays& a) {
  const int n = F.n, nsn = F.nsn;
  int H = 0;
  for (int q = 0; q < nsn; ++q) H = std::max(H, F.height[q]);
  a.nlev = H + 1;
  std::vector<std::vector<int>> by_h(H + 1);
  for (int q = 0; q < nsn; ++q) by_h[F.height[q]].push_back(q);
  // block offsets and front offsets
  std::vector<long> linv_off(nsn + 1, 0), l21_off(nsn + 1, 0);
  std::vector<int> front_off(nsn + 1, 0);
  a.max_ncol = 0;
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    linv_off[q + 1] = linv_off[q] + (long)ncol * ncol;
    l21_off[q + 1] = l21_off[q] + (long)nstr * ncol;
    front_off[q + 1] = front_off[q] + ncol + nstr;
    a.max_ncol = std::max(a.max_ncol, ncol);
  }
  a.front_total = front_off[nsn];
  // matrices: L_21 (nstr x ncol, column-major) and its transpose; the inverse
  // of the diagonal block (column-major) and its transpose
  a.l21.assign(l21_off[nsn], 0.0);
  a.l21t.assign(l21_off[nsn], 0.0);
  a.linv.assign(linv_off[nsn], 0.0);
  a.linvt.assign(linv_off[nsn], 0.0);
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    const int m = ncol + nstr;
    const double* P = &F.panel[F.panel_off[q]];
    for (int j = 0; j < ncol; ++j)
      for (int t = 0; t < nstr; ++t) {
        const double v = P[(size_t)j * m + ncol + t];
        a.l21[l21_off[q] + (long)j * nstr + t] = v;
        a.l21t[l21_off[q] + (long)t * ncol + j] = v;
      }
    // Z = L_ss^-1 column by column, by forward substitution on e_c
    double* Z = &a.linv[linv_off[q]];
    for (int c = 0; c < ncol; ++c)
      for (int i = c; i < ncol; ++i) {
        double acc = i == c ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) acc -= P[(size_t)k * m + i] * Z[(size_t)c * ncol + k];
        Z[(size_t)c * ncol + i] = acc / P[(size_t)i * m + i];
      }
    double* ZT = &a.linvt[linv_off[q]];
    for (int c = 0; c < ncol; ++c)
      for (int i = 0; i < ncol; ++i) ZT[(size_t)i * ncol + c] = Z[(size_t)c * ncol + i];
  }
  // tasks by level
  a.fr_lvl.assign(1, 0);
  a.col_lvl.assign(1, 0);
  a.str_lvl.assign(1, 0);
  a.fr_dest.clear();
  a.fr_xsrc.clear();
  a.fr_ptr.assign(1, 0);
  a.fr_src.clear();
  a.col_a.clear();
  a.col_b.clear();
  a.col_c.clear();
  a.str_a.clear();
  a.str_b.clear();
  a.str_c.clear();
  for (int h = 0; h <= H; ++h) {
    for (int q : by_h[h]) {
      const int c0 = F.col0[q], ncol = F.col0[q + 1] - c0;
      const int so = F.str_off[q], nstr = F.str_off[q + 1] - so;
      const int m = ncol + nstr;
      // front gathers: per entry, the child update entries that land there
      std::vector<std::vector<int>> src(m);
      for (int qc = F.child_off[q]; qc < F.child_off[q + 1]; ++qc) {
        const int c = F.child_idx[qc];
        for (int t = F.str_off[c]; t < F.str_off[c + 1]; ++t) src[F.map[t]].push_back(t);
      }
      for (int p = 0; p < m; ++p) {
        a.fr_dest.push_back(front_off[q] + p);
        a.fr_xsrc.push_back(p < ncol ? c0 + p : -1);
        for (int t : src[p]) a.fr_src.push_back(t);
        a.fr_ptr.push_back((int)a.fr_src.size());
      }
      for (int i = 0; i < ncol; ++i) {
        a.col_a.insert(a.col_a.end(), {c0, ncol, i, front_off[q]});
        a.col_b.insert(a.col_b.end(), {linv_off[q], l21_off[q]});
        a.col_c.insert(a.col_c.end(), {so, nstr});
      }
      for (int t = 0; t < nstr; ++t) {
        a.str_a.insert(a.str_a.end(), {c0, ncol, t, front_off[q]});
        a.str_b.insert(a.str_b.end(), {l21_off[q] + t, (long)so + t});
        a.str_c.insert(a.str_c.end(), {nstr, 0});
      }
    }
    a.fr_lvl.push_back((int)a.fr_dest.size());
    a.col_lvl.push_back((int)(a.col_a.size() / 4));
    a.str_lvl.push_back((int)(a.str_a.size() / 4));
  }
  // lanes per task: grow G while the level's tasks still fit one pass of the
  // workgroup and each lane keeps at least four terms
  a.lanes.clear();
  for (int h = 0; h <= H; ++h) {
    int ncol_sum = 0, nstr_sum = 0, ncol_max = 0, nstr_max = 0;
    for (int q : by_h[h]) {
      const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
      ncol_sum += ncol;
      nstr_sum += nstr;
      ncol_max = std::max(ncol_max, ncol);
      nstr_max = std::max(nstr_max, nstr);
    }
    auto pick = [](int tasks, int len) {
      int G = 1;
      while (G < 64 && (long)tasks * G * 2 <= kSpThreads && G * 8 <= len) G *= 2;
      return G;
    };
    a.lanes.insert(a.lanes.end(), {pick(ncol_sum, ncol_max), pick(nstr_sum, ncol_max), pick(ncol_sum, nstr_max),
                                   pick(ncol_sum, ncol_max)});
  }
  a.iperm.assign(n, 0);
  for (int i = 0; i < n; ++i) a.iperm[F.perm[i]] = i;
}

rfcmp_status spchol_upload(const SpFactor& F, SpDevice& D, hipStream_t s) {
  const int n = F.n, nsn = F.nsn;
  SpArrays a;
  spchol_arrays(F, a);
  D.n = n;
  D.nsn = nsn;
  D.grounded = F.grounded ? 1 : 0;
  D.max_front = F.max_front;
  D.max_ncol = a.max_ncol;
  D.nlev = a.nlev;
  D.seconds = F.seconds;
  D.nstr_total = F.str_off[nsn];
  D.front_total = a.front_total;
  D.nnz = (int64_t)(a.l21.size() + a.l21t.size() + a.linv.size() + a.linvt.size());
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> rfcmp_status {
    RF_TRY(b.alloc(std::max<size_t>(bytes, 16)));
    if (bytes) RF_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return RFCMP_OK;
  };
  auto upv = [&](DevBuf& b, const auto& v) { return up(b, v.data(), sizeof(v[0]) * v.size()); };
  RF_TRY(upv(D.perm, F.perm));
  RF_TRY(upv(D.iperm, a.iperm));
  RF_TRY(upv(D.str, F.str));
  RF_TRY(upv(D.fr_lvl, a.fr_lvl));
  RF_TRY(upv(D.fr_dest, a.fr_dest));
  RF_TRY(upv(D.fr_xsrc, a.fr_xsrc));
  RF_TRY(upv(D.fr_ptr, a.fr_ptr));
  RF_TRY(upv(D.fr_src, a.fr_src));
  RF_TRY(upv(D.col_lvl, a.col_lvl));
  RF_TRY(upv(D.col_a, a.col_a));
  RF_TRY(upv(D.col_b, a.col_b));
  RF_TRY(upv(D.col_c, a.col_c));
  RF_TRY(upv(D.str_lvl, a.str_lvl));
  RF_TRY(upv(D.lanes, a.lanes));
  RF_TRY(upv(D.str_a, a.str_a));
  RF_TRY(upv(D.str_b, a.str_b));
  RF_TRY(upv(D.str_c, a.str_c));
  RF_TRY(upv(D.l21, a.l21));
  RF_TRY(upv(D.l21t, a.l21t));
  RF_TRY(upv(D.linv, a.linv));
  RF_TRY(upv(D.linvt, a.linvt));
  // the host arrays above are locals: wait for the copies
  RF_HIP(hipStreamSynchronize(s));
  return RFCMP_OK;
}

// Leaf size of the dissection: measured on the level-4 and level-5 spheres
// (16: about 1.3 and 6 MB for L; 64 stores three times the entries of 8).
constexpr int kSpLeaf = 16;

HostFactor factor_mesh_matrix(const MeshHost& h, int which) {
  HostFactor r;
  try {
    SpMatrix A;
    if (which == 0)
      laplacian_matrix(h, A);
    else if (which == 1)
      gram_ll_matrix(h, A);
    else
      gram_tp_matrix(h, A);
    r.F = std::make_shared<SpFactor>();
    r.status = spchol_factor(A, which == 0, kSpLeaf, 1, *r.F);
    if (r.status < 0) r.error = last_error();
  } catch (const std::bad_alloc&) {
    r.status = RFCMP_E_OOM;
    r.error = "host allocation failed in the sparse factorisation";
  }
  return r;
}

rfcmp_status mesh_sparse_projectors(rfcmp_mesh m, bool need_gtp) {
  MeshDev& d = m->d;
  const int nq = need_gtp ? 3 : 2;
  bool todo = false;
  for (int q = 0; q < nq; ++q) todo |= !d.sp[q];
  if (!todo) return RFCMP_OK;
  if (!d.proj_stream[0]) {
    RF_HIP(hipStreamCreateWithFlags(&d.proj_stream[0], hipStreamNonBlocking));
    RF_HIP(hipEventCreateWithFlags(&d.proj_done[0], hipEventDisableTiming));
  }
  for (int q = 0; q < nq; ++q) {
    if (d.sp[q]) continue;
    HostFactor hf;
    if (q < 2 && m->fac_async[q].valid()) {
      hf = m->fac_async[q].get();
    } else {
      if (q == 2) build_cell_nb(m->h);
      hf = factor_mesh_matrix(m->h, q);
    }
    if (hf.status < 0) {
      set_error("%s", hf.error.c_str());
      return hf.status;
    }
    auto dev = std::make_unique<SpDevice>();
    RF_TRY(spchol_upload(*hf.F, *dev, d.proj_stream[0]));
    d.sp[q] = std::move(dev);
  }
  return RFCMP_OK;
}

}  // namespace rfcmp
