// Solves with the sparse projector factors on the device (FP64), and the
// upload of a host factor.  See spchol.h.
//
// One workgroup per right-hand side (and factor of a pair).  The input is
// formed while it is permuted into the scratch (the operator's Sigma^T and
// Lambda^T gathers, as in the dense products), then:
//   forward, heights up: each supernode is taken by one wave, which builds
//     its front in LDS (its entries of the vector, then its children's update
//     vectors added at their positions), forms y = L_ss^-1 v (a product with
//     the stored inverse of the diagonal block) and its update vector
//     u = v_struct - L_21 y for its parent;
//   backward, heights down: x_s = L_ss^-T (y - L_21^T x_struct), where the
//     struct rows belong to ancestors, already solved;
// and the result is permuted back.  Supernodes of one height are spread over
// the waves; heights are separated by workgroup barriers.  For the grounded
// Laplacian factor the input and the output are made mean-free (L^+).
// Every sum runs in a fixed order: the results do not depend on timing.
#include <algorithm>

#include "spchol.h"
#include "symv_input.h"

namespace rfcmp {
namespace {

struct SpArg {
  int n, nlev, grounded, slice, y_off;  // slice: LDS entries per wave; y part of the slice at y_off
  const int *perm, *iperm, *col0, *str_off, *str, *map, *child_off, *child_idx, *lvl_off, *lvl_node;
  const long *l21_off, *linv_off;
  const double *l21, *linv;
  SymvInput in;
  double2* y;
  double2* scratch;
  long sstride;  // scratch entries per right-hand side
  int nrhs;
};
struct SpArgs {
  SpArg a[2];
};

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cfma(double a, double2 v, double2 acc) {
  return make_double2(fma(a, v.x, acc.x), fma(a, v.y, acc.y));
}

// Order the wave's LDS and global accesses: everything the wave wrote is
// visible to all its lanes afterwards (no other wave is involved).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
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

__global__ void __launch_bounds__(1024) k_spsolve(const SpArgs args) {
  const SpArg& A = args.a[blockIdx.y];
  const int r = blockIdx.x;
  if (r >= A.nrhs) return;
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  double2* red = lds;                       // W entries
  double2* f = lds + W + wave * A.slice;    // the wave's front
  double2* yv = f + A.y_off;                // the wave's diagonal-block solution
  double2* x = A.scratch + (long)r * A.sstride;
  double2* u = x + A.n;
  const int n = A.n;

  // permuted input; mean-free for the Laplacian
  double2 s = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 v = input_entry(A.in, r, A.perm[i]);
    x[i] = v;
    s = cadd(s, v);
  }
  if (A.grounded) {
    const double2 t = block_sum(s, red);
    const double2 mean = make_double2(t.x / n, t.y / n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = make_double2(x[i].x - mean.x, x[i].y - mean.y);
  }
  __syncthreads();

  // forward
  for (int lev = 0; lev < A.nlev; ++lev) {
    for (int q = A.lvl_off[lev] + wave; q < A.lvl_off[lev + 1]; q += W) {
      const int sn = A.lvl_node[q];
      const int c0 = A.col0[sn], ncol = A.col0[sn + 1] - c0;
      const int so = A.str_off[sn], nstr = A.str_off[sn + 1] - so;
      const int m = ncol + nstr;
      for (int i = lane; i < m; i += 64) f[i] = i < ncol ? x[c0 + i] : make_double2(0.0, 0.0);
      wave_sync();
      for (int qc = A.child_off[sn]; qc < A.child_off[sn + 1]; ++qc) {
        const int c = A.child_idx[qc];
        const int cs = A.str_off[c], cn = A.str_off[c + 1] - cs;
        for (int t = lane; t < cn; t += 64) {
          const int p = A.map[cs + t];
          f[p] = cadd(f[p], u[cs + t]);
        }
        wave_sync();
      }
      const double* Li = A.linv + A.linv_off[sn];
      for (int i0 = 0; i0 < ncol; i0 += 64) {
        const int i = i0 + lane;
        const int jend = min(ncol, i0 + 64);
        double2 acc = make_double2(0.0, 0.0);
        if (i < ncol)
          for (int j = 0; j < jend; ++j) acc = cfma(Li[(long)j * ncol + i], f[j], acc);
        if (i < ncol) {
          yv[i] = acc;
          x[c0 + i] = acc;
        }
      }
      wave_sync();
      const double* L2 = A.l21 + A.l21_off[sn];
      for (int t = lane; t < nstr; t += 64) {
        double2 acc = f[ncol + t];
        for (int j = 0; j < ncol; ++j) acc = cfma(-L2[(long)j * nstr + t], yv[j], acc);
        u[so + t] = acc;
      }
      wave_sync();
    }
    __syncthreads();
  }

  // backward
  for (int lev = A.nlev - 1; lev >= 0; --lev) {
    for (int q = A.lvl_off[lev] + wave; q < A.lvl_off[lev + 1]; q += W) {
      const int sn = A.lvl_node[q];
      const int c0 = A.col0[sn], ncol = A.col0[sn + 1] - c0;
      const int so = A.str_off[sn], nstr = A.str_off[sn + 1] - so;
      for (int t = lane; t < nstr; t += 64) f[t] = x[A.str[so + t]];
      wave_sync();
      const double* L2 = A.l21 + A.l21_off[sn];
      for (int j = lane; j < ncol; j += 64) {
        double2 z = x[c0 + j];
        for (int t = 0; t < nstr; ++t) z = cfma(-L2[(long)j * nstr + t], f[t], z);
        yv[j] = z;
      }
      wave_sync();
      const double* Li = A.linv + A.linv_off[sn];
      for (int i = lane; i < ncol; i += 64) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = i; j < ncol; ++j) acc = cfma(Li[(long)i * ncol + j], yv[j], acc);
        x[c0 + i] = acc;
      }
      wave_sync();
    }
    __syncthreads();
  }

  // back to the original order; mean-free for the Laplacian
  double2 mean = make_double2(0.0, 0.0);
  if (A.grounded) {
    double2 t = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < n; i += blockDim.x) t = cadd(t, x[i]);
    t = block_sum(t, red);
    mean = make_double2(t.x / n, t.y / n);
  }
  double2* yr = A.y + (long)r * n;
  for (int g = threadIdx.x; g < n; g += blockDim.x) {
    const double2 v = x[A.iperm[g]];
    yr[g] = make_double2(v.x - mean.x, v.y - mean.y);
  }
}

int lds_limit() {
  static int lim = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      return 65536;
    if (v > 65536) (void)hipFuncSetAttribute((const void*)k_spsolve, hipFuncAttributeMaxDynamicSharedMemorySize, v);
    return v;
  }();
  return lim;
}

}  // namespace

rfcmp_status spsolve_jobs(const SpSolveJob* jobs, int njobs, int nrhs, hipStream_t s, const char* tag) {
  if (njobs < 1 || njobs > 2 || nrhs <= 0) {
    set_error("spsolve: 1 or 2 jobs and nrhs > 0 required");
    return RFCMP_E_ARG;
  }
  SpArgs args{};
  int slice = 0;
  for (int q = 0; q < njobs; ++q) {
    const SpDevice& F = *jobs[q].F;
    slice = std::max(slice, F.max_front + F.max_ncol);
  }
  // waves per workgroup: as many fronts as fit the LDS, at most 16
  const int limit = lds_limit();
  int W = 16;
  while (W > 1 && (size_t)(W + (size_t)W * slice) * sizeof(double2) > (size_t)limit) --W;
  if ((size_t)(W + (size_t)W * slice) * sizeof(double2) > (size_t)limit) {
    set_error("spsolve: a front of %d entries does not fit the %d bytes of LDS", slice, limit);
    return RFCMP_E_STATE;
  }
  for (int q = 0; q < njobs; ++q) {
    const SpDevice& F = *jobs[q].F;
    SpArg& a = args.a[q];
    a.n = F.n;
    a.nlev = F.nlev;
    a.grounded = F.grounded;
    a.slice = slice;
    a.y_off = F.max_front;
    a.perm = F.perm.as<int>();
    a.iperm = F.iperm.as<int>();
    a.col0 = F.col0.as<int>();
    a.str_off = F.str_off.as<int>();
    a.str = F.str.as<int>();
    a.map = F.map.as<int>();
    a.child_off = F.child_off.as<int>();
    a.child_idx = F.child_idx.as<int>();
    a.lvl_off = F.lvl_off.as<int>();
    a.lvl_node = F.lvl_node.as<int>();
    a.l21_off = F.l21_off.as<long>();
    a.linv_off = F.linv_off.as<long>();
    a.l21 = F.l21.as<double>();
    a.linv = F.linv.as<double>();
    a.in = jobs[q].in;
    a.y = jobs[q].y;
    a.scratch = jobs[q].scratch;
    a.sstride = F.scratch_entries();
    a.nrhs = (q == 1 && jobs[1].nrhs > 0) ? std::min(jobs[1].nrhs, nrhs) : nrhs;
  }
  // the y part of a slice starts after the largest front of the launch
  for (int q = 0; q < njobs; ++q) args.a[q].y_off = slice - jobs[q].F->max_ncol;
  const size_t lds = (size_t)(W + (size_t)W * slice) * sizeof(double2);
  ProfScope prof(tag, s);
  hipLaunchKernelGGL(k_spsolve, dim3((unsigned)nrhs, (unsigned)njobs), dim3(64 * W), lds, s, args);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

void spchol_arrays(const SpFactor& F, SpArrays& a) {
  const int n = F.n, nsn = F.nsn;
  // levels by height
  int H = 0;
  for (int q = 0; q < nsn; ++q) H = std::max(H, F.height[q]);
  a.nlev = H + 1;
  a.lvl_off.assign(H + 2, 0);
  a.lvl_node.assign(nsn, 0);
  for (int q = 0; q < nsn; ++q) a.lvl_off[F.height[q] + 1]++;
  for (int h = 0; h <= H; ++h) a.lvl_off[h + 1] += a.lvl_off[h];
  {
    std::vector<int> fill(a.lvl_off.begin(), a.lvl_off.end() - 1);
    for (int q = 0; q < nsn; ++q) a.lvl_node[fill[F.height[q]]++] = q;
  }
  // L_21 blocks and inverses of the diagonal blocks
  a.l21_off.assign(nsn + 1, 0);
  a.linv_off.assign(nsn + 1, 0);
  a.max_ncol = 0;
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    a.l21_off[q + 1] = a.l21_off[q] + (long)nstr * ncol;
    a.linv_off[q + 1] = a.linv_off[q] + (long)ncol * ncol;
    a.max_ncol = std::max(a.max_ncol, ncol);
  }
  a.l21.assign(a.l21_off[nsn], 0.0);
  a.linv.assign(a.linv_off[nsn], 0.0);
  for (int q = 0; q < nsn; ++q) {
    const int ncol = F.col0[q + 1] - F.col0[q], nstr = F.str_off[q + 1] - F.str_off[q];
    const int m = ncol + nstr;
    const double* P = &F.panel[F.panel_off[q]];
    for (int j = 0; j < ncol; ++j)
      for (int t = 0; t < nstr; ++t) a.l21[a.l21_off[q] + (long)j * nstr + t] = P[(size_t)j * m + ncol + t];
    // Z = L_ss^-1 column by column, by forward substitution on e_c
    double* Z = &a.linv[a.linv_off[q]];
    for (int c = 0; c < ncol; ++c)
      for (int i = c; i < ncol; ++i) {
        double acc = i == c ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) acc -= P[(size_t)k * m + i] * Z[(size_t)c * ncol + k];
        Z[(size_t)c * ncol + i] = acc / P[(size_t)i * m + i];
      }
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
  D.nnz = a.l21_off[nsn] + a.linv_off[nsn];
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> rfcmp_status {
    RF_TRY(b.alloc(std::max<size_t>(bytes, 16)));
    if (bytes) RF_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return RFCMP_OK;
  };
  RF_TRY(up(D.perm, F.perm.data(), sizeof(int) * n));
  RF_TRY(up(D.iperm, a.iperm.data(), sizeof(int) * n));
  RF_TRY(up(D.col0, F.col0.data(), sizeof(int) * (nsn + 1)));
  RF_TRY(up(D.str_off, F.str_off.data(), sizeof(int) * (nsn + 1)));
  RF_TRY(up(D.str, F.str.data(), sizeof(int) * F.str.size()));
  RF_TRY(up(D.map, F.map.data(), sizeof(int) * F.map.size()));
  RF_TRY(up(D.child_off, F.child_off.data(), sizeof(int) * (nsn + 1)));
  RF_TRY(up(D.child_idx, F.child_idx.data(), sizeof(int) * F.child_idx.size()));
  RF_TRY(up(D.lvl_off, a.lvl_off.data(), sizeof(int) * a.lvl_off.size()));
  RF_TRY(up(D.lvl_node, a.lvl_node.data(), sizeof(int) * nsn));
  RF_TRY(up(D.l21_off, a.l21_off.data(), sizeof(long) * (nsn + 1)));
  RF_TRY(up(D.linv_off, a.linv_off.data(), sizeof(long) * (nsn + 1)));
  RF_TRY(up(D.l21, a.l21.data(), sizeof(double) * a.l21.size()));
  RF_TRY(up(D.linv, a.linv.data(), sizeof(double) * a.linv.size()));
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
