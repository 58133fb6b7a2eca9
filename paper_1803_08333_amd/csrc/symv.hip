// Symmetric streaming matrix-vector products.
//
// Every dense matrix the operator applies is symmetric: T_A and V are
// complex-symmetric Galerkin blocks (T_A = T_A^T, V = V^T), and L^+, G_ll^-1
// and G_tp^-1 are real symmetric.  The products are HBM-bound (about one flop
// per byte), so reading each off-diagonal entry once and using it for two
// outputs halves the time:  with the matrix cut into S x S blocks,
//   block (P, Q), P < Q:  y_P += M_PQ x_Q   and   y_Q += M_PQ^T x_P,
//   block (P, P):         y_P += M_PP x_P   (read whole),
// only blocks with Q >= P are read.  Each workgroup owns one block and writes
// its two partial outputs to a slot of a partial buffer, part[K][L] = the
// contribution to output block K from the block pairing K with L; a second
// kernel sums the slots of each output block in a fixed order.  The result
// is deterministic (no atomics) and the matrix is read from its upper block
// triangle only.
//
// A block is streamed in sub-tiles of 32 rows x S columns: each thread loads
// 16-byte column pairs of several rows into registers (coalesced: a wave
// reads a whole row), accumulates the transposed product M^T x_P for its
// column pair straight from registers, and stores the sub-tile to LDS, from
// where eight threads per row form the row sums M x_Q (thread s of a row
// takes pairs s, s + 8, ..., so a row's threads read adjacent LDS words; the
// eight partial sums meet through DPP lane moves).
// Two sub-tiles are in flight per workgroup: the loads of sub-tile t + 2 are
// issued as soon as sub-tile t sits in LDS.  Products are formed
// and accumulated in FP64 (complex64 entries are widened), x and y are
// complex128.
//
// The input x is formed while it is staged (SymvInput): a plain vector, or a
// sparse incidence product (Sigma^T, Lambda^T) or fused operator line of
// vectors already in HBM.  Each workgroup forms only the 2 x 128 entries it
// needs, reading a few source entries per entry from L2.  One launch can
// carry two products of the same element type (their blocks side by side in
// the grid), so a small matrix rides along with a large one.
#include "symv.h"
#include "symv_input.h"

namespace rfcmp {

namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
// rows per sub-tile for block size S: the sub-tile is 4 KB of pairs per 256 threads
template <int S>
constexpr int rows_sub() { return S == 128 ? 32 : 16; }
// Pairs per LDS tile row: a 16-lane pass of the row sums covers 256 / S rows
// (two at S = 128), so rows are padded to start 128 bytes apart in the banks.
template <int S>
constexpr int tile_ld() { return S / 2 + 8; }
constexpr int kMaxNR = 4;      // right-hand sides per pass

// Entry e (0, 1) of a 16-byte column pair, widened to FP64 (re, im).
struct C64 {
  typedef vf4 Pair;
  __device__ static inline Pair first_only(Pair v) {
    v.z = 0.0f;
    v.w = 0.0f;
    return v;
  }
  template <bool CONJ>
  __device__ static inline void entry(const Pair& v, int e, double& re, double& im) {
    re = e ? (double)v.z : (double)v.x;
    const double t = e ? (double)v.w : (double)v.y;
    im = CONJ ? -t : t;
  }
};
struct F64 {
  typedef vd2 Pair;
  __device__ static inline Pair first_only(Pair v) {
    v.y = 0.0;
    return v;
  }
  template <bool CONJ>
  __device__ static inline void entry(const Pair& v, int e, double& re, double& im) {
    re = e ? v.y : v.x;
    im = 0.0;
  }
};

template <class T>
__device__ inline typename T::Pair zero_pair() {
  typename T::Pair z;
  z = 0;
  return z;
}

__global__ void k_form_input(const SymvInput in, int n, double2* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (g < n) out[(long)r * n + g] = input_entry(in, r, g);
}

// Kernel arguments: up to two products; blocks [0, nblk0) belong to job 0.
struct JobArg {
  const void* M;
  int n;
  long ldp;  // row length in 16-byte pairs
  int nsb;
  SymvInput in;
  double2* part;
  double2* y;
};
struct JobsArg {
  JobArg j[2];
  int nblk0;
  int nsb0;
};

// DPP move of a double: lane i takes the value of the lane CTRL selects
// (quad_perm or row shift); lanes without a source get 0.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over each aligned group of TPR (8 or 16) lanes; lanes TPR - 4 .. TPR - 1
// of a group hold it.
template <int TPR>
__device__ inline double sum_lanes(double v) {
  static_assert(TPR == 8 || TPR == 16, "group size");
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_move<0x114>(v);  // row_shr:4: lanes 4..7 (of 8) add lanes 0..3
  if (TPR == 16) v += dpp_move<0x118>(v);  // row_shr:8: lanes 12..15 add lanes 4..7
  return v;
}

// One block (P, Q) of a product.  EDGE: the block reaches past n, so loads
// are masked (rows beyond n are not read, columns beyond n read as zero).
// The block's rows start at the uniform address `strip`; each thread
// addresses its 16-byte pairs by 32-bit offsets from it.
template <class T, int S, int NR, bool CONJ, bool EDGE>
__device__ void symv_block(const char* __restrict__ strip, int n, int ldp, int P, int Q,
                           const SymvInput& in, double2* __restrict__ part, int nsb,
                           typename T::Pair (*tile)[tile_ld<S>()], double2 (*xs)[NR][S]) {
  typedef typename T::Pair Pair;
  constexpr int kRowsSub = rows_sub<S>();
  constexpr int PP = S / 2;                       // column pairs per row
  constexpr int G = kThreads / PP;                // row groups in the load layout
  constexpr int LPT = kRowsSub / G;               // loads per thread per sub-tile
  constexpr int NSUB = S / kRowsSub;              // sub-tiles per block
  constexpr int TPR = kThreads / kRowsSub;        // threads per row in the row sums
  constexpr int PPT = PP / TPR;                   // pairs per thread in the row sums
  static_assert(kRowsSub % G == 0 && PP % TPR == 0 && NSUB % 2 == 0, "block shape");
  const bool diag = (P == Q);
  const int tid = threadIdx.x;

  // load layout: column pair p, rows g0 + G q of each sub-tile
  const int p = tid % PP, g0 = tid / PP;
  const int gc = Q * S + 2 * p;  // first global column of the pair
  const bool c0 = gc < n, c1 = gc + 1 < n;
  const unsigned off0 = ((unsigned)g0 * (unsigned)ldp + (unsigned)(gc >> 1)) * 16u;
  const unsigned rowstep = (unsigned)G * (unsigned)ldp * 16u;
  const unsigned substep = (unsigned)kRowsSub * (unsigned)ldp * 16u;
  Pair ra[LPT], rb[LPT];  // two sub-tiles in flight

#define SYMV_LOAD(REG, SUB)                                                                        \
  _Pragma("unroll") for (int q = 0; q < LPT; ++q) {                                                \
    const Pair* a = reinterpret_cast<const Pair*>(strip + off0 + (SUB) * substep + q * rowstep);   \
    if (EDGE) {                                                                                    \
      const int gr = P * S + (SUB) * kRowsSub + g0 + G * q;                                        \
      Pair v = zero_pair<T>();                                                                     \
      if (gr < n && c0) v = __builtin_nontemporal_load(a);                                         \
      REG[q] = c1 ? v : T::first_only(v);                                                          \
    } else {                                                                                       \
      REG[q] = __builtin_nontemporal_load(a);                                                      \
    }                                                                                              \
  }
  SYMV_LOAD(ra, 0)
  SYMV_LOAD(rb, 1)
  for (int t = tid; t < 2 * NR * S; t += kThreads) {
    const int side = t / (NR * S), r = (t / S) % NR, i = t % S;
    const int g = (side == 0 ? P : Q) * S + i;
    // x_Q is stored even columns first, then odd ones, so that the row sums
    // (neighbouring threads, neighbouring pairs) read it without bank conflicts
    const int slot = side ? (i & 1) * (S / 2) + (i >> 1) : i;
    xs[side][r][slot] = (!EDGE || g < n) ? input_entry(in, r, g) : make_double2(0.0, 0.0);
  }

  double cr[2][NR], ci[2][NR];  // transposed sums of the two columns
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int r = 0; r < NR; ++r) cr[e][r] = ci[e][r] = 0.0;
  const int rrow = tid / TPR, seg = tid % TPR;  // row-sum layout
  __syncthreads();  // xs ready

#define SYMV_CONSUME(REG, SUB)                                                                     \
  {                                                                                                \
    if (!diag) {                                                                                   \
      _Pragma("unroll") for (int q = 0; q < LPT; ++q) {                                            \
        const int lr = (SUB) * kRowsSub + g0 + G * q;                                              \
        _Pragma("unroll") for (int e = 0; e < 2; ++e) {                                            \
          double ar, ai;                                                                           \
          T::template entry<CONJ>(REG[q], e, ar, ai);                                              \
          _Pragma("unroll") for (int r = 0; r < NR; ++r) {                                         \
            const double2 xv = xs[0][r][lr];                                                       \
            cr[e][r] = fma(ar, xv.x, fma(-ai, xv.y, cr[e][r]));                                    \
            ci[e][r] = fma(ar, xv.y, fma(ai, xv.x, ci[e][r]));                                     \
          }                                                                                        \
        }                                                                                          \
      }                                                                                            \
    }                                                                                              \
    __syncthreads(); /* the previous row sums are done with the tile */                            \
    _Pragma("unroll") for (int q = 0; q < LPT; ++q) tile[g0 + G * q][p] = REG[q];                  \
    if ((SUB) + 2 < NSUB) { SYMV_LOAD(REG, (SUB) + 2) }                                            \
    __syncthreads();                                                                               \
    double rr[NR], ri[NR];                                                                         \
    _Pragma("unroll") for (int r = 0; r < NR; ++r) rr[r] = ri[r] = 0.0;                            \
    _Pragma("unroll") for (int u = 0; u < PPT; ++u) {                                              \
      const int pc = seg + TPR * u; /* neighbouring threads read neighbouring pairs */             \
      const Pair v = tile[rrow][pc];                                                               \
      _Pragma("unroll") for (int e = 0; e < 2; ++e) {                                              \
        double ar, ai;                                                                             \
        T::template entry<CONJ>(v, e, ar, ai);                                                     \
        _Pragma("unroll") for (int r = 0; r < NR; ++r) {                                           \
          const double2 xv = xs[1][r][e * (S / 2) + pc];                                           \
          rr[r] = fma(ar, xv.x, fma(-ai, xv.y, rr[r]));                                            \
          ri[r] = fma(ar, xv.y, fma(ai, xv.x, ri[r]));                                             \
        }                                                                                          \
      }                                                                                            \
    }                                                                                              \
    _Pragma("unroll") for (int r = 0; r < NR; ++r) {                                               \
      rr[r] = sum_lanes<TPR>(rr[r]);                                                               \
      ri[r] = sum_lanes<TPR>(ri[r]);                                                               \
    }                                                                                              \
    if (seg == TPR - 4) {                                                                          \
      const int i = (SUB) * kRowsSub + rrow;                                                       \
      _Pragma("unroll") for (int r = 0; r < NR; ++r)                                               \
        part[(((long)P * nsb + Q) * NR + r) * S + i] = make_double2(rr[r], ri[r]);                 \
    }                                                                                              \
  }
#pragma unroll 1
  for (int sub = 0; sub < NSUB; sub += 2) {
    SYMV_CONSUME(ra, sub)
    SYMV_CONSUME(rb, sub + 1)
  }
#undef SYMV_CONSUME
#undef SYMV_LOAD

  if (!diag) {
    // reduce the transposed sums over the G row groups through LDS
    __syncthreads();
    double2* red = reinterpret_cast<double2*>(&tile[0][0]);  // [G][S][NR]
    static_assert(sizeof(double2) * G * S * NR <= sizeof(Pair) * kRowsSub * tile_ld<S>(), "reduction fits the tile");
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int r = 0; r < NR; ++r) red[(g0 * S + 2 * p + e) * NR + r] = make_double2(cr[e][r], ci[e][r]);
    __syncthreads();
    for (int t = tid; t < S * NR; t += kThreads) {
      const int c = t % S, r = t / S;
      double sr = 0.0, si = 0.0;
      for (int g = 0; g < G; ++g) {
        const double2 v = red[(g * S + c) * NR + r];
        sr += v.x;
        si += v.y;
      }
      part[(((long)Q * nsb + P) * NR + r) * S + c] = make_double2(sr, si);
    }
  }
}

// Partial buffer layout: part[((K * nsb + L) * NR + r) * S + i], complex128.
// Job 0 has NR0 right-hand sides, job 1 NR1.
template <class T, int S, int NR0, int NR1, bool CONJ>
__global__ __launch_bounds__(kThreads) void k_symv(const JobsArg args) {
  typedef typename T::Pair Pair;
  constexpr int NRM = NR0 > NR1 ? NR0 : NR1;
  const int job = (int)blockIdx.x < args.nblk0 ? 0 : 1;
  const JobArg& ja = args.j[job];
  const int n = ja.n, nsb = ja.nsb;

  // block (P, Q), Q >= P, from the linear upper-triangle index
  int P = 0, rem = (int)blockIdx.x - (job ? args.nblk0 : 0);
  while (rem >= nsb - P) {
    rem -= nsb - P;
    ++P;
  }
  const int Q = P + rem;
  __shared__ Pair tile[rows_sub<S>()][tile_ld<S>()];
  __shared__ double2 xs[2][NRM][S];  // x_P (rows), x_Q (columns)
  const char* strip = static_cast<const char*>(ja.M) + (size_t)P * S * (size_t)ja.ldp * 16;
  const bool edge = (Q + 1) * S > n;  // else (P + 1) S <= n as well
  if (job == 0 || NR0 == NR1) {
    auto x0 = reinterpret_cast<double2(*)[NR0][S]>(&xs[0][0][0]);
    if (!edge)
      symv_block<T, S, NR0, CONJ, false>(strip, n, (int)ja.ldp, P, Q, ja.in, ja.part, nsb, tile, x0);
    else
      symv_block<T, S, NR0, CONJ, true>(strip, n, (int)ja.ldp, P, Q, ja.in, ja.part, nsb, tile, x0);
  } else {
    auto x1 = reinterpret_cast<double2(*)[NR1][S]>(&xs[0][0][0]);
    if (!edge)
      symv_block<T, S, NR1, CONJ, false>(strip, n, (int)ja.ldp, P, Q, ja.in, ja.part, nsb, tile, x1);
    else
      symv_block<T, S, NR1, CONJ, true>(strip, n, (int)ja.ldp, P, Q, ja.in, ja.part, nsb, tile, x1);
  }
}

// y[r][K S + i] = sum over L (in order) of part[K][L][r][i].  Workgroup
// (K, r): eight threads per row each add an eighth of the slots (all loads
// issued before the adds, so they overlap), then the eighths are added in
// order through LDS.  Blocks [0, nsb0) of the grid reduce job 0, the rest
// job 1.
template <int S>
constexpr int red_parts() { return 1024 / S; }
template <int S, int NR0, int NR1>
__global__ __launch_bounds__(1024) void k_symv_reduce(const JobsArg args) {
  constexpr int kRedParts = red_parts<S>();
  __shared__ double2 q8[kRedParts][S];
  const int job = (int)blockIdx.x < args.nsb0 ? 0 : 1;
  const JobArg& ja = args.j[job];
  const int n = ja.n, nsb = ja.nsb;
  const int NR = job ? NR1 : NR0;
  const int K = (int)blockIdx.x - (job ? args.nsb0 : 0), r = blockIdx.y;
  if (r >= NR) return;
  const int i = threadIdx.x % S, qt = threadIdx.x / S;
  const int per = (nsb + kRedParts - 1) / kRedParts;
  const int L0 = qt * per;
  const double2* src = ja.part + (((long)K * nsb) * NR + r) * S + i;
  double sr = 0.0, si = 0.0;
  for (int b0 = 0; b0 < per; b0 += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int L = L0 + b0 + u;
      v[u] = (b0 + u < per && L < nsb) ? src[(long)L * NR * S] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sr += v[u].x;
      si += v[u].y;
    }
  }
  q8[qt][i] = make_double2(sr, si);
  __syncthreads();
  const int row = K * S + i;
  if (qt == 0 && row < n) {
    double2 t = q8[0][i];
    for (int u = 1; u < kRedParts; ++u) {
      t.x += q8[u][i].x;
      t.y += q8[u][i].y;
    }
    ja.y[(long)r * n + row] = t;
  }
}

constexpr int kSmax = 256, kSmin = 128;

// The product kernel is timed under `tag` (one right-hand side) or
// "<tag>_nr<k>" (k right-hand sides), the slot sums under "symv_reduce".
template <class T, int S, int NR0, int NR1, bool CONJ>
void launch(const JobsArg& a, int nblk, int nsbsum, hipStream_t s, const char* tag) {
  {
    ProfScope prof(NR0 == 1 ? tag : profile_tag_suffix(tag, NR0), s);
    hipLaunchKernelGGL((k_symv<T, S, NR0, NR1, CONJ>), dim3((unsigned)nblk), dim3(kThreads), 0, s, a);
  }
  ProfScope prof("symv_reduce", s);
  constexpr int NRM = NR0 > NR1 ? NR0 : NR1;
  hipLaunchKernelGGL((k_symv_reduce<S, NR0, NR1>), dim3((unsigned)nsbsum, NRM), dim3(1024), 0, s, a);
}

// Block size: 256 x 256 blocks (longer streams per workgroup, fewer slots)
// once they still give the grid a few hundred workgroups, else 128 x 128.
constexpr int kMinBlocks256 = 400;

// Advance every source pointer of an input by r0 right-hand sides.
SymvInput shift_input(SymvInput in, int r0) {
  for (int q = 0; q < 4; ++q)
    if (in.p[q]) in.p[q] += (long)r0 * in.stride[q];
  return in;
}

template <class T, bool CONJ>
rfcmp_status symv_any(const SymvJob* jobs, int njobs, int nrhs, void* scratch, size_t scratch_bytes,
                      hipStream_t s, const char* tag) {
  if (njobs < 1 || njobs > 2) {
    set_error("symv: %d jobs (1 or 2 allowed)", njobs);
    return RFCMP_E_ARG;
  }
  if (nrhs <= 0) return RFCMP_OK;
  // right-hand sides of each job: nrhs, or fewer for job 1 (a product riding
  // along with fewer columns; then nrhs <= kMaxNR)
  int jn[2] = {nrhs, nrhs};
  if (njobs == 2 && jobs[1].nrhs > 0 && jobs[1].nrhs < nrhs) {
    if (nrhs > kMaxNR || !(nrhs == 2 && jobs[1].nrhs == 1)) {
      set_error("symv: job 1 with %d of %d right-hand sides is not supported", jobs[1].nrhs, nrhs);
      return RFCMP_E_ARG;
    }
    jn[1] = jobs[1].nrhs;
  }
  size_t need = 0;
  for (int q = 0; q < njobs; ++q) {
    if (jobs[q].n <= 0 || jobs[q].ld % 2 != 0 || jobs[q].ld < jobs[q].n) {
      set_error("symv: job %d has n = %lld, ld = %lld", q, (long long)jobs[q].n, (long long)jobs[q].ld);
      return RFCMP_E_ARG;
    }
    need += symv_scratch_bytes(jobs[q].n, std::min(jn[q], kMaxNR));
  }
  if (need > scratch_bytes) {
    set_error("symv: needs %zu bytes of scratch, %zu given", need, scratch_bytes);
    return RFCMP_E_ARG;
  }
  long blocks_big = 0;
  for (int q = 0; q < njobs; ++q) {
    const long nb = (jobs[q].n + kSmax - 1) / kSmax;
    blocks_big += nb * (nb + 1) / 2;
  }
  const int S = blocks_big >= kMinBlocks256 ? kSmax : kSmin;
  for (int r0 = 0; r0 < nrhs; r0 += kMaxNR) {
    const int nr = std::min(kMaxNR, nrhs - r0);
    const bool split = jn[1] != nrhs;  // job 1: one column (nr == 2 here)
    JobsArg a{};
    char* sp = static_cast<char*>(scratch);
    int nblk = 0, nsbsum = 0;
    for (int q = 0; q < njobs; ++q) {
      const SymvJob& jb = jobs[q];
      JobArg& ja = a.j[q];
      ja.M = jb.M;
      ja.n = (int)jb.n;
      ja.ldp = (long)(jb.ld / 2);
      ja.nsb = int((jb.n + S - 1) / S);
      ja.in = shift_input(jb.in, r0);
      ja.part = reinterpret_cast<double2*>(sp);
      ja.y = jb.y + (long)r0 * jb.n;
      sp += symv_scratch_bytes(jb.n, q == 1 && split ? 1 : nr);
      if (q == 0) {
        a.nblk0 = ja.nsb * (ja.nsb + 1) / 2;
        a.nsb0 = ja.nsb;
      }
      nblk += ja.nsb * (ja.nsb + 1) / 2;
      nsbsum += ja.nsb;
    }
#define RF_SYMV_NR(SV)                                                          \
  if (split) {                                                                  \
    launch<T, SV, 2, 1, CONJ>(a, nblk, nsbsum, s, tag);                         \
  } else {                                                                      \
    switch (nr) {                                                               \
      case 1: launch<T, SV, 1, 1, CONJ>(a, nblk, nsbsum, s, tag); break;        \
      case 2: launch<T, SV, 2, 2, CONJ>(a, nblk, nsbsum, s, tag); break;        \
      case 3: launch<T, SV, 3, 3, CONJ>(a, nblk, nsbsum, s, tag); break;        \
      default: launch<T, SV, 4, 4, CONJ>(a, nblk, nsbsum, s, tag); break;       \
    }                                                                           \
  }
    if (S == kSmax) {
      RF_SYMV_NR(kSmax)
    } else {
      RF_SYMV_NR(kSmin)
    }
#undef RF_SYMV_NR
  }
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

}  // namespace

size_t symv_scratch_bytes(int64_t n, int nrhs) {
  // the smaller block size needs the most slots
  const int64_t nsb = (n + kSmin - 1) / kSmin;
  const int nr = std::min(std::max(nrhs, 1), kMaxNR);
  return sizeof(double2) * (size_t)(nsb * nsb * nr * kSmin);
}

rfcmp_status symv_form_input(const SymvInput& in, int64_t n, int nrhs, double2* out, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return RFCMP_OK;
  hipLaunchKernelGGL(k_form_input, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, in, (int)n, out);
  RF_HIP(hipGetLastError());
  return RFCMP_OK;
}

rfcmp_status csymv_jobs(const SymvJob* jobs, int njobs, bool conj, int nrhs, void* scratch, size_t scratch_bytes,
                        hipStream_t s, const char* tag) {
  if (conj) return symv_any<C64, true>(jobs, njobs, nrhs, scratch, scratch_bytes, s, tag);
  return symv_any<C64, false>(jobs, njobs, nrhs, scratch, scratch_bytes, s, tag);
}

rfcmp_status dsymv_jobs(const SymvJob* jobs, int njobs, int nrhs, void* scratch, size_t scratch_bytes,
                        hipStream_t s, const char* tag) {
  return symv_any<F64, false>(jobs, njobs, nrhs, scratch, scratch_bytes, s, tag);
}

rfcmp_status csymv(const float2* M, int64_t n, int64_t ld, bool conj, const double2* x, double2* y, int nrhs,
                   void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag) {
  SymvJob j;
  j.M = M;
  j.n = n;
  j.ld = ld;
  j.in.p[0] = x;
  j.in.stride[0] = n;
  j.y = y;
  return csymv_jobs(&j, 1, conj, nrhs, scratch, scratch_bytes, s, tag);
}

rfcmp_status dsymv(const double* M, int64_t n, int64_t ld, const double2* x, double2* y, int nrhs,
                   void* scratch, size_t scratch_bytes, hipStream_t s, const char* tag) {
  SymvJob j;
  j.M = M;
  j.n = n;
  j.ld = ld;
  j.in.p[0] = x;
  j.in.stride[0] = n;
  j.y = y;
  return dsymv_jobs(&j, 1, nrhs, scratch, scratch_bytes, s, tag);
}

}  // namespace rfcmp
