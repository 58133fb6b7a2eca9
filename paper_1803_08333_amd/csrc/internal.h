// Internal declarations of the rfcmp library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <future>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rfcmp.h"

namespace rfcmp {

void set_error(const char* fmt, ...);
void clear_error();
const char* last_error();  // of the calling thread

#define RF_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::rfcmp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                    \
      return e_ == hipErrorOutOfMemory ? RFCMP_E_OOM : RFCMP_E_HIP;                    \
    }                                                                                  \
  } while (0)

#define RF_TRY(expr)                       \
  do {                                     \
    rfcmp_status s_ = (expr);              \
    if (s_ < 0) return s_;                 \
  } while (0)

// Where a device block came from: the caller's allocator (rfcmp_set_allocator;
// free_fn non-null) or the library's own cache over hipMalloc (free_fn null).
// Each block is returned to the allocator that made it, even if another one
// has been registered since.
struct AllocOrigin {
  rfcmp_free_fn free_fn = nullptr;
  void* ctx = nullptr;
};

// Device memory (devmem.cpp): dev_alloc returns a block of at least n bytes on
// the current device (its size in *got, its device in *device, its origin in
// *origin) or nullptr; dev_free returns a block after the device is idle.
void* dev_alloc(size_t n, size_t* got, int* device, AllocOrigin* origin);
void dev_free(void* p, size_t bytes, int device, const AllocOrigin& origin);
size_t dev_cache_release();
size_t dev_cache_bytes();

// Owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;     // bytes requested
  size_t capacity = 0;  // bytes of the block
  int device = -1;
  AllocOrigin origin;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) dev_free(p, capacity, device, origin);
    p = nullptr;
    bytes = capacity = 0;
    device = -1;
    origin = AllocOrigin{};
  }
  rfcmp_status alloc(size_t n) {
    release();
    if (n == 0) return RFCMP_OK;
    p = dev_alloc(n, &capacity, &device, &origin);
    if (!p) {
      set_error("device allocation of %zu bytes failed", n);
      return RFCMP_E_OOM;
    }
    bytes = n;
    return RFCMP_OK;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

inline size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Optional kernel timing for benchmarks: when enabled, a start/stop HIP event
// pair is recorded on the launch stream around each tagged launch.
bool profiling_enabled();
bool profiling_selected(const char* tag);
// "<tag>_nr<k>", interned (valid for the life of the process).
const char* profile_tag_suffix(const char* tag, int k);
void profile_record(const char* tag, hipEvent_t start, hipEvent_t stop);
hipEvent_t profile_event();
struct ProfScope {
  const char* tag;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* t, hipStream_t st) : tag(t), s(st) {
    if (profiling_enabled() && profiling_selected(t)) {
      a = profile_event();
      b = profile_event();
      if (a && b) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      profile_record(tag, a, b);
    }
  }
};

// Host-side topology and geometry (FP64), built by rfcmp_mesh_create.
struct MeshHost {
  int64_t V = 0, C = 0, N = 0;
  int32_t genus = 0;
  std::vector<double> xyz;            // [V][3]
  std::vector<int32_t> tri;           // [C][3]
  std::vector<int32_t> edge_vtx;      // [N][2] (min, max)
  std::vector<int32_t> edge_cell;     // [N][2] (c+, c-)
  std::vector<int32_t> edge_local;    // [N][2] local index in c+, c-
  std::vector<int32_t> cell_edge;     // [C][3] edge of local edge i
  std::vector<int8_t> cell_sign;      // [C][3] Sigma[edge, cell]
  std::vector<double> area;           // [C]
  std::vector<double> centroid;       // [C][3]
  std::vector<double> hmax;           // [C] longest edge of each cell
  std::vector<int32_t> noc;           // [V] cells at each vertex
  std::vector<int32_t> vtx_edge_ptr;  // [V+1] CSR: edges at each vertex
  std::vector<int32_t> vtx_edge_idx;  // [2N]
  std::vector<int8_t> vtx_edge_sgn;   // [2N] Lambda[edge, vertex]
  std::vector<int32_t> cell_nb_ptr;   // [C+1] CSR: cells sharing a vertex (incl. self); build_cell_nb
  std::vector<int32_t> cell_nb_idx;
};

struct SplitMatrix;  // BF16x3 planes of a matrix (gemm.h)
struct HmMesh;       // cluster tree of the compressed blocks (hmat.h)
struct HmOp;         // compressed blocks of an operator (hmat.h)
struct SpFactor;     // sparse Cholesky factor, host (spchol.h)
struct SpDevice;     // sparse Cholesky factor, device (spchol.h)

// The near pairs of one factor (c <= c', self pairs included) and what the
// T_A assembly looks them up with (assemble.hip): the near partners of each
// cell, ascending (ptr/other), with code 2 p + t for pair p (t = 1: the
// pair is stored with the partner first), and per pair of edge tiles
// (I <= J, index J (J + 1)/2 + I) whether any of its cell pairs is near.
struct NearData {
  std::vector<int32_t> pairs, ptr, other, code;
  std::vector<uint8_t> tile_near;
};

// A sparse factor computed on a host thread.
struct HostFactor {
  rfcmp_status status = RFCMP_OK;
  std::string error;
  std::shared_ptr<SpFactor> F;
};

// Device copies and the dense FP64 projector matrices of one mesh.
struct MeshDev {
  bool uploaded = false;     // mesh arrays on the device
  bool ready = false;        // dense projector inverses built
  bool has_gtp = false;
  // sparse projector factors on the device: L (grounded), G_ll, G_tp
  std::unique_ptr<SpDevice> sp[3];
  int64_t ldL = 0, ldG = 0, ldT = 0;  // padded leading dims of L^+, G_ll^-1, G_tp^-1
  DevBuf cen;        // double [C][3]
  DevBuf vtx;        // double [C][9]  cell vertices
  DevBuf area;       // double [C]
  DevBuf qoff;       // float4 [C][7]  quadrature points minus centroid
  DevBuf fvoff;      // float4 [C][3]  vertex i minus centroid
  DevBuf sgn;        // float  [C][3]
  DevBuf cell_edge;  // int [C][3]
  DevBuf edge_cell;  // int [N][2]
  DevBuf edge_slot;  // int [N][2]  3*c+ + l+, 3*c- + l-
  DevBuf edge_vtx;   // int [N][2]
  DevBuf ve_ptr, ve_idx, ve_sgn;  // Lambda^T CSR
  DevBuf Lp;         // double [ldL][ldL]: (Sigma^T Sigma)^+
  DevBuf Gll_inv;    // double [ldG][ldG]
  DevBuf Gtp_inv;    // double [ldT][ldT]
  std::unique_ptr<SplitMatrix> Lp16, Gll16, Gtp16;  // BF16x3 planes, built on demand
  // assembly edge tiles (kEdgeTile consecutive edges each) and the cells
  // each tile touches: et_cell[et_ptr[t] ..] ascending, et_rows the rows in
  // the tile of each such cell's three local edges (8 bits each, 0xFF: not in
  // the tile), cell_home the tile of each cell's local edge 0
  int64_t etiles = 0;
  int et_cells_max = 0;
  DevBuf et_ptr, et_cell, et_rows, cell_home;
  double near_factor = -1.0;  // factor of the cached near-pair list
  int64_t npairs = 0;
  DevBuf near;       // int [npairs][2]
  DevBuf nearB;      // complex64 [npairs][3][3] near-pair blocks
  DevBuf np_ptr, np_other, np_code, tile_near;  // NearData on the device
  NearData near_host;  // host copy
  // The projector matrices are built on two internal streams (L^+ on the
  // first, G_ll^-1 and G_tp^-1 on the second), each with its own FP64 panel
  // buffers for the inverse.  A stream that uses them first waits for
  // proj_done (wait_projectors).
  DevBuf gj_u[2], gj_r[2];
  DevBuf scat_ij, scat_v;  // coordinate list of G_tp (second stream)
  hipStream_t proj_stream[2] = {nullptr, nullptr};  // non-blocking, default priority
  hipEvent_t proj_start = nullptr, proj_done[2] = {nullptr, nullptr};
  bool proj_pending = false;
  MeshDev();
  ~MeshDev();
};

}  // namespace rfcmp

struct rfcmp_mesh_s {
  rfcmp::MeshHost h;
  rfcmp::MeshDev d;
  int device = -1;
  // near-pair list for near_async_factor, computed on a host thread from
  // mesh creation on (declared last: its destructor waits for the thread
  // before h goes)
  double near_async_factor = -1.0;
  std::future<rfcmp::NearData> near_async;
  // sparse factors of L and G_ll, computed on host threads from mesh
  // creation on (declared after h: their destructors wait for the threads)
  std::future<rfcmp::HostFactor> fac_async[2];
  // cluster tree of the compressed blocks, built with the first compressed
  // operator (destroyed where hmat.h is complete: rfcmp_mesh_destroy)
  std::unique_ptr<rfcmp::HmMesh> hm;
  rfcmp_mesh_s();
  ~rfcmp_mesh_s();
};

namespace rfcmp {
// T_A and V are stored whole (both triangles, exactly symmetric).  The
// symmetric streaming products read the upper triangle of kTriBlock x
// kTriBlock blocks (row m, columns n >= kTriBlock floor(m / kTriBlock)); the
// FP64 multi-right-hand-side products read every entry.
constexpr int kTriBlock = 256;
// Edges per tile of the T_A assembly (a divisor of kTriBlock).
constexpr int kEdgeTile = 64;
static_assert(kTriBlock % kEdgeTile == 0, "edge tiles nest in the stored blocks");
}  // namespace rfcmp

struct rfcmp_op_s {
  rfcmp_op_s();
  ~rfcmp_op_s();
  rfcmp_mesh mesh = nullptr;
  double k = 0;
  int power_steps = 0;  // power-iteration steps run (0 for k-scaling)
  rfcmp_options opt{};
  double alpha = 0, beta = 0, gamma = 0;
  double lam[3] = {0, 0, 0};
  int64_t ldA = 0, ldV = 0;  // leading dims (complex entries) of T_A and V
  rfcmp::DevBuf TA;          // float2 [N][ldA], block upper triangle (kTriBlock)
  rfcmp::DevBuf Vb;          // float2 [C][ldV]
  rfcmp::DevBuf work;        // complex128 workspace for work_nrhs right-hand sides
  int work_nrhs = 0;
  double* host_scal = nullptr;      // pinned and mapped, 16 + 8 * work_nrhs doubles
  double* host_scal_dev = nullptr;  // its device address
  std::unique_ptr<rfcmp::SplitMatrix> TA16, V16;  // BF16x3 planes (precision 1)
  rfcmp::DevBuf gemm_scratch;
  rfcmp::DevBuf z_scratch;     // slice partials of the FP64 multi-RHS products
  rfcmp::DevBuf symv_scratch;  // partial sums of the symmetric products
  // CG iterations replayed as HIP graphs (one per parity of the iteration:
  // the recurrence scalars alternate between two buffers), run on an
  // internal stream; key: the kernel arguments they were captured with
  hipStream_t cg_stream = nullptr;
  hipGraphExec_t cg_exec[2] = {nullptr, nullptr};
  uint64_t cg_key[2] = {0, 0};
  rfcmp::DevBuf sp_scratch;    // sparse projector solves: one region per factor (L, G_ll, G_tp)
  int64_t sp_region[3] = {0, 0, 0};  // complex128 offsets of the regions
  int sp_scratch_nrhs = 0;
  // compressed blocks (options.aca_tol > 0): T_A and V live here, TA and Vb
  // stay empty
  std::unique_ptr<rfcmp::HmOp> hm;
  rfcmp::DevBuf bcg_scratch;   // block CG: small matrices, Gram partials
  double2* bcg_host = nullptr;      // block CG: pinned and mapped Gram results, upload staging, norms
  double2* bcg_host_dev = nullptr;  // its device address
};

namespace rfcmp {

// mesh.cpp
rfcmp_status build_mesh_host(const double* xyz, int64_t nv, const int32_t* tri, int64_t nc, MeshHost& h);
void near_pairs(const MeshHost& h, double factor, std::vector<int32_t>& out);
void near_data(const MeshHost& h, double factor, NearData& out);
// Edge tiles of the T_A assembly (kEdgeTile consecutive edges): the cells
// of each tile (ptr/cell, ascending), the rows in the tile of their local
// edges (rows, 8 bits each, 0xFF outside), the tile of each cell's local edge
// 0 (home) and the most cells of a tile (cmax).
void edge_tiles(const MeshHost& h, std::vector<int>& ptr, std::vector<int>& cell, std::vector<int>& rows,
                std::vector<int>& home, int& cmax);
void build_cell_nb(MeshHost& h);

// assemble.hip
rfcmp_status mesh_upload(rfcmp_mesh m, hipStream_t s);
rfcmp_status assemble_blocks(rfcmp_op op, hipStream_t s);
// sv != nullptr: the split excitation e = Sigma sv + e (sv [nrhs][C], e the
// plane wave less its static part)
rfcmp_status rhs_planewave(rfcmp_op op, const double* khat, const double* pol, int nrhs,
                           double2* e, hipStream_t s, double2* sv = nullptr);
rfcmp_status rhs_planewave_noalloc(rfcmp_op op, const double* khat, const double* pol, int nrhs, double2* e,
                                   hipStream_t s);
rfcmp_status rhs_gap(rfcmp_mesh m, const int32_t* edges, const double2* volts, int ngap, int nrhs, double2* e,
                     hipStream_t s);
// js != nullptr: j is the loop part and js the star part of the current
rfcmp_status far_field(rfcmp_op op, const double2* j, const double2* js, int nrhs, const double* dirs, int ndir,
                       double2* F, double* rcs, hipStream_t s);

// spsolve.hip: the sparse factors of a mesh (which 0 = L, grounded; 1 = G_ll;
// 2 = G_tp, needs build_cell_nb first), and their upload: joins the host
// threads started at mesh creation (or factors here), uploads on an internal
// stream and waits for the copies.
HostFactor factor_mesh_matrix(const MeshHost& h, int which);
rfcmp_status mesh_sparse_projectors(rfcmp_mesh m, bool need_gtp);

// dense.hip
rfcmp_status mesh_projectors(rfcmp_mesh m, bool need_gtp, hipStream_t s);
// Make s wait for the projector builds enqueued by mesh_projectors.
rfcmp_status wait_projectors(rfcmp_mesh m, hipStream_t s);
// In-place inverse of an SPD matrix, FP64: A [n][n] (n a multiple of 64)
// holds an SPD matrix in its leading nvalid x nvalid block and the identity
// in the padding; on return that block holds A^-1 - shift 1 1^T (exactly
// symmetric), the padding the identity again.  ubuf, rbuf: device scratch of
// n * 64 doubles each.  Enqueued on s; does not wait.
rfcmp_status spd_inverse(double* A, int64_t n, int64_t nvalid, double shift, double* ubuf, double* rbuf,
                         hipStream_t s);
// Several such inverses, each on its own stream, their launches interleaved.
struct SpdInverseJob {
  double* A;
  int64_t n, nvalid;
  double shift;
  double *ubuf, *rbuf;
  hipStream_t s;
};
rfcmp_status spd_inverse_many(const SpdInverseJob* jobs, int njobs);

}  // namespace rfcmp
