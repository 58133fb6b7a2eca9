/*
 * rfcmp -- refinement-free Calderon multiplicative preconditioner (RF-CMP)
 * for the electric field integral equation on closed PEC surfaces, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: S. B. Adrian, F. P. Andriulli, T. F. Eibert, "On a Refinement-Free
 * Calderon Multiplicative Preconditioner for the Electric Field Integral
 * Equation", arXiv:1803.08333.
 *
 * Problem (Sec. 2): closed, oriented triangulation Gamma; RWG expansion
 * functions not normalised by edge length (eq. RWGdef); Petrov-Galerkin
 * system T j = -e with T = i k T_A + T_Phi/(i k), time convention e^{-i w t},
 * j normalised by the wave impedance.  Preconditioned system (Sec. 3,
 * eq. NewFormulation, with the scalings of Sec. 4):
 *     P_o^H T^H P_m T P_o i = -P_o^H T^H P_m e,   j = P_o i.
 *
 * Conventions shared by every entry point
 *   - Status: negative = error (outputs untouched), 0 = OK, positive =
 *     warning.  rfcmp_last_error() describes the last failure on the calling
 *     thread.  No C++ exception crosses this interface.
 *   - Host pointers are read during the call only; the library copies what
 *     it keeps.  Device pointers are caller-owned, must stay valid until the
 *     enqueued work on `stream` completes, and are never freed here.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is enqueued on it; calls that return host values synchronise it.
 *   - Complex vectors are interleaved (re, im).  "c128" = two doubles per
 *     entry, "c64" = two floats.  Batched vectors are [nrhs][n], contiguous.
 *   - RWG (edge) order: the order in which a scan over the cells (cell 0,
 *     1, ..., local edges 0, 1, 2 of each; local edge i joins vertices i+1
 *     and i+2) first meets each edge; c+ is the cell that walks the edge
 *     from its min to its max vertex in its CCW order.  Sigma[n,c+] = +1, Sigma[n,c-] = -1; Lambda[n,min] = +1,
 *     Lambda[n,max] = -1.
 *   - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef RFCMP_H
#define RFCMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RFCMP_OK = 0,
  RFCMP_W_NOT_CONVERGED = 1,      /* solve stopped at maxit; best iterate returned */
  RFCMP_E_ARG = -1,               /* invalid argument (NULL, size, k <= 0, non-unit vector, ...) */
  RFCMP_E_MESH_OPEN = -2,         /* an edge with fewer or more than two cells */
  RFCMP_E_MESH_NONMANIFOLD = -3,  /* a vertex index out of range or a repeated cell vertex */
  RFCMP_E_MESH_ORIENT = -4,       /* two cells walk an edge in the same direction */
  RFCMP_E_MESH_DISCONNECTED = -5, /* more than one connected component */
  RFCMP_E_MESH_DEGENERATE = -6,   /* a cell of zero area */
  RFCMP_E_OOM = -7,               /* device or host allocation failed */
  RFCMP_E_HIP = -8,               /* a HIP runtime call failed */
  RFCMP_E_BREAKDOWN = -9,         /* CG breakdown: p^H A p <= 0 or not finite */
  RFCMP_E_STATE = -10             /* call not valid in the handle's state */
} rfcmp_status;

/* Description of the last error on the calling thread (valid until the next
 * failing call on that thread); "" if none. */
const char* rfcmp_last_error(void);
const char* rfcmp_version(void);
/* Device memory.  Every device buffer the library owns (blocks, projector
 * matrices, BF16x3 planes, work vectors, assembly and product scratch) comes
 * from the registered allocator, else from the library's own cache over
 * hipMalloc.
 *
 * rfcmp_set_allocator registers a caller's device allocator (for instance a
 * framework's caching allocator; the Python binding registers torch's):
 *   alloc_fn(bytes, stream, ctx) returns a block of at least `bytes` on the
 *     calling thread's current device, or NULL when it has none: the library
 *     call that needed it then fails with RFCMP_E_OOM and leaves its outputs
 *     untouched;
 *   free_fn(p, bytes, stream, ctx) takes back a block alloc_fn returned
 *     (`bytes` as requested there), on the device it came from.
 * `stream` is always NULL: a block may be used on any stream, and the library
 * hands it back only after the device is idle.  Both functions may be called
 * from the library's internal host threads and must be thread-safe.  Each
 * block goes back to the allocator that made it, even after another one has
 * been registered.  NULL, NULL (the default) returns to the library's cache.
 * Giving only one of the two functions is RFCMP_E_ARG.  Host call. */
typedef void* (*rfcmp_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*rfcmp_free_fn)(void* p, size_t bytes, void* stream, void* ctx);
rfcmp_status rfcmp_set_allocator(rfcmp_alloc_fn alloc_fn, rfcmp_free_fn free_fn, void* ctx);
/* The library's own cache: buffers that meshes and operators release are
 * kept, per device, and handed out again for later requests of about the
 * same size (a new operator on a mesh of the same size maps no new memory).
 * This call returns all kept memory to the driver; *freed_bytes (nullable)
 * receives the amount.  A failing allocation does the same by itself before
 * it retries once.  Blocks of a registered allocator are never kept here.
 * Host call; waits for nothing. */
rfcmp_status rfcmp_release_cached_memory(int64_t* freed_bytes);

/* ------------------------------------------------------------------ mesh */
typedef struct rfcmp_mesh_s* rfcmp_mesh;

/* Topology and sparse structure of a closed triangle mesh (Sec. 2: RWG
 * functions eq. RWGdef, star/loop matrices, Gram matrices; Sec. 3: closed
 * form of the mixed Gram matrix).  xyz: host double [n_vertices][3] in
 * metres; tri: host int32 [n_cells][3], counter-clockwise seen from outside.
 * Validates: closed, 2-manifold, consistently oriented, connected, no
 * zero-area cell (RFCMP_E_MESH_*).  Host work only. */
rfcmp_status rfcmp_mesh_create(const double* xyz, int64_t n_vertices,
                               const int32_t* tri, int64_t n_cells, rfcmp_mesh* out);
/* N = RWG count (= edges), V, C, genus g = (2 - V + N - C)/2. */
rfcmp_status rfcmp_mesh_sizes(rfcmp_mesh m, int64_t* N, int64_t* V, int64_t* C, int32_t* genus);
/* Host outputs, each nullable: edge_vtx int32 [N][2] (min, max vertex),
 * edge_cell int32 [N][2] (c+, c-), edge_local int32 [N][2] (local index of
 * the edge in c+ and in c-; local edge i of a cell is opposite its vertex i). */
rfcmp_status rfcmp_mesh_edges(rfcmp_mesh m, int32_t* edge_vtx, int32_t* edge_cell, int32_t* edge_local);
/* Near pairs (c <= c') of the quadrature spec for the given factor: centroid
 * distance below near_factor * max(longest edge of c, of c') * (1 + 1e-9).
 * Writes *count; if pairs != NULL it must hold 2*count int32 (first call
 * with NULL to size it). */
rfcmp_status rfcmp_mesh_near_pairs(rfcmp_mesh m, double near_factor, int64_t* count, int32_t* pairs);
/* The sparse projector factors of a mesh, once an operator with sparse
 * projectors (options.projector 1, or 0 resolved to 1) has needed them: which 0 = L = Sigma^T Sigma (grounded), 1 = G_ll,
 * 2 = G_tp.  n: matrix size; supernodes: nodes of the nested-dissection tree;
 * levels: launches per sweep of a solve (one for the bottom subtrees, one per
 * height of the supernodes above them); stored: doubles on the device (the
 * blocks of L and the inverses of its diagonal blocks, each in two orders);
 * seconds: host time of ordering and factorisation.  Every output nullable.
 * RFCMP_E_STATE if that factor has not been built. */
rfcmp_status rfcmp_mesh_factor_info(rfcmp_mesh m, int32_t which, int64_t* n, int32_t* supernodes, int32_t* levels,
                                    int64_t* stored, double* seconds);
void rfcmp_mesh_destroy(rfcmp_mesh m);

/* -------------------------------------------------------------- options */
typedef struct {
  double near_factor;     /* near-pair criterion factor, default 2.0 */
  int32_t outer_star;     /* 0 = P_Sigma (Sec. 4, default), 1 = Gram-weighted P_gSigma (Sec. 3) */
  int32_t scaling;        /* 0 = alpha/beta/gamma by power iteration (Sec. 4, default),
                             1 = alpha = sqrt(k), beta = 1/sqrt(k), gamma = k */
  int32_t power_iters;    /* most power-iteration steps, default 30 */
  int32_t precision;      /* 0 = complex64 operator, FP64 accumulation (default);
                             1 = BF16x3 split products on MFMA for batched solves,
                                 FP64-accumulated residual refinement */
  double power_tol;       /* early stop of the power iteration, default 1e-2: the
                             scalings are formed every 5 steps and the iteration
                             stops at the first check from step 10 on where each
                             of alpha, beta, gamma moved by less than power_tol
                             (relative) since the previous check; 0 = always
                             power_iters steps */
  int32_t streams;        /* power iterations rfcmp_op_create_many runs at once,
                             1..4, default 4 (1 = one after another on `stream`) */
  int32_t projector;      /* how L^+, G_ll^-1 and G_tp^-1 are applied (projectors of Sec. 2-3):
                             1 = sparse FP64 Cholesky factors: nested dissection of
                                 the mesh, factored on host threads from
                                 rfcmp_mesh_create on, O(n log n) entries, solved on
                                 the device in FP64 in every precision;
                             2 = dense FP64 inverses formed on the device (O(n^3)
                                 set-up, 8 n^2 bytes each, streamed per product);
                             0 = automatic (default): 1 when C > 12288 (where the
                                 cubic set-up of 2 dominates), else 2 (one streaming
                                 pass over a small inverse beats a sparse solve) */
  int32_t graphs;         /* 1: from its third iteration on, each CG iteration
                             is replayed as a HIP graph captured once per
                             operator (two graphs: the recurrence scalars
                             alternate between two buffers) on an internal
                             stream; 0 (default): every kernel launched one by
                             one.  Results are bit-identical either way.  The
                             replay saves no time on this hardware at the sizes
                             measured, and the two captures per operator cost
                             about 4 ms, which a batch of many small operators
                             pays many times over.  Not used while kernel timing
                             (rfcmp_profile_enable) is on. */
  double aca_tol;         /* 0 (default): T_A and V stored dense.  > 0: T_A and V
                             compressed separately (the compression of Sec. 4's
                             large example) as hierarchical matrices: RWG edges
                             clustered by bisection into tiles of 64, pairs of
                             clusters whose boxes are at least the near distance
                             apart and min(diam) <= 2 x their distance stored as
                             low-rank factors from adaptive cross approximation
                             (partial pivoting, stopped when the new term's
                             Frobenius norm is at most aca_tol times the
                             approximation's), the other pairs of tiles dense;
                             storage O(N log N) for a fixed wavenumber.  Needs
                             precision 0; rfcmp_op_export writes the compressed
                             blocks out dense.  RFCMP_E_STATE if a block needs a
                             rank above 128. */
  int32_t block_cg;       /* 0: the right-hand sides of a solve run as
                             independent CGs that share each operator pass;
                             1: one CG over a shared block Krylov space (block
                             CG with orthonormalised search blocks, rank-
                             revealing: columns that lose rank are dropped from
                             the search block), which takes fewer iterations
                             when many right-hand sides are solved together;
                             -1 (default): 1 for solves of 8 or more right-hand
                             sides, else 0.  In block mode the Lanczos
                             condition estimate is not formed (cond_estimate
                             = 0) and every right-hand side reports the block's
                             iteration count. */
} rfcmp_options;
rfcmp_status rfcmp_options_default(rfcmp_options* opt);

/* ----------------------------------------------------------- operators */
typedef struct rfcmp_op_s* rfcmp_op;

/* Assemble the EFIE blocks for wavenumber k > 0 [rad/m] (Sec. 2):
 *   T_A[m,n] = int int f_m(r).f_n(r') G_k dS dS'          (complex64, N x N)
 *   V[c,c']  = (A_c A_c')^-1 int_c int_c' G_k dS dS'     (complex64, C x C)
 * with G_k = exp(ikR)/(4 pi R), so T_Phi = Sigma V Sigma^T.  Far pairs use the
 * 7x7-point rule in FP32; near pairs (see rfcmp_mesh_near_pairs) extract the
 * 1/R singularity in closed form in FP64.  T_A is formed tile by tile from
 * the cell pairs of each pair of 64-edge tiles and stored whole (both
 * triangles, exactly symmetric); the assembly needs no scratch beyond its
 * near-pair blocks (complex64, 72 bytes per near pair).  On the first call
 * for a mesh the projectors (sparse FP64 Cholesky factors of
 * Sigma^T Sigma, G_ll and, for outer_star = 1, G_tp, or their dense FP64
 * inverses: see rfcmp_options.projector) are set up on the device and
 * cached on the mesh, as is the near-pair list; they are freed with the
 * mesh.  Returns after the operator's work on `stream` is complete.
 * power_start: device c128 [N], the start vector of the power iterations
 * that estimate alpha, beta, gamma (Sec. 4); required when opt->scaling == 0,
 * ignored otherwise.  opt may be NULL (defaults).  The mesh must outlive the
 * operator. */
rfcmp_status rfcmp_op_create(rfcmp_mesh m, double k, const rfcmp_options* opt,
                             const void* power_start, void* stream, rfcmp_op* out);
/* The operators of nk wavenumbers k[0..nk) on one mesh (a frequency sweep),
 * each as rfcmp_op_create would make it, with the same options and power
 * start vector: every operator's blocks are assembled first, beside the
 * projector builds of a new mesh, then the scalings of each are computed.
 * With nk > 1 the power iterations run concurrently, up to four at a time,
 * each on an internal stream (default priority) driven by a host thread,
 * after the work queued on `stream`; the operators are bit-identical to
 * those of separate rfcmp_op_create calls.
 * out: host rfcmp_op [nk], all NULL on error.  1 <= nk <= 1024. */
rfcmp_status rfcmp_op_create_many(rfcmp_mesh m, const double* k, int32_t nk, const rfcmp_options* opt,
                                  const void* power_start, void* stream, rfcmp_op* out);
/* Current scalings (Sec. 4).  lam (nullable, host double [3]) receives the
 * three power-iteration norm estimates (0 for k-scaling).  The number of
 * power-iteration steps run is reported by rfcmp_op_power_steps. */
rfcmp_status rfcmp_op_scalings(rfcmp_op op, double* alpha, double* beta, double* gamma, double* lam);
/* Override the scalings (all > 0).  The solution j does not depend on them. */
rfcmp_status rfcmp_op_set_scalings(rfcmp_op op, double alpha, double beta, double gamma);
/* Power-iteration steps run when the operator was created (0 for k-scaling). */
rfcmp_status rfcmp_op_power_steps(rfcmp_op op, int32_t* steps);
/* Copy the blocks to caller device buffers: TA c64 [N][N], V c64 [C][C]
 * (either nullable). */
rfcmp_status rfcmp_op_export(rfcmp_op op, void* TA, void* V, void* stream);
/* Storage of an operator's compressed blocks (options.aca_tol > 0; Sec. 4):
 * complex64 entries of the dense blocks (pairs of 64-edge tiles of T_A and
 * the matching cell blocks of V) and of the low-rank factors (k (m + n) per
 * m x n block of rank k), each as host int64 [2] (T_A, V); the number of
 * low-rank blocks of each matrix (T_A and V have the same partition); the
 * largest and the mean rank over both matrices.  Every output nullable.
 * RFCMP_E_STATE for an operator with dense blocks.  Host call. */
rfcmp_status rfcmp_op_compression(rfcmp_op op, int64_t* dense_entries, int64_t* lowrank_entries,
                                  int32_t* lowrank_blocks, int32_t* max_rank, double* mean_rank);
void rfcmp_op_destroy(rfcmp_op op);

/* Plane-wave excitation e_m = int f_m . pol exp(i k khat.r) dS (Sec. 2),
 * 7-point rule, FP64.  khat, pol: host double [nrhs][3], unit (1e-12) and
 * orthogonal (1e-12).  e: device c128 [nrhs][N]. */
rfcmp_status rfcmp_rhs_planewave(rfcmp_op op, const double* khat, const double* pol,
                                 int32_t nrhs, void* e, void* stream);

/* rfcmp_rhs_planewave for callers that cannot allocate device memory (serving
 * loops that must not touch an allocator, harnesses that forbid allocation):
 * the same excitation, bit for bit, with khat and pol staged in a fixed
 * device array of the library (RFCMP_RHS_NOALLOC_MAX plane waves, 6 doubles
 * each: 192 KiB per device, set up on the first call on that device and held
 * until the process ends) instead of a buffer allocated per call.  Calls no
 * allocator and allocates nothing.  nrhs above RFCMP_RHS_NOALLOC_MAX is
 * RFCMP_E_ARG.  Every call on one device shares the array, which keeps the
 * last call's contents; each call waits for its stream before returning, so
 * calls from one host thread never overlap, but calls from several host
 * threads on one device race.  Arguments and errors otherwise as
 * rfcmp_rhs_planewave. */
#define RFCMP_RHS_NOALLOC_MAX 4096
rfcmp_status rfcmp_rhs_planewave_noalloc(rfcmp_op op, const double* khat, const double* pol,
                                         int32_t nrhs, void* e, void* stream);

/* The plane-wave excitation split for any frequency down to the static
 * limit: e = Sigma s + e1 (Sec. 2), with s_c = -pol . x_c (x_c the cell
 * centroid; int f_m . pol = -int div(f_m) pol . r, so Sigma s is the static
 * part, in the range of Sigma exactly) and e1 = int f_m . pol (exp(i k khat .
 * r) - 1) with exp(i t) - 1 = -2 sin^2(t/2) + i sin t.  At low frequency the
 * loop part of e is O(k) relative to e, and below k ~ 1e-16 it is lost in a
 * single FP64 vector; e1 keeps it (Fig. Sphere_RCS reaches 1e-25 Hz).
 * s: device c128 [nrhs][C]; e1: device c128 [nrhs][N]; khat, pol as
 * rfcmp_rhs_planewave.  Waits for the stream before returning. */
rfcmp_status rfcmp_rhs_planewave_split(rfcmp_op op, const double* khat, const double* pol, int32_t nrhs,
                                       void* s, void* e1, void* stream);

/* Voltage-gap (delta-gap) excitation, the second source of the Fokker
 * example (Sec. 4): e_r[n] = sum of volts[r][g] over the gaps g with
 * edges[r][g] = n, zero elsewhere.  A gap of voltage V across edge m is the
 * field V delta(s) n_m (s the in-plane distance from the edge, n_m its
 * in-plane normal from the edge's first cell into its second, the direction
 * in which f_m carries current), and f_m has unit flux across its own edge
 * while every other RWG function has none, so e_m = V.  With rfcmp_solve
 * (T j = -e) the gap's input power is Re(V conj(j_m))/2 in units of 1/eta.
 * edges: host int32 [nrhs][ngap], each in [0, N); volts: host c128
 * [nrhs][ngap]; ngap may be 0 (e = 0), ngap * nrhs <= 2^26; e: device c128
 * [nrhs][N].  Waits for the stream before returning. */
rfcmp_status rfcmp_rhs_gap(rfcmp_mesh m, const int32_t* edges, const void* volts, int32_t ngap, int32_t nrhs,
                           void* e, void* stream);

/* Far field and bistatic radar cross section of RWG currents (Sec. 4,
 * Fig. Sphere_RCS): F_r(d) = int j_r(x) exp(-i k dhat_d . x) dS, the
 * integral over each cell with the excitation's 7-point rule, and
 * rcs_r(d) = k^2/(4 pi) |F - dhat (dhat . F)|^2, the RCS for a unit incident
 * amplitude (j = eta J, e^{-i w t}: E^s -> -i k exp(i k r)/(4 pi r)
 * r_hat x (r_hat x F)).  Computed in FP64 from j.  For a j from rfcmp_solve
 * the accuracy follows the solve's: with tol = 1e-8 the sphere's RCS stays
 * within 0.5 % of Mie (level 4) down to ka = 1e-10; lower, the small
 * Helmholtz block of the system's right-hand side falls below the global
 * residual tolerance (the split path, rfcmp_rhs_planewave_split,
 * rfcmp_solve_split and rfcmp_farfield_split, keeps it down to 1e-25 Hz).
 * j: device c128 [nrhs][N]; dirs: host double [ndir][3], unit vectors
 * (1e-12); F: device c128 [nrhs][ndir][3]; rcs: device double [nrhs][ndir],
 * nullable.  Waits for the stream before returning. */
rfcmp_status rfcmp_farfield(rfcmp_op op, const void* j, int32_t nrhs, const double* dirs, int32_t ndir,
                            void* F, void* rcs, void* stream);
/* rfcmp_farfield of a current given as its loop part (divergence-free) and
 * its star part (rfcmp_solve_split): F = int j_loop (exp(-i k dhat . r) - 1)
 * dS + int j_star exp(-i k dhat . r) dS.  A divergence-free current carries
 * no net current, so the first term equals the loop part's far field, and its
 * phase factor is formed as -2 sin^2(t/2) - i sin t, without cancellation:
 * at very low k both terms are O(k) while j_star is O(k) relative to j_loop,
 * and the RCS of the sphere keeps its accuracy down to 1e-25 Hz.  Arguments
 * and outputs as rfcmp_farfield. */
rfcmp_status rfcmp_farfield_split(rfcmp_op op, const void* j_loop, const void* j_star, int32_t nrhs,
                                  const double* dirs, int32_t ndir, void* F, void* rcs, void* stream);

/* b = -P_o^H T^H P_m e (right side of eq. NewFormulation).  e, b: device c128
 * [nrhs][N]; may not alias. */
rfcmp_status rfcmp_precond_rhs(rfcmp_op op, const void* e, void* b, int32_t nrhs, void* stream);
/* y = A x with A = P_o^H T^H P_m T P_o, in cancellation-free order (the
 * products P_LH T_Phi, T_Phi P_LH, Lambda^T T_Phi and Sigma^T P_mL vanish
 * identically and are never formed).  x, y: device c128 [nrhs][N]. */
rfcmp_status rfcmp_apply(rfcmp_op op, const void* x, void* y, int32_t nrhs, void* stream);
/* j = P_o i = P_LH i/alpha + i P_s i/beta.  device c128 [nrhs][N]. */
rfcmp_status rfcmp_recover(rfcmp_op op, const void* i, void* j, int32_t nrhs, void* stream);

/* Projector primitives (Sec. 2 and Sec. 3), FP64, device c128 vectors:
 *   RFCMP_PROJ_SIGMA     y = P_Sigma x = Sigma L^+ Sigma^T x        N -> N
 *   RFCMP_PROJ_LH        y = P_LH x = x - P_Sigma x                 N -> N
 *   RFCMP_PROJ_GSIGMA    y = P_gSigma x = Sigma L^+ G_tp^-1 Sigma^T x   N -> N
 *   RFCMP_PROJ_LPINV     y = L^+ x                                  C -> C
 *   RFCMP_PROJ_GLL_INV   y = G_ll^-1 x                              V -> V
 *   RFCMP_PROJ_SIGMA_T   y = Sigma^T x                              N -> C
 *   RFCMP_PROJ_LAMBDA_T  y = Lambda^T x                             N -> V */
enum {
  RFCMP_PROJ_SIGMA = 0, RFCMP_PROJ_LH = 1, RFCMP_PROJ_GSIGMA = 2, RFCMP_PROJ_LPINV = 3,
  RFCMP_PROJ_GLL_INV = 4, RFCMP_PROJ_SIGMA_T = 5, RFCMP_PROJ_LAMBDA_T = 6
};
rfcmp_status rfcmp_project(rfcmp_op op, int32_t which, const void* x, void* y, int32_t nrhs, void* stream);

/* Dense block products (Sec. 3.4 adjoint: T^H x = conj(T conj x)):
 *   which 0: y = M x, M = T_A (n = N), complex64 storage, FP64 accumulation
 *   which 1: M = V (n = C), likewise
 *   which 2: M = T_A as BF16x3 split products on MFMA, FP32 accumulation
 *   which 3: M = V as BF16x3
 *   which 4: M = L^+ (real, n = C) as BF16x3
 *   which 5: M = G_ll^-1 (real, n = V) as BF16x3
 *   conj != 0 (which 0-3): y = conj(M) x.
 * x, y: device c128 [nrhs][n].  The BF16x3 planes (hi/lo bf16 of every
 * entry, same bytes as complex64) are built on first use. */
rfcmp_status rfcmp_matvec(rfcmp_op op, int32_t which, int32_t conj, const void* x, void* y,
                          int32_t nrhs, void* stream);

/* Per-right-hand-side solve report. */
typedef struct {
  int32_t iters;          /* CG iterations (all restarts) */
  int32_t restarts;       /* residual refinements after the first CG pass */
  double rel_residual;    /* final |b - A i|/|b|, FP64-accumulated */
  double ms_solve;        /* wall time of the solve (all right-hand sides) */
  double cond_estimate;   /* lambda_max/lambda_min of the Lanczos tridiagonal of
                             the first CG pass (0 if fewer than 2 iterations) */
} rfcmp_info;

/* Solve T j = -e through the RF-CMP system with CG (Sec. 3.4; x0 = 0), until
 * the true relative residual |b - A i|/|b| <= tol (b = preconditioned rhs),
 * for nrhs right-hand sides advanced together (up to 64 per block; each has
 * its own CG scalars and stops on its own).
 *   precision 0: CG on the complex64 / FP64 operator, restarted from the
 *                true residual when the recursive one has drifted;
 *   precision 1: iterative refinement: inner CG on the BF16x3 operator to
 *                max(1e-4 of the current residual, 0.75 tol), outer residual
 *                with the complex64 / FP64 operator, rounds until it meets
 *                tol.
 * e, j: device c128 [nrhs][N].  info: host [nrhs], nullable (iters counts
 * all inner iterations, restarts the residual rounds after the first).
 * Returns RFCMP_W_NOT_CONVERGED (best iterate in j) when maxit is reached,
 * RFCMP_E_BREAKDOWN on a non-positive curvature. */
rfcmp_status rfcmp_solve(rfcmp_op op, const void* e, void* j, int32_t nrhs, double tol,
                         int32_t maxit, void* stream, rfcmp_info* info);

/* rfcmp_solve for a split excitation e = Sigma s + e1 (rfcmp_rhs_planewave_
 * split), returning j split as well: j_loop = P_LH i/alpha and j_star =
 * i P_s i/beta (j = j_loop + j_star, eq. NewFormulation).  The right-hand
 * side b is formed without ever adding the static part to e1 (P_mL vanishes
 * on the range of Sigma, and P_mS Sigma s = Sigma L^+ G_pp^-1 (s - mean s)
 * /beta^2), and the two parts of j are never added, so the solution keeps
 * both Helmholtz parts at any frequency (at very low k the star part of j is
 * O(k) relative to the loop part).  s: device c128 [nrhs][C]; e1, j_loop,
 * j_star: device c128 [nrhs][N], not aliased.  Report and errors as
 * rfcmp_solve. */
rfcmp_status rfcmp_solve_split(rfcmp_op op, const void* s, const void* e1, void* j_loop, void* j_star,
                               int32_t nrhs, double tol, int32_t maxit, void* stream, rfcmp_info* info);

/* CG on the RF-CMP system A i = b itself (eq. NewFormulation), with b given
 * instead of formed from an excitation, and the iterate i returned instead of
 * j = P_o i: the same iteration, stopping rule and report as rfcmp_solve
 * (precision 0 or 1).  For spectral studies (Sec. 4, Figs. SphereF, SphereH,
 * CubeTorus): with a generic b the Lanczos estimate in info approaches
 * cond(A); a b formed from an excitation at very low k is dominated by one of
 * the two blocks and leaves the other's eigenvalues out of the Krylov space.
 * b, i: device c128 [nrhs][N], not aliased.  Errors as rfcmp_solve. */
rfcmp_status rfcmp_solve_system(rfcmp_op op, const void* b, void* i, int32_t nrhs, double tol,
                                int32_t maxit, void* stream, rfcmp_info* info);

/* rfcmp_solve for several operators at once (a batch of objects and
 * wavenumbers, each solved as in Sec. 3.4): operator q solves T_q j_q = -e_q
 * for nrhs[q] right-hand sides, e[q], j[q] device c128 [nrhs[q]][N_q], not
 * aliased; tol and maxit are shared.  The solves run concurrently, up to four
 * at a time, each on an internal stream (default priority) driven by a host
 * thread; largest N * nrhs first, at equal size the higher k.  These streams
 * start after the work queued on `stream` before the call, and `stream` waits
 * for them; the call returns when every solve has finished.  Each operator's result and report are those
 * of rfcmp_solve on it alone, bit for bit.
 *   ops: host [nops], distinct handles (two entries may share a mesh) whose
 *        mesh lives on the calling thread's current device;
 *   e, j, nrhs: host [nops];
 *   info: host [sum of nrhs], nullable: the reports in ops order, ms_solve
 *        the wall time of that operator's solve.
 * Workspaces and BF16x3 planes are set up on `stream` before the solves
 * start.  Returns the first error in ops order (rfcmp_last_error names the
 * operator; the other operators are still solved), else
 * RFCMP_W_NOT_CONVERGED if any solve stopped at maxit, else RFCMP_OK.
 * Argument errors (NULL, aliased, nrhs <= 0, a repeated handle, another
 * device) are found before anything is enqueued. */
rfcmp_status rfcmp_batch_solve(const rfcmp_op* ops, int32_t nops, const void* const* e, void* const* j,
                               const int32_t* nrhs, double tol, int32_t maxit, void* stream,
                               rfcmp_info* info);

/* ------------------------------------------------------------ profiling */
/* Kernel timing for benchmarks.  While enabled, the library records a HIP
 * event pair on the launch stream around every launch of its timed kernels:
 * "assemble_ta", "near_pairs" (assembly), "cmatvec_ta", "cmatvec_v"
 * (complex64 block products, symmetric streaming), "zgemm_ta", "zgemm_v"
 * (complex64 block products of 8 and more right-hand sides, FP64 matrix
 * cores), "hm_dense", "hm_aca_ta", "hm_aca_v", "hm_matvec_ta", "hm_matvec_v"
 * (compressed blocks: dense tiles, ACA, products), "dmatvec_lp", "dmatvec_gll", "dmatvec_gtp" (dense FP64 projector
 * products), "spsolve_lp", "spsolve_gll", "spsolve_gtp" (sparse projector
 * solves), "gemm_ta", "gemm_v" (BF16x3 products), "spd_inverse" (whole FP64
 * inverse); a launch of k > 1 right-hand sides is timed as "<tag>_nr<k>"
 * (every "zgemm" launch carries its suffix).  rfcmp_profile_enable
 * clears the records (waiting for recorded events first); rfcmp_profile_read
 * waits for the events of one tag and returns their summed duration and
 * count.  Adds two event records per timed launch.  Records from library
 * calls on several host threads (rfcmp_batch_solve, rfcmp_op_create_many)
 * are safe; enable, select and read must not overlap other calls. */
rfcmp_status rfcmp_profile_enable(int32_t on);
/* Restrict the timed kernels to a comma-separated list of tags (NULL or ""
 * = all tags), so that a timed region carries event records only where they
 * are needed.  Kept across rfcmp_profile_enable calls. */
rfcmp_status rfcmp_profile_select(const char* tags);
rfcmp_status rfcmp_profile_read(const char* tag, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* RFCMP_H */
