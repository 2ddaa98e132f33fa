/*
 * cbfm.h - C ABI of the MI355X (gfx950) implementation of the characteristic
 * basis function method with the Calderon multiplicative preconditioner for
 * the PMCHWT formulation of scattering by a homogeneous dielectric body
 * (Tanaka, Niino, Nishimura, arXiv 2111.11058).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Units: lengths in free-space wavelengths is customary but not required;
 *   k0 and eta0 are passed explicitly.  Time convention e^{jwt}; Green's
 *   function G_i = e^{-j k_i R} / (4 pi R) (paper Sec. II-A).
 * - Exterior medium 1 is vacuum (k1 = k0, eta1 = eta0).  The interior medium
 *   2 has relative eps_r and mu_r (complex; a lossy eps_r = e' - j e'' has
 *   Im k2 < 0).  k2 = k0 sqrt(eps_r mu_r), eta2 = eta0 sqrt(mu_r/eps_r),
 *   principal square roots.
 * - RWG basis (paper Sec. II-B, Rao-Wilton-Glisson): edges are the unique
 *   vertex pairs (min v, max v) sorted lexicographically ("canonical order");
 *   T+ of an edge is the triangle whose counter-clockwise (outward) cycle
 *   runs min -> max; f = (l / 2A+)(r - p+) on T+, (l / 2A-)(p- - r) on T-.
 * - Operators (paper Sec. II-B, Galerkin entries of K_i and T_i):
 *     [T_i]_mn = j k_i int int G_i [f_m . f_n - div f_m div f_n / k_i^2]
 *     [K_i]_mn = int int f_m . (grad' G_i x f_n)     (gradient on the source)
 *   With this reading of the operator signs the solved coefficient vector is
 *   the negative of the physical currents; far fields and RCS are unchanged.
 *   Z = [[K, -TE], [TH, K]] with K = K1 + K2, TE = eta1 T1 + eta2 T2,
 *   TH = T1/eta1 + T2/eta2; unknowns [alpha^M ; alpha^J] (discretised PMCHWT
 *   system and coefficient vector, Sec. II-B).
 * - Quadrature: 7-point degree-5 rule on every triangle; near triangle pairs
 *   (same triangle, a shared vertex, or centroid distance < 1.5 x the longer
 *   of the two longest edges) use closed-form integration of the 1/R, R
 *   (resp. 1/R^3, 1/R) parts on the source triangle; K of a coplanar near
 *   pair is 0.
 * - Complex numbers are interleaved (re, im): double2 for FP64, float2 for
 *   FP32, matching torch.complex128 / torch.complex64 elements.
 * - Matrices are row-major with an explicit leading dimension.  A block of
 *   several vectors (right-hand sides) is stored vector after vector:
 *   element i of vector c at [c * n + i].
 * - Device pointers ("_dev") must point to device memory of the current HIP
 *   device, large enough for the stated extent; host pointers ("_host") are
 *   read or written during the call only.  All device work is enqueued on
 *   ``stream`` (a hipStream_t; NULL = the default stream) and the call
 *   returns without synchronising unless it says otherwise.  Calls that
 *   return host results synchronise the stream.
 * - Handles (cbfm_mesh, cbfm_cbf) own their device memory and are immutable
 *   after creation; several streams may use one handle concurrently.
 * - Errors: every call returns a cbfm_status; no C++ exception crosses the
 *   ABI.  On CBFM_E_ARG / CBFM_E_MESH outputs are untouched.
 *   cbfm_last_error() gives a thread-local message for the last failure.
 */
#ifndef CBFM_H
#define CBFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cbfm_mesh_s* cbfm_mesh;
typedef struct cbfm_cbf_s* cbfm_cbf;
typedef struct cbfm_mom_s* cbfm_mom;

typedef enum {
  CBFM_OK = 0,
  CBFM_E_ARG = -1,     /* invalid argument (null pointer, size, range)      */
  CBFM_E_MESH = -2,    /* not a closed, consistently oriented 2-manifold    */
  CBFM_E_NOMEM = -3,   /* device or host allocation failed                  */
  CBFM_E_HIP = -4,     /* a HIP call failed                                 */
  CBFM_E_NOCONV = -5,  /* GMRES reached max_iter; outputs hold the iterate  */
  CBFM_E_RANK = -6,    /* a cell kept no CBF (L_m = 0), or a matrix to be
                          solved or inverted has no nonzero pivot          */
  CBFM_E_STATE = -7    /* handles of different meshes mixed                 */
} cbfm_status;

typedef enum {
  CBFM_FP64 = 0,       /* everything in double                                  */
  CBFM_FP32 = 1,       /* regular-pair fill in float; the rest in double        */
  CBFM_MIXED_FP32 = 2, /* projection only: float fill and panel, projection on  */
                       /* the FP32 matrix cores (FP32 accumulation)             */
  CBFM_MIXED_BF16 = 3, /* projection only: as MIXED_FP32 with BF16 inputs to   */
                       /* the matrix cores (FP32 accumulation)                  */
  CBFM_MIXED_BF16X3 = 4 /* projection only: split BF16 (x = hi + lo, products  */
                        /* hi hi + hi lo + lo hi, about 16 significant bits)    */
} cbfm_precision;

/* Output layout of cbfm_fill_pmchwt: three (four for MEDIA4) nrow x ncol
   complex matrices, matrix after matrix. */
enum {
  CBFM_LAYOUT_MEDIA3 = 0, /* [K1 + K2, T1, T2]                                */
  CBFM_LAYOUT_OPS3 = 1,   /* [K, TE = eta1 T1 + eta2 T2, TH = T1/eta1 + T2/eta2] */
  CBFM_LAYOUT_MEDIA4 = 2  /* [K1, K2, T1, T2]: every medium's operators apart */
};

/* Interior medium and free-space constants. */
typedef struct {
  double k0;            /* free-space wavenumber                      */
  double eta0;          /* free-space wave impedance                  */
  double eps_re, eps_im;/* interior relative permittivity             */
  double mu_re, mu_im;  /* interior relative permeability             */
} cbfm_medium;

/* Thread-local description of the last error (never NULL). */
const char* cbfm_last_error(void);

/* ------------------------------------------------------- device memory ---
 * cbfm_set_allocator: the caller's device allocator (for example PyTorch's
 * caching allocator) for all device memory of the library: the buffers that
 * handles own and the stream-ordered scratch of every call.  alloc(bytes,
 * stream) returns device memory of the current device, usable in the order
 * of `stream` (NULL for handle buffers, which any stream may use), or NULL
 * on failure (the call then fails with CBFM_E_NOMEM); release(p, stream)
 * gives it back once the work queued on `stream` is done with it (handle
 * buffers: when the handle is freed, stream NULL).  The routines may be
 * called from any thread (serving workers), and must be callable until
 * every block obtained through them is released.  Passing NULL for both
 * restores the library's own device allocations (hipMalloc with a cache of
 * freed scratch blocks).  Blocks keep the routine that gave them out; the
 * cached hipMalloc blocks are freed when an allocator is set.  Not
 * thread-safe against calls in flight: set it before other work.          */
typedef void* (*cbfm_alloc_fn)(size_t bytes, void* stream);
typedef void (*cbfm_release_fn)(void* p, void* stream);
cbfm_status cbfm_set_allocator(cbfm_alloc_fn alloc, cbfm_release_fn release);

/* Device bytes the library holds from its own hipMalloc allocations (handle
   buffers and cached or live scratch; memory from a caller's allocator is
   not counted), the most it held at once since the process started, and
   the part now idle in the scratch cache of the current device (any may
   be NULL).                                                               */
cbfm_status cbfm_memory_stats(int64_t* held, int64_t* peak, int64_t* cached);

/* ABI version (incremented on incompatible change). */
int32_t cbfm_version(void);  /* 7: cbfm_ipcbf_params gained block (6: cbfm_solver_params
                                gained block; 5: sstep; 4: basis_fp32; 3: cbfm_request gained
                                inner_fp32; 2: cbfm_solver_params gained cmp_mode, cmp_inner_tol) */

/* -------------------------------------------------------------- timers ---
 * Opt-in kernel timing for measurement: when enabled, the library records a
 * pair of HIP events on the launch stream around each launch of a named
 * kernel family and accumulates the elapsed times when they are read.
 * Names (bit i of the mask) and the unit of their algorithmic work:
 *   0 "fill_regular"  triangle pairs      1 "fill_near"    near pairs
 *   2 "assemble"      (none, 0)           3 "gemm"         real flops
 *   4 "gmres_dots"    bytes of basis vectors the Arnoldi dot pass reads
 *   5 "gmres_update"  bytes the Arnoldi update pass reads and writes (basis,
 *                     w and the Hessenberg entries of p = H a)
 *   6 "fill_regular_f32"  triangle pairs of the regular fill in float
 *   7 "xgemm"         real flops of the FP32 / BF16 matrix-core GEMMs
 *   8 "gemm_panel"    real flops of the "gemm" launches that ran on the
 *                     row-block kernel (one product of at most 32 columns,
 *                     such as the GMRES matrix-vector product), its
 *                     reduction of the K-split parts included
 * ("fill_regular" and "gemm" then count the double-precision launches.)
 * (the GMRES figures count every right-hand side of the batch, also those
 * already converged, which the kernels skip).
 * cbfm_timer_enable(mask) clears all timers and times the families whose
 * bit is set in mask (-1: all, 0: none).  Every timed launch adds two event
 * records to its stream, so time only the families being measured.
 * cbfm_timer_read synchronises the recorded events and returns the number
 * of launches, their total duration in milliseconds and their summed work
 * (any output may be NULL; CBFM_E_ARG for an unknown name).               */
cbfm_status cbfm_timer_enable(int32_t mask);
cbfm_status cbfm_timer_read(const char* name, int64_t* launches, double* total_ms, double* work);

/* ---------------------------------------------------------------- mesh ---
 * cbfm_mesh_load: validate a closed triangle mesh and build the RWG tables
 * (paper Sec. II-B basis expansion; Sec. III-A cell division: every edge
 * belongs to exactly one cell).
 *   xyz_host   nv x 3 vertex coordinates (double)
 *   tri_host   nt x 3 vertex indices (int32), counter-clockwise seen from
 *              outside
 *   edge_block_host  ne entries in canonical edge order giving each edge's
 *              cell in [0, nblocks), or NULL for a single cell (nblocks is
 *              then ignored)
 * Fails with CBFM_E_MESH if an edge is not shared by exactly two triangles
 * with opposite directions, a triangle is degenerate, the enclosed volume is
 * not positive, or a cell is empty.  Uploads the tables to the current
 * device (synchronous).  The handle is freed with cbfm_mesh_free.
 * Arrays: the load also notes whether every cell is cell 0 moved by one
 * vector (equal RWG counts; RWG i of each cell, in cell order, on triangles
 * whose vertices in stored order are cell 0's plus the shift, within 1e-9 of
 * the mesh extent; no triangle carrying RWGs of two cells), which
 * cbfm_build_cbf and cbfm_project use (paper Sec. IV-A: identical cells).
 */
cbfm_status cbfm_mesh_load(const double* xyz_host, int64_t nv, const int32_t* tri_host,
                           int64_t nt, const int32_t* edge_block_host, int32_t nblocks,
                           cbfm_mesh* out);

/* Sizes: RWG count ne, triangle count nt, cell count, near-pair count
   (any pointer may be NULL). */
cbfm_status cbfm_mesh_info(cbfm_mesh m, int64_t* ne, int64_t* nt, int32_t* nblocks,
                           int64_t* n_near);

/* Canonical edge table: ne x 2 vertex ids (int32, host), or NULL; the
   cell of each edge (int32, host), or NULL. */
cbfm_status cbfm_mesh_edges(cbfm_mesh m, int32_t* edge_vertices_host, int32_t* edge_block_host);

/* Frees the mesh.  Every cbfm_cbf built on or imported for it must be freed
   first: a CBF handle reads the mesh's tables, also from the library's side
   stream while the CMP inverse that cbfm_build_cbf queued is running. */
void cbfm_mesh_free(cbfm_mesh m);

/* cbfm_mesh_analyze: the host-side part of cbfm_mesh_load only (validation,
   canonical edges, near-pair list), touching no device, e.g. to check a mesh
   on a machine without a GPU.  Same arguments and failures as
   cbfm_mesh_load.  Outputs (each may be NULL): ne; edges_host (ne x 2,
   capacity 3 nt / 2 rows); tri_edge_host and tri_sign_host (nt x 3: edge
   and RWG sign (+1 on T+, -1 on T-) of the local function whose free vertex
   is vertex a of the triangle); n_near; near_host (n_near x 3: P, Q,
   coplanar; capacity given by near_cap rows, CBFM_E_ARG if too small).    */
cbfm_status cbfm_mesh_analyze(const double* xyz_host, int64_t nv, const int32_t* tri_host,
                              int64_t nt, const int32_t* edge_block_host, int32_t nblocks,
                              int64_t* ne, int32_t* edges_host, int32_t* tri_edge_host,
                              int32_t* tri_sign_host, int64_t* n_near, int32_t* near_host,
                              int64_t near_cap);

/* ---------------------------------------------------------------- fill ---
 * cbfm_fill_pmchwt: Galerkin matrices of the PMCHWT operators (paper
 * Sec. II-B, entries [K_i]_mn, [T_i]_mn and the block matrix Z) for test
 * RWGs row0 .. row0+nrow-1 and trial RWGs col0 .. col0+ncol-1 (canonical
 * order).
 *   precision  CBFM_FP64: arithmetic and output in double (out: double2);
 *              CBFM_FP32: regular pairs in float, near pairs in double,
 *              output float2.
 *   layout     CBFM_LAYOUT_MEDIA3 or CBFM_LAYOUT_OPS3 (see above)
 *   out_dev    3 matrices (4 for MEDIA4), matrix o element (r, c) at
 *              out_dev[(o * nrow + r) * ld + c]; ld >= ncol.  MEDIA4 fills
 *              [K1 + K2, T1, T2] and, apart, the K operator of the body with
 *              the exterior medium inside (exactly 2 K1: the kernel sums
 *              two equal media), then K1 = that / 2 and K2 = (K1 + K2) - K1;
 *              it takes twice the time of the other layouts
 * Uses stream-ordered scratch of about 3 * 9 * ntr * ntc complex elements,
 * ntr/ntc the triangles touching the row/column ranges.  Synchronises the
 * stream.
 */
cbfm_status cbfm_fill_pmchwt(cbfm_mesh m, const cbfm_medium* med, int32_t precision,
                             int64_t row0, int64_t nrow, int64_t col0, int64_t ncol,
                             int32_t layout, void* out_dev, int64_t ld, void* stream);

/* cbfm_fill_pmchwt_noalloc: cbfm_fill_pmchwt (same arguments, same
 * results) for callers that cannot allocate device memory -- code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation: it calls no hipMalloc, hipFree or other allocating routine.
 * Its workspace (index tables, near-pair intermediates, triangle-local
 * blocks) is a library array of CBFM_FILL_NOALLOC_MAX_BYTES bytes per
 * device, held from the first call on that device until the process ends;
 * ranges whose workspace exceeds it (about 27 x (triangles touching the
 * rows) x (triangles touching the columns) x 16 bytes in FP64, 8 in FP32)
 * are rejected with CBFM_E_ARG before any device work.  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * several streams or host threads) race and must be serialised by the
 * caller.  Nothing in the array needs clearing between calls.
 * Synchronises the stream, as cbfm_fill_pmchwt does.                      */
#define CBFM_FILL_NOALLOC_MAX_BYTES (64ll << 20)
/* (the MEDIA4 layout is not offered by the allocation-free fill) */
cbfm_status cbfm_fill_pmchwt_noalloc(cbfm_mesh m, const cbfm_medium* med, int32_t precision,
                                     int64_t row0, int64_t nrow, int64_t col0, int64_t ncol,
                                     int32_t layout, void* out_dev, int64_t ld, void* stream);

/* cbfm_rhs: tested incident plane waves (paper Sec. II-B, v^E and v^H):
   v = [v^E ; v^H] with v^E_m = int f_m . E_inc, v^H_m = -int f_m . H_inc,
   E_inc = p exp(-j k0 k . r), H_inc = k x E_inc / eta0, 7-point rule.
     inc_host  nrhs x 6 doubles (kx, ky, kz, px, py, pz), unit k, unit p
     v_dev     nrhs x 2ne double2, vector after vector                      */
cbfm_status cbfm_rhs(cbfm_mesh m, const cbfm_medium* med, const double* inc_host, int64_t nrhs,
                     void* v_dev, void* stream);

/* ---------------------------------------------------------------- CBFs ---
 * cbfm_build_cbf: primary CBFs with dual orthogonalisation (paper Sec.
 * III-A eq. of the primary CBFs, Sec. III-B eqs. of G_m, G'_m, the SVD and
 * C^M = J^M U_L, C^J = J^J V_L): per cell, Z_mm J_m = V_m for the n_gen
 * generating waves (Gauss-Jordan elimination, pivot rows chosen by partial
 * pivoting in a tournament over row groups, all cells in one batch),
 * G'_m = (J^M)^H G_m J^J, SVD, keep sigma_i/sigma_1 >=
 * delta_svd (at most max_L if max_L > 0).  FP64 throughout.
 * Synchronises the stream (the kept counts L_m are host data).
 * On a mesh of translated copies of one cell (see cbfm_mesh_load) the
 * waves on each cell are those on cell 0 times one phase per wave, so every
 * cell receives cell 0's count, singular values and CBFs (the same spaces).
 * Before returning, the CMP inverse of the new set (see cbfm_cmp_apply) is
 * queued on a library-owned side stream that waits for the build's work on
 * `stream`, so that it runs beside what the caller queues next; its first
 * use waits for it, and cbfm_cbf_free waits for it before freeing.
 * Returns CBFM_E_ARG for n_gen outside [1, 4096] or a mesh of more than
 * 32767 cells or 32767 RWGs in one cell, CBFM_E_RANK if a cell's Z_mm is
 * singular or a cell keeps no CBF.                                         */
typedef struct {
  const double* gen_host; /* n_gen x 6 (k, p) generating plane waves */
  int32_t n_gen;
  double delta_svd;
  int32_t max_L;          /* 0 = no cap */
} cbfm_cbf_params;

cbfm_status cbfm_build_cbf(cbfm_mesh m, const cbfm_medium* med, const cbfm_cbf_params* prm,
                           void* stream, cbfm_cbf* out);

/* cbfm_cbf_import: wrap given CBFs (for parity checks with an external
   computation).  L_host: per-cell counts; CM_host / CJ_host: cell after cell,
   each N_m x L_m row-major double2 with rows in canonical edge order of the
   cell's edges; sigma_host: sum(L) doubles (cell after cell).  On a mesh of
   translated copies of one cell, CBFs identical (bit for bit) in every cell
   are shared as those of cbfm_build_cbf (projection by cell offsets).      */
cbfm_status cbfm_cbf_import(cbfm_mesh m, const int32_t* L_host, const void* CM_host,
                            const void* CJ_host, const double* sigma_host, void* stream,
                            cbfm_cbf* out);

/* Sizes: total N_CBF = 2 sum L, per-cell L (nblocks int32, or NULL), kept
   singular values (sum L doubles, cell after cell, or NULL).               */
cbfm_status cbfm_cbf_info(cbfm_cbf c, int64_t* n_cbf, int32_t* L_host, double* sigma_host);

/* Copy the CBF coefficients to the host in the cbfm_cbf_import layout.     */
cbfm_status cbfm_cbf_export(cbfm_cbf c, void* CM_host, void* CJ_host);

void cbfm_cbf_free(cbfm_cbf c);

/* ---------------------------------------------------------- projection ---
 * cbfm_project: reduced matrix Z_r = (C^JM)^H Z C^MJ (paper Sec. III-C,
 * outer CBFM equation): rows [J-test CBFs of cells 1..M ; M-test CBFs],
 * columns [M-trial CBFs ; J-trial CBFs], each group cell after cell.
 * The PMCHWT fill is computed inside and projected on the matrix cores; Z
 * is held only in stream-ordered scratch, one panel of cells at a time.  By
 * reciprocity of the Galerkin blocks (each operator's block of a triangle
 * pair is the transpose of the reversed pair's under the regular rule) a
 * panel fills its test triangles against its own and the later cells'
 * source triangles only, and the blocks of the later cells' rows against
 * its columns come from the transposes (near pairs are computed in both
 * orientations).  precision: CBFM_FP64, CBFM_FP32
 * (fill as in cbfm_fill_pmchwt, projection in double) or the mixed forms
 * CBFM_MIXED_FP32 / CBFM_MIXED_BF16 / CBFM_MIXED_BF16X3 (float fill, float
 * panel, FP32, BF16 or split-BF16 matrix-core projection with FP32
 * accumulation; Z_r still stored double).  With CBFs built on a mesh of
 * translated copies of one cell (FP64), the block of two cells depends only
 * on their offset: one block is filled and projected per distinct offset
 * and copied to the pairs sharing it.
 *   Zr_dev  N_CBF x N_CBF double2, row-major, ldz >= N_CBF                 */
cbfm_status cbfm_project(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, int32_t precision,
                         void* Zr_dev, int64_t ldz, void* stream);

/* cbfm_project_ex: cbfm_project with an explicit scratch budget for the row
 * panels (paper Sec. III-C, outer CBFM equation; the same Z_r).  Cells are
 * grouped into panels of consecutive cells (on meshes of 4,096 triangles
 * or more at most an eighth of the cells each) whose fill and projection
 * scratch fits panel_bytes (a panel always
 * holds at least one cell; on a mesh of translated cells, groups of cell
 * offsets).  panel_bytes = 0 takes
 * the default of cbfm_project: a quarter of the free device memory, at most
 * 32 GiB.  npanels_host (or NULL) receives the number of panels used.     */
cbfm_status cbfm_project_ex(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, int32_t precision,
                            void* Zr_dev, int64_t ldz, int64_t panel_bytes, int32_t* npanels_host,
                            void* stream);

/* cbfm_project_batch: Z_r of `count` scatterers of any sizes and media at
 * once (as cbfm_project for each): the regular-pair fills of all of them run
 * in one persistent launch over (scatterer, test triangle, source tile)
 * work items, the projection GEMMs of all of them in two batched launches.
 * Scatterers are grouped while their whole-Z scratch fits a quarter of the
 * free device memory; one that does not fit goes through cbfm_project's
 * panels.  meshes, media, cbfs, Zr, ldz: arrays of `count` entries.        */
cbfm_status cbfm_project_batch(int32_t count, const cbfm_mesh* meshes, const cbfm_medium* media,
                               const cbfm_cbf* cbfs, int32_t precision, void* const* Zr_dev,
                               const int64_t* ldz, void* stream);

/* CMP modes: the exact inverse (the plain path), or the paper's inexact
   inner solve of G^CBF j_CBF = y by GMRES with the diagonal preconditioner
   D^CBF = diag(1 / [G^CBF]_ii) (Sec. III-C, the paragraph on D^CBF; the
   numerical section uses the allowance 1e-5). */
enum { CBFM_CMP_EXACT = 0, CBFM_CMP_INNER_GMRES = 1 };

/* ----------------------------------------------------------------- CMP ---
 * cbfm_cmp_apply: x = (G^CBF)^{-1} y with G^CBF = (C^JM)^H G_ffff C^MJ
 * (paper Sec. III-C, CBF Gram matrix and inner CBFM equation), exact:
 * G^CBF = blkdiag(-B^H, B) with B = (C^M)^H G C^J, and B^{-1} is formed on
 * first use by in-place Gauss-Jordan elimination (cell by cell when no
 * triangle carries RWGs of two cells) and kept in the cbfm_cbf handle.
 * Returns CBFM_E_RANK if B has no nonzero pivot.
 *   y_dev, x_dev  nrhs x N_CBF double2, vector after vector (may alias)    */
cbfm_status cbfm_cmp_apply(cbfm_cbf c, int64_t nrhs, const void* y_dev, void* x_dev,
                           void* stream);

/* cbfm_cmp_apply_ex: as cbfm_cmp_apply with mode CBFM_CMP_EXACT; with
 * CBFM_CMP_INNER_GMRES, x is the GMRES solution of G^CBF x = y with the
 * right preconditioner D^CBF (x0 = 0, restarted every min(2 sum L, 500)
 * iterations, at most 4 x 2 sum L), stopped at the relative residual
 * inner_tol (0: 1e-5); the operator G^CBF D^CBF (2 sum L square) is formed
 * on the first such call and kept in the handle.  Synchronises the stream
 * in the inexact mode.                                                     */
cbfm_status cbfm_cmp_apply_ex(cbfm_cbf c, int64_t nrhs, const void* y_dev, void* x_dev, int32_t mode,
                              double inner_tol, void* stream);

/* --------------------------------------------------------------- solve ---
 * cbfm_solve: for each incidence, v_r = (C^JM)^H v, right-preconditioned
 * GMRES on Z_r (G^CBF)^{-1} y = v_r (x0 = 0, restart, stop at relative
 * residual <= tol), j_CBF = (G^CBF)^{-1} y, j = C^MJ j_CBF (paper Sec. III-C
 * outer/inner equations and the current reconstruction), then RCS (paper's
 * monostatic definition, Knott): with N = int J e^{jk0 r.r'}, L = int M
 * e^{jk0 r.r'}, sigma = k0^2/(4 pi) |eta0 N_perp - r x L|^2 (|E0| = 1).
 *   inc_host   nrhs x 6 (k, p)
 *   Zr_dev     from cbfm_project, ldz
 *   j_dev      nrhs x 2ne double2 output [alpha^M ; alpha^J] (or NULL)
 *   iters_host, relres_host   nrhs outputs (or NULL)
 *   dirs_host  ndir x 3 unit observation directions -> rcs_host nrhs x ndir
 *              total bistatic sigma; NULL -> monostatic co-polarised sigma
 *              (direction -k, component along p), rcs_host nrhs
 *   use_cmp    1: right preconditioner (G^CBF)^{-1}; 0: none (y = j_CBF),
 *              the K-diagonal CBFM without the CMP; 2: the T-diagonal
 *              CBFM of Sec. IV-A, (C^JM)^H Z_t C^JM j_t^CBF = v_r with Z_t
 *              the MoM arrangement (Z with its column blocks swapped), that
 *              is Z_r with its two column halves swapped, no preconditioner
 * Synchronises the stream.  CBFM_E_NOCONV if, for some RHS, the relative
 * residual of the preconditioned system recomputed in double at the end
 * (relres_host) exceeds tol; every cycle starts from that true residual, so
 * this happens only when max_iter is reached.                             */
typedef struct {
  double tol;
  int32_t max_iter;   /* Arnoldi iterations over all cycles                */
  int32_t restart;    /* cycle length                                      */
  int32_t use_cmp;
  int32_t inner_fp32; /* 1: mixed form -- Krylov basis and operator in     */
                      /* float, each cycle started from the residual       */
                      /* b - A x formed in double (iterative refinement)   */
                      /* and stopped once it has reduced it by inner_tol   */
  double inner_tol;   /* mixed and compressed-basis forms; 0 -> 1e-6        */
  int32_t use_graph;  /* 1: Arnoldi iterations in chunks of four captured   */
                      /* once per cycle into a HIP graph and replayed      */
  int32_t cmp_mode;   /* with use_cmp 1: CBFM_CMP_EXACT, or               */
                      /* CBFM_CMP_INNER_GMRES -- the paper's inexact      */
                      /* (G^CBF)^{-1} (see cbfm_cmp_apply_ex), inside     */
                      /* flexible GMRES (the preconditioner changes from  */
                      /* one iteration to the next, so the iterate is     */
                      /* built from the preconditioned vectors); double   */
                      /* cycles, no graphs                                */
  double cmp_inner_tol; /* inexact CMP allowance; 0 -> 1e-5                */
  int32_t basis_fp32; /* 1: compressed-basis form -- double arithmetic    */
                      /* (operator, work vector, Hessenberg, residuals)   */
                      /* with the Krylov basis stored in float, which     */
                      /* halves the bytes of the Arnoldi passes; the      */
                      /* Arnoldi relation then holds to float rounding,   */
                      /* so each cycle stops once it has reduced the      */
                      /* residual b - A x (formed in double) by inner_tol */
                      /* (or reached tol) and the next starts from it.    */
                      /* Not with inner_fp32 or CBFM_CMP_INNER_GMRES      */
                      /* (CBFM_E_ARG).  cbfm_mom_solve takes it with an   */
                      /* FP64 operator (ignored for FP32, whose cycles    */
                      /* are float); cbfm_solve_matfree rejects it.       */
  int32_t sstep;      /* 4 or 8: s-step (communication-avoiding) cycles of */
                      /* the same GMRES -- per block of sstep iterations, */
                      /* a Newton basis (shifts: Ritz values of a first   */
                      /* plain cycle of sstep + 1 iterations, Leja order) */
                      /* by sstep matrix-vector products, two block       */
                      /* Gram-Schmidt passes and two Cholesky QR passes,  */
                      /* and the Hessenberg columns rebuilt from their    */
                      /* coefficients: the basis is read 4 times per      */
                      /* block instead of twice per iteration.  After a   */
                      /* Cholesky breakdown the solve continues with      */
                      /* plain cycles, and so do the last iterations when */
                      /* fewer than sstep are left before max_iter (the   */
                      /* count stops at max_iter exactly).  0: plain      */
                      /* cycles.  Not with                                */
                      /* inner_fp32, basis_fp32, use_graph or             */
                      /* CBFM_CMP_INNER_GMRES (CBFM_E_ARG); cbfm_solve    */
                      /* only.                                            */
  int32_t block;      /* block GMRES: 2..32 -- the right-hand sides, in    */
                      /* groups of that many, share one Krylov space      */
                      /* built from the block of their residuals; 1 --    */
                      /* groups of up to 32, fewer when N_CBF / 33 is     */
                      /* smaller (so that a cycle holds 32 block          */
                      /* iterations: shorter restarted cycles stagnate);  */
                      /* 0 -- off.  Each iterate                          */
                      /* minimises its own residual over all of it (the   */
                      /* outer equation of Sec. III-C for many            */
                      /* incidences at once).  Each block iteration       */
                      /* applies the operator to the group's last basis   */
                      /* block; two block Gram-Schmidt passes, each       */
                      /* followed by a Cholesky QR of the block on a Gram */
                      /* matrix summed and factored in double-double with */
                      /* diagonal pivoting (dependent directions, below   */
                      /* 1e-13 of the block's largest, are replaced by    */
                      /* random vectors outside the Arnoldi relation);    */
                      /* the block Hessenberg matrix reduced by           */
                      /* Householder QR as it grows.  restart and         */
                      /* max_iter count block iterations (a cycle holds   */
                      /* at most N_CBF / group - 1) and iters_host        */
                      /* returns them.  Not with inner_fp32, basis_fp32,  */
                      /* use_graph, sstep or CBFM_CMP_INNER_GMRES         */
                      /* (CBFM_E_ARG); cbfm_solve, and cbfm_mom_solve     */
                      /* with an FP64 operator.                           */
} cbfm_solver_params;

cbfm_status cbfm_solve(cbfm_mesh m, const cbfm_medium* med, cbfm_cbf c, const void* Zr_dev,
                       int64_t ldz, const double* inc_host, int64_t nrhs,
                       const cbfm_solver_params* prm, void* j_dev, int32_t* iters_host,
                       double* relres_host, const double* dirs_host, int64_t ndir,
                       double* rcs_host, void* stream);

/* ---------------------------------------------------- the whole system ---
 * A cbfm_mom holds the whole discretised PMCHWT system of a mesh and medium
 * on the device, in the MoM arrangement of the numerical section (Sec. IV)
 * with its diagonal preconditioner:
 *   A = Z_t D^{-1},  Z_t = [[-TE, K], [K, TH]] acting on j_t = [alpha^J; alpha^M],
 *   D = diag(Z_t),
 * where the paper tests the T blocks with Buffa-Christiansen functions and
 * this library with the RWG functions themselves (the BC basis is not
 * built), so Z_t is the matrix Z of the conventions above with its two
 * column blocks swapped.  A is (2 ne)^2 complex numbers: 16 bytes each in
 * FP64, 8 in FP32 (regular pairs filled in float, near pairs in double):
 * for 29,952 RWGs 57 GB or 29 GB of device memory.
 *
 * cbfm_mom_build: fill and store A and D.  precision CBFM_FP64 or
 *   CBFM_FP32.  panel_bytes: scratch budget of the fill's row panels (0: a
 *   quarter of the free device memory, at most 32 GiB).  Synchronises the
 *   stream.  The mesh must outlive the handle.  CBFM_E_NOMEM if A does not
 *   fit.                                                                    */
cbfm_status cbfm_mom_build(cbfm_mesh m, const cbfm_medium* med, int32_t precision, int64_t panel_bytes,
                           void* stream, cbfm_mom* out);
/* The order n = 2 ne and the precision of A (each may be NULL).          */
cbfm_status cbfm_mom_info(cbfm_mom o, int64_t* n, int32_t* precision);
/* Copy rows row0 .. row0 + nrow - 1 of A into A_dev (row stride ld >= n,
   double2 for FP64, float2 for FP32) and D into d_dev (n double2); either
   may be NULL.  A's rows are [E-tests; H-tests] and its columns [alpha^J;
   alpha^M], each half with the RWGs in the library's cell order (canonical
   edges stably sorted by cell), not the canonical one.  Enqueued on the
   stream.                                                                  */
cbfm_status cbfm_mom_export(cbfm_mom o, int64_t row0, int64_t nrow, void* A_dev, int64_t ld, void* d_dev,
                            void* stream);
void cbfm_mom_free(cbfm_mom o);

/* cbfm_mom_solve: the MoM baseline of Sec. IV -- right-preconditioned GMRES
 * on Z_t D^{-1} u = v from u = 0 (Z_t D^{-1} = A), j_t = D^{-1} u, for every
 * incidence; the residual ||v - Z j|| / ||v|| is what tol bounds.  Outputs
 * as cbfm_solve: j_dev (nrhs x 2ne, canonical order, [alpha^M; alpha^J]),
 * iters, relres (true relative residual), RCS.  Fields of prm: tol,
 * max_iter, restart, inner_fp32 / inner_tol (float Krylov cycles refined
 * against the double residual; an FP32 operator always runs float cycles
 * and forms its residual in float, so tolerances below about 1e-6 are out
 * of its reach), use_graph; use_cmp is ignored.  CBFM_E_NOCONV as
 * cbfm_solve.  Synchronises the stream.                                    */
cbfm_status cbfm_mom_solve(cbfm_mom o, const double* inc_host, int64_t nrhs, const cbfm_solver_params* prm,
                           void* j_dev, int32_t* iters_host, double* relres_host, const double* dirs_host,
                           int64_t ndir, double* rcs_host, void* stream);

/* cbfm_build_ipcbf: improved primary CBFs by the GMRES version of Sec.
 * III-A: each of the n_gen generating plane waves is solved on the whole
 * scatterer as in cbfm_mom_solve, to the loose relative residual delta_r
 * (full GMRES unless restart > 0); cell m keeps the rows of its RWGs,
 * J^M_m and J^J_m (N_m x n_gen), and the sets are orthogonalised exactly as
 * in cbfm_build_cbf (Sec. III-B: G'_m, SVD, truncation at delta_svd, at
 * most max_L if > 0).  iters_host / relres_host (n_gen each, or NULL): the
 * iterations and true residual of every wave.  CBFM_E_NOCONV (no handle)
 * if a wave does not reach delta_r within max_iter, CBFM_E_RANK as
 * cbfm_build_cbf.  The CBF handle belongs to the operator's mesh; the CMP
 * inverse is queued as after cbfm_build_cbf.  Synchronises the stream.    */
typedef struct {
  const double* gen_host; /* n_gen x 6 (k, p) generating plane waves */
  int32_t n_gen;
  double delta_r;         /* GMRES residual allowance, in (0, 1)     */
  double delta_svd;
  int32_t max_L;          /* 0 = no cap                              */
  int32_t max_iter;
  int32_t restart;        /* 0 = max_iter (full GMRES)               */
  int32_t block;          /* 0: one Krylov space per wave; 1, 2..32:
                             block GMRES as cbfm_solver_params.block
                             (the waves share a Krylov space per group;
                             max_iter, restart and iters_host count
                             block iterations)                       */
} cbfm_ipcbf_params;
cbfm_status cbfm_build_ipcbf(cbfm_mom o, const cbfm_ipcbf_params* prm, void* stream, cbfm_cbf* out,
                             int32_t* iters_host, double* relres_host);

/* cbfm_solve_matfree: cbfm_solve (use_cmp 0 or 1) with the reduced
 * operator applied without forming Z_r (Sec. III-C, the remark after the
 * current reconstruction: the products with C^MJ, C^JM and G^CBF are cheap
 * and the one with Z is the expensive one): every GMRES product computes
 * (C^JM)^H Z C^MJ (G^CBF)^{-1} y from the stored operator, Z u = A D P^T u
 * with P^T swapping the halves of u.  Double Krylov cycles only
 * (inner_fp32 = use_graph = 0).  Outputs as cbfm_solve.                    */
cbfm_status cbfm_solve_matfree(cbfm_mom o, cbfm_cbf c, const double* inc_host, int64_t nrhs,
                               const cbfm_solver_params* prm, void* j_dev, int32_t* iters_host,
                               double* relres_host, const double* dirs_host, int64_t ndir, double* rcs_host,
                               void* stream);

/* ------------------------------------------------------------- serving ---
 * A request server for scattering solves of mixed size (the whole path of a
 * request: mesh, CBF build, fill fused with the projection, CMP-GMRES and
 * monostatic RCS, as the calls above).  `slots` worker threads, each with
 * its own HIP stream on the current device, take requests in arrival order,
 * first fit: a request is admitted when its estimated device footprint fits
 * in what the budget leaves beside the requests running and the resident
 * scatterers (which are evicted, least recently used first, while unused),
 * or alone on an idle server.  Requests that arrive while others run are
 * admitted as slots and memory free up, and their GPU work overlaps.
 * Requests with the same nonzero scatterer_key share one resident mesh, CBF
 * set and Z_r (built by the first; the caller guarantees that equal keys
 * mean equal geometry, cells, medium, waves, delta_svd and precision).
 * All inputs are copied at submission.                                     */
typedef struct cbfm_server_s* cbfm_server;

typedef struct {
  const double* xyz_host;       /* nv x 3                                   */
  int64_t nv;
  const int32_t* tri_host;      /* nt x 3                                   */
  int64_t nt;
  const int32_t* edge_block;    /* per canonical edge, or NULL (one cell)   */
  int32_t nblocks;
  cbfm_medium medium;
  const double* gen_host;       /* n_gen x 6 generating plane waves         */
  int32_t n_gen;
  double delta_svd;
  int32_t precision;            /* projection precision (cbfm_precision)    */
  const double* inc_host;       /* nrhs x 6 incidences                      */
  int64_t nrhs;
  double tol;                   /* GMRES relative residual                  */
  int32_t max_iter;             /* 0: 3000                                  */
  int32_t restart;              /* 0: min(N_CBF, 1000)                      */
  int32_t inner_fp32;           /* 1: float Krylov cycles refined against
                                   the double residual (cbfm_solve's mixed
                                   form, inner_tol 0)                       */
  uint64_t scatterer_key;       /* 0: nothing kept after the request        */
} cbfm_request;

/* Estimated peak device bytes of a request (CBF build, fill + projection
   panels of at most 1 GiB unless one cell needs more, Z_r and the GMRES
   workspace), as the server uses it for admission.                        */
cbfm_status cbfm_request_footprint(const cbfm_request* req, int64_t* bytes);

cbfm_status cbfm_server_create(int32_t slots, int64_t budget_bytes, cbfm_server* out);
/* Queue a request; *ticket identifies it.  Never blocks on the GPU.        */
cbfm_status cbfm_server_submit(cbfm_server srv, const cbfm_request* req, int64_t* ticket);
/* Wait for a request and release it: rcs_host (nrhs monostatic sigma),
   iters_host (nrhs), times_host (3: submitted, started, finished, seconds
   on the server's clock); each may be NULL.  Returns the request's status
   (its message through cbfm_last_error).                                  */
cbfm_status cbfm_server_wait(cbfm_server srv, int64_t ticket, double* rcs_host, int32_t* iters_host,
                             double* times_host);
/* Peak device bytes admitted (running requests plus resident scatterers),
   the most requests that ran at once, resident scatterers now.            */
cbfm_status cbfm_server_stats(cbfm_server srv, int64_t* peak_bytes, int32_t* max_running,
                              int32_t* resident);
/* Waits for every queued request, stops the workers, frees residents.    */
void cbfm_server_destroy(cbfm_server srv);

#ifdef __cplusplus
}
#endif

#endif /* CBFM_H */
