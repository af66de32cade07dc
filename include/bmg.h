/*
 * bmg.h - C ABI of the MI355X bootstrap multigrid (BMG) eigensolver.
 *
 * Problem (paper: Brannick & Cao, "A Bootstrap Multigrid Eigensolver",
 * Sec. 2.2, eq. pb-eig-fea): on a closed surface Gamma approximated by flat
 * triangles whose vertices lie on Gamma (Sec. 2.1), find the eigenpairs of the
 * P1 surface-FEM pencil  A u = lambda M u  (A: stiffness, M: consistent mass),
 * with M-orthonormal eigenvectors (Sec. 2.1).  The library computes the k pairs
 * whose eigenvalues are nearest a shift sigma (Alg. 2, step 2 and Remark 4.1)
 * with the bootstrap multigrid cycle of Alg. 2/3: a relaxation cycle for the
 * shifted source problem (eq. pb-f-aux-mat, Remark 3.2) on a block of test
 * vectors, geometric prolongation / restriction between uniformly refined
 * meshes with projected midpoints (Sec. 3, eq. proj-1), and a Rayleigh-Ritz
 * step in the coarse space enriched with the block (eq. pb-c-aux-mat).
 *
 * Conventions shared by every entry point:
 *   - Every function returns BMG_OK (0) or a negative bmg_status.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory of the current device (e.g. torch.cuda tensors).
 *   - Blocks of vectors on the device are interleaved row-major [N][m]
 *     (vertex-major: the m values of one vertex are contiguous).
 *   - A `stream` argument is a hipStream_t passed as void*; NULL means the
 *     default (null) stream.  Work is enqueued on it in order.
 *   - The library never keeps a caller pointer after a call returns.
 *   - Errors: BMG_EINVAL for invalid arguments (nothing is enqueued),
 *     BMG_EDEVICE for a HIP runtime error (bmg_last_error() gives its text),
 *     BMG_ENOMEM when a device allocation fails.
 */
#ifndef BMG_H
#define BMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BMG_OK = 0,
  BMG_EINVAL = -1,
  BMG_ENOMEM = -2,
  BMG_EDEVICE = -3,
  BMG_ENOCONV = -4,
  BMG_EBUSY = -5,
  BMG_ECANCELED = -6
} bmg_status;

typedef enum {
  BMG_SPHERE = 0,    /* regular icosahedron inscribed in the unit sphere      */
  BMG_ELLIPSOID = 1, /* unit-sphere hierarchy mapped by x -> (a0 x, a1 y, a2 z) */
  BMG_TORUS = 2,     /* nu x nv parametric grid of the torus (R, r)            */
  BMG_CUSTOM = 3     /* caller's coarse mesh and projection onto Gamma         */
} bmg_surface_kind;

/* Description of the surface and of its coarsest triangulation (Sec. 2.1:
 * vertices on Gamma; Sec. 3: refinement moves midpoints onto Gamma).
 * Unused fields are ignored for the built-in kinds. */
typedef struct {
  int32_t kind;            /* bmg_surface_kind */
  double axes[3];          /* BMG_ELLIPSOID semi-axes (a0, a1, a2) > 0 */
  double R, r;             /* BMG_TORUS radii, R > r > 0 */
  int32_t nu, nv;          /* BMG_TORUS grid, nu >= 3, nv >= 3 (benchmark: 64 x 32) */
  int32_t n_vert, n_tri;   /* BMG_CUSTOM coarse mesh sizes */
  const double* xyz;       /* BMG_CUSTOM host [n_vert][3], copied during the call */
  const int32_t* tri;      /* BMG_CUSTOM host [n_tri][3], outward oriented, copied */
  /* BMG_CUSTOM projection onto Gamma, called on each new midpoint (in place);
   * NULL keeps the flat midpoint.  Called only during bmg_build_hierarchy. */
  void (*project)(double p[3], void* ctx);
  void* ctx;
} bmg_surface_desc;

typedef struct bmg_hierarchy bmg_hierarchy; /* opaque; device-resident after build */

/* Build levels 0..n_refine (Sec. 3 uniform refinement with projected
 * midpoints; Sec. 2.2 P1 assembly of A_l, M_l in FP64 with FP32 copies; vertex
 * colouring; parent tables of the prolongation of eq. proj-1; the level-0
 * generalized eigendecomposition of Alg. 2 step 1) and upload it to the
 * current device on `stream`.  The call returns after the upload completes.
 * Numbering: coarse edges (a<b) in lexicographic order, the midpoint of edge
 * e is vertex N_{l-1}+e; triangle (a,b,c) -> (a,ab,ca),(ab,b,bc),(ca,bc,c),
 * (ab,bc,ca).
 * Errors: BMG_EINVAL for a NULL/ill-formed descriptor, n_refine outside
 * [0, 10], a custom mesh that is not a closed, consistently oriented
 * 2-manifold (every directed edge once, its reverse once), a vertex valence
 * above 30, or a coarse mesh with more than 4096 vertices.  The level-0
 * eigendecomposition runs on the host (Jacobi) for coarse meshes of up to 1024
 * vertices and with rocSOLVER's dsygvd on the device above that (the 64 x 32
 * torus grid has 2048).
 * Ownership: *out belongs to the caller until bmg_free_hierarchy. */
int bmg_build_hierarchy(const bmg_surface_desc* desc, int32_t n_refine, void* stream,
                        bmg_hierarchy** out);

/* The same construction without any device work (no GPU needed): meshes,
 * matrices, colouring, parent tables and the level-0 eigendecomposition are
 * built on the host for inspection with bmg_hierarchy_info/_export.  Such a
 * hierarchy is rejected by bmg_solve and bmg_apply (BMG_EINVAL).  Coarse
 * meshes are limited to 1024 vertices here (BMG_EINVAL above). */
int bmg_build_hierarchy_host(const bmg_surface_desc* desc, int32_t n_refine, bmg_hierarchy** out);

void bmg_free_hierarchy(bmg_hierarchy* h);

typedef struct {
  int32_t n_levels;      /* n_refine + 1 */
  int32_t level;         /* the level described below */
  int64_t n_vert;        /* N_l */
  int64_t n_tri;         /* triangles of level l */
  int64_t nnz;           /* nonzeros of A_l (= of M_l; same pattern) */
  int32_t ell_width;     /* padded row width of the ELL storage */
  int32_t n_colours;     /* colours of the Gauss-Seidel colouring */
  double area;           /* |Gamma_h| = sum of triangle areas = 1^T M_l 1 */
  int64_t device_bytes;  /* device memory held for this level */
} bmg_level_info;

/* Sizes of one level (0 <= level < n_levels).  BMG_EINVAL on a bad level. */
int bmg_hierarchy_info(const bmg_hierarchy* h, int32_t level, bmg_level_info* out);

typedef enum {
  BMG_EXPORT_XYZ = 0,      /* double [N][3] vertex coordinates                     */
  BMG_EXPORT_TRI = 1,      /* int32  [F][3] triangles                              */
  BMG_EXPORT_PARENTS = 2,  /* int32  [N_l - N_{l-1}][2] parents (a<b) of new vertices (l >= 1) */
  BMG_EXPORT_ELL_COLS = 3, /* int32  [N][W] column indices; entry 0 is the diagonal; padding repeats the row index */
  BMG_EXPORT_ELL_A = 4,    /* double [N][W] values of A_l (padding 0)              */
  BMG_EXPORT_ELL_M = 5,    /* double [N][W] values of M_l (padding 0)              */
  BMG_EXPORT_COLOURS = 6,  /* int32  [N] colour of each vertex                      */
  BMG_EXPORT_LUMPED = 7,   /* double [N] row sums of M_l                            */
  BMG_EXPORT_COARSE_EIG = 8, /* level 0 only: double [N_0] eigenvalues then [N_0][N_0]
                               row-major M_0-orthonormal eigenvectors (column j = pair j) */
  BMG_EXPORT_COLOURS2 = 9   /* int32  [N] colour of each vertex in the distance-2
                               colouring of the Kaczmarz smoother                    */
} bmg_export_what;

/* Copy one host-side array of a level into `host_out` (capacity in bytes).
 * For inspection and for checking the hierarchy against an independent
 * implementation.  BMG_EINVAL if the level/what is invalid or the capacity is
 * too small; *bytes_needed (nullable) receives the size in every case. */
int bmg_hierarchy_export(const bmg_hierarchy* h, int32_t level, int32_t what, void* host_out,
                         int64_t capacity, int64_t* bytes_needed);

/* ---------------------------------------------------------------- solve --- */

/* Smoothers of the correction cycle, on S_l = A_l - sigma_l M_l.
 * GS: multicolour symmetric Gauss-Seidel (greedy colouring, colours up then
 *   down).  JACOBI: weighted Jacobi with opts.omega.
 * KACZMARZ: multicolour symmetric Kaczmarz relaxation (Sec. 5.3, the paper's
 *   smoother for the shifted, indefinite source problems): for each row i,
 *   x <- x + ((f_i - s_i^T x) / |s_i|^2) s_i, the projection onto row i's
 *   hyperplane (weight 1; opts.omega is not used).  Rows of one colour of a
 *   greedy distance-2 colouring (no two rows of a colour share a column) are
 *   projected at once; colours up, then down.  It converges for any
 *   nonsingular S (it is Gauss-Seidel on S S^T) but damps more slowly than
 *   GS where GS converges. */
typedef enum { BMG_SMOOTH_GS = 0, BMG_SMOOTH_JACOBI = 1, BMG_SMOOTH_KACZMARZ = 2 } bmg_smoother;
typedef enum { BMG_FP64 = 0, BMG_MIXED = 1 } bmg_precision;

/* Iteration schemes.
 * BMG_SCHEME_ENRICHED: fixed shift; the n_c level-0 eigenvectors nearest sigma,
 *   prolongated to level L, stay in every Rayleigh-Ritz step beside the block
 *   (the enriched coarse space V_H + X_h of Alg. 2 step 4); the correction's
 *   coarsest level follows the Weyl rule of l_c below.  Meant for the lower end
 *   of the spectrum.
 * BMG_SCHEME_SHIFTED: interior shifts (Sec. 5.2, Remark 4.1, Alg. 3 step 4,
 *   Alg. 4 step 1).  All eigenpairs of one coarse level l_c are computed once
 *   per hierarchy (dense, kept with it); l_c is the coarsest level with
 *   sigma^2 h_max,l^2 |Gamma_h| / m <= 60 (h_max,l its longest edge: its
 *   eigenvalues near sigma are then within a few block windows of the fine
 *   ones) and N_l >= 2 m, capped at 12288 vertices (m is then raised when it
 *   was not given, at most 96).  The block
 *   starts from the m level-l_c eigenvectors nearest the level's shift,
 *   prolongated and relaxed once on the source problem of eq. pb-f-aux-mat;
 *   each level l_c <= l < L of the correction uses A_l - sigma_l M_l with the
 *   adaptive shift sigma_l = sigma + mean over the block of (the Rayleigh
 *   quotient of its values at the level-l vertices on level l - its Ritz
 *   value), recomputed before every correction (and once between two starts);
 *   the coarse solve at l_c is the truncated spectral inverse (modes within
 *   1e-2 max(1, |sigma|) of sigma_lc dropped); the Ritz step uses the span of
 *   the block alone.  seed and n_c are not used.
 * BMG_SCHEME_AUTO: SHIFTED when sigma > 0, else ENRICHED. */
typedef enum { BMG_SCHEME_AUTO = 0, BMG_SCHEME_ENRICHED = 1, BMG_SCHEME_SHIFTED = 2 } bmg_scheme;

typedef struct {
  int32_t m;          /* test vectors; 0 -> 4 ceil(1.25 k / 4) (sigma = 0) or
                         4 ceil(1.5 k / 4) (sigma != 0), raised by the
                         shifted scheme's coarse-level cap, then (bmg_solve
                         only) widened to whole clusters: until the first
                         eigenvalue of a coarse level left out of the block
                         is 1.25 times as far from sigma as the k-th (Sec. 4,
                         the choice of Lambda), at most 96 - n_c and half the
                         finest level's rows; a multiple of 4 */
  int32_t nu1, nu2;   /* pre- and post-smoothing sweeps per level (2, 2) */
  int32_t smoother;   /* bmg_smoother: multicolour symmetric Gauss-Seidel (colours
                         ascending before, descending after the coarse correction)
                         or weighted Jacobi with D = diag(A_l - sigma M_l) */
  int32_t precision;  /* bmg_precision: BMG_MIXED runs the correction cycle in FP32
                         (values and accumulation); residuals, Gram matrices, the
                         Ritz problem and the iterate stay FP64 */
  int32_t max_cycles; /* 200 */
  int32_t n_c;        /* level-0 eigenvectors in the enrichment; 0 -> min(N_0, 32)
                         rounded down to even (ENRICHED scheme only) */
  int32_t l_c;        /* coarsest level of the correction cycle; -1 -> ENRICHED:
                         the coarsest l with N_l >= 8 |Gamma_h| sigma / (4 pi);
                         SHIFTED: the rule of bmg_scheme */
  double omega;       /* Jacobi weight (default 0.85) */
  double angle_tol;   /* Davis-Kahan stopping bound on rho_i / delta_i (1e-7) */
  uint64_t seed;      /* test vectors: element (i,j) ~ N(0,1) from SplitMix64
                         counters 2c, 2c+1 with c = i m + j, Box-Muller */
  const double* initial_block; /* optional host [N_L][m] block replacing the seeded one */
  int32_t timed_kernel; /* bmg_kernel_class to bracket with HIP events on `stream`,
                           or -1; see bmg_solve_stats.  class + 256 (l + 1) times
                           a V-cycle class on level l only */
  int32_t scheme;       /* bmg_scheme (BMG_SCHEME_AUTO) */
  /* Level ramp (BFMG, Alg. 4): with ramp_cycles > 0 the solve starts on level
   * l0 from that level's exact eigenpairs nearest sigma (Alg. 4 step 1; all
   * its pairs are computed once per hierarchy and level, at most 12288
   * vertices) and visits every level l0 < l < L with the block prolongated
   * from the level below, a Rayleigh-Ritz step and ramp_cycles cycles of that
   * level's own BMG cycle (its finest level is l), before continuing on level L
   * as usual (max_cycles, certificate).  The k values nearest sigma after each
   * level go to stats->ramp_evals.  With max_cycles = ramp_cycles this is the
   * one-pass BFMG of the paper's Table 1 (every level gets the same number
   * of cycles; the solve then ends with BMG_ENOCONV unless the certificate
   * held).  ramp_level: l0 in [l_c, L], or -1 for the coarsest level at or
   * above l_c with at least 2 m vertices (BMG_EINVAL outside that range or
   * above 12288 vertices).  ramp_cycles at most 64.  seed and initial_block
   * are not used by a ramp; the Ritz warm start is off during the ramp. */
  int32_t ramp_cycles;  /* 0 */
  int32_t ramp_level;   /* -1 */
} bmg_solve_opts;

/* Kernel classes that bmg_solve can time.  EIGRES, SPMM_AM, GRAM, UPDATE and
 * RITZ run once per cycle on the finest level L; the V-cycle classes are timed
 * on every level that runs as multi-block kernels (the levels below those run
 * inside the one-workgroup LDS tail and are not counted).  Each class is one
 * kernel symbol, so its average launch time is comparable with a profiler's.
 * With the weighted-Jacobi smoother the cycle runs three fused kernels
 * (SMOOTH_PAIR, RESTRICT_RES, PROLONG_SMOOTH) in place of the zero-start
 * sweep, the first sweep, the residual, the restriction, the prolongation and
 * the first post-sweep.
 * Algorithmic bytes per launch at a level with n rows, nnz nonzeros (ELL rows
 * of width W), m block columns, b = 4 (mixed) or 8 (FP64) bytes per correction
 * value, n_prev rows on the next coarser level, N = N_L, nz = n_c + m:
 *   EIGRES    residual SpMM:  20 nnz + 8 N m (U) + b N m (R) + 8 N (D^-1)
 *   SPMM_AM   A and M SpMM:   20 nnz + 8 N m (U) + 16 N m (A U, M U); in a solve it
 *             runs only at set-up (the products with W_c); the cycle's products
 *             are formed inside the GRAM kernel
 *   SMOOTH    Jacobi: one sweep from a nonzero iterate:
 *             (4 + b) nnz + 3 b n m   (S and columns; x, f read; y written);
 *             Gauss-Seidel: one colour pass over n_k rows:
 *             (4 + b) W n_k + b m (n + 2 n_k)   (its rows of S; x read once;
 *             f read and x written on its rows)
 *   RESIDUAL  (4 + b) nnz + 3 b n m;   RESTRICT  b n m + b n_prev m + 4 n_prev RW;
 *   PROLONG   b n_prev m + 2 b n m + 8 (n - n_prev);
 *   SMOOTH_PAIR     (4 + b) nnz + 2 b n m            (f read, y written);
 *   RESTRICT_RES    (4 + b) nnz + 2 b n m + b n_prev m + 4 n_prev RW
 *                   (e, f read; the coarse right-hand side written);
 *   PROLONG_SMOOTH  (4 + b) nnz + 3 b n m + b n_prev m + 8 (n - n_prev)
 *                   (e, f read, y written; the coarse correction read);
 *   SMOOTH_ADD      (4 + b) nnz + 2 b n m + 16 n m   (the cycle's last Jacobi
 *                   sweep on the finest level: x, f read; its result added to
 *                   the FP64 iterate U, read and written);
 *   GRAM      fused A U, M U and Z^T [A U | M U]: 2 N (2 n_c m + m (m + 1))
 *             flops, the outputs the Ritz step needs (one triangle of each
 *             symmetric m x m block); the products' 20 nnz + 8 N nz bytes read;
 *   UPDATE    8 N nz + 8 N m bytes, 2 N nz m flops;   RITZ  one workgroup. */
typedef enum {
  BMG_K_EIGRES = 0, BMG_K_SPMM_AM = 1, BMG_K_SMOOTH = 2, BMG_K_RESIDUAL = 3,
  BMG_K_RESTRICT = 4, BMG_K_PROLONG = 5, BMG_K_GRAM = 6, BMG_K_UPDATE = 7, BMG_K_RITZ = 8,
  BMG_K_SMOOTH_PAIR = 9, BMG_K_RESTRICT_RES = 10, BMG_K_PROLONG_SMOOTH = 11,
  BMG_K_SMOOTH_ADD = 12
} bmg_kernel_class;

/* Fill *o with the defaults listed above. */
void bmg_solve_opts_default(bmg_solve_opts* o);

typedef struct {
  int32_t cycles;      /* correction + Ritz cycles performed */
  int32_t converged;   /* 1 if every returned pair met the certificate */
  int32_t m, n_c, l_c; /* values actually used */
  int32_t group_size;  /* requests solved together in the solve that produced this
                          result (bmg_solve_group; 1 for bmg_solve) */
  double t_solve_ms;   /* HIP-event time on `stream` from entry to output */
  double max_rho_over_delta; /* final max over returned pairs of rho_i / delta_i */
  double max_kato_temple;    /* final max of rho_i^2 / (delta_i max(|theta_i|, 1)) */
  double* rho;         /* nullable host [k]: rho_i = 2 ||r_i||_{D^-1} >= ||r_i||_{M^-1} */
  double* delta;       /* nullable host [k]: distance to the nearest Ritz value outside
                          the cluster of theta_i */
  double timed_kernel_ms;     /* summed HIP-event time of opts->timed_kernel launches */
  double timed_kernel_bytes;  /* summed algorithmic bytes (flops for GRAM/UPDATE) */
  int64_t timed_kernel_units; /* launches */
  int32_t ritz_sweeps_max;    /* most Jacobi sweeps of one Ritz step */
  int32_t ritz_fallbacks;     /* Ritz steps that needed SVQB instead of Cholesky */
  int32_t scheme;             /* bmg_scheme used (ENRICHED or SHIFTED) */
  int32_t reserved2;
  double coarse_eig_ms;       /* SHIFTED: wall time of the level-l_c eigensolve when it
                                 was built (never part of t_solve_ms) */
  double lc_shift;            /* SHIFTED: final adaptive shift of level l_c; else sigma */
  double* ramp_evals;         /* nullable host [n_levels][k]: with a level ramp, row l holds
                                 the k eigenvalue approximations nearest sigma (ascending)
                                 after level l (l0 <= l < L) and row L the returned ones;
                                 rows below l0 are not written */
  int32_t ramp_start;         /* l0 of the ramp, or -1 */
  int32_t reserved3;
} bmg_solve_stats;

/* The k eigenpairs of (A_L, M_L) nearest sigma on the finest level L.
 *   evals: host [k], ascending (unshifted lambda).
 *   evecs: NULL, or column-major [k][ld] (column j = eigenvector j, ld >= N_L),
 *          host memory if evecs_on_device == 0, device memory otherwise.
 *          Columns are M_L-orthonormal; the entry of largest magnitude of each
 *          column is positive (the lowest index on ties).
 * Stopping rule (the paper runs a fixed number of cycles; this certificate is
 * the library's reading): with r_i = A u_i - theta_i M u_i, rho_i = 2
 * ||r_i||_{D^-1} (D = lumped mass) and delta_i the distance from theta_i to the
 * nearest Ritz value outside its cluster (relative gap < 1e-2 joins a cluster),
 * stop when rho_i^2 / delta_i <= 0.1 tol max(|theta_i|, 1) and
 * rho_i / delta_i <= angle_tol for every returned pair.
 * Errors: BMG_EINVAL if k < 1, m < k, m % 4 != 0, m > N_L / 2, n_c + m > 96,
 * tol <= 0 or NaN, sigma not finite, an unknown scheme, or (SHIFTED) a level
 * l_c above 12288 vertices; BMG_ENOCONV when max_cycles is reached (evals,
 * evecs and stats still hold the current pairs) or when the Ritz step finds
 * fewer than m independent directions (evals and evecs are then not written);
 * BMG_ENOMEM.
 * The first SHIFTED solve on a hierarchy also computes the level-l_c
 * eigendecomposition, before t_solve_ms starts (its time is coarse_eig_ms).
 * The call blocks until the result is on the host (evals) / in evecs.
 * Concurrent calls on one hierarchy are allowed on different streams. */
int bmg_solve(bmg_hierarchy* h, int32_t k, double sigma, double tol, const bmg_solve_opts* opts,
              double* evals, double* evecs, int64_t ld, int32_t evecs_on_device, void* stream,
              bmg_solve_stats* stats);

/* One request of a grouped solve (bmg_solve_group): the arguments of one
 * bmg_solve call and its result. */
typedef struct {
  int32_t k;                  /* pairs wanted */
  double tol;                 /* as in bmg_solve */
  const bmg_solve_opts* opts; /* NULL: defaults; see bmg_solve_group for what must agree */
  double* evals;              /* out: host [k] */
  double* evecs;              /* out: NULL or column-major [k][ld], host or device memory */
  int64_t ld;
  int32_t evecs_on_device;
  int32_t status;             /* out: this request's bmg_status */
  bmg_solve_stats* stats;     /* nullable, as in bmg_solve (ramp_evals not written) */
} bmg_group_request;

/* Serving (growth pattern 5 of the hot path): n requests for eigenpairs of
 * the same hierarchy nearest the same sigma, solved together.  Their test
 * blocks are concatenated column-wise into one [N_L][sum m_i] block, so every
 * launch of the correction cycle (sweeps, residuals, transfers, the coarse
 * end) and of the eigen-residual runs once for all of them, and the whole
 * cycle is replayed as one HIP graph; the Gram, Rayleigh-Ritz and update steps
 * run per request on its column slice.  A request is certified, and its
 * output written, at the first cycle where its own pairs meet its tolerance,
 * exactly as in bmg_solve; the others continue.  Every column's arithmetic in
 * the cycle is the same as in a solo solve; the residual norms are summed in a
 * different grouping of rows, so a request's result equals its bmg_solve
 * result to rounding (and may take one cycle more or less).
 * Must agree across the group: the scheme (ENRICHED: sigma <= 0, or scheme
 * BMG_SCHEME_ENRICHED), precision, smoother, nu1, nu2, omega, n_c, l_c; no
 * initial_block or level ramp.  Per request: k, tol, m (sum of m at most 512),
 * seed, max_cycles, angle_tol.  Returns BMG_OK when every request converged,
 * else the first failing request's status (each request's own status is in
 * reqs[i].status); BMG_EINVAL (nothing run) when the group breaks the rules
 * above or a request is invalid for bmg_solve. */
int bmg_solve_group(bmg_hierarchy* h, double sigma, int32_t n, bmg_group_request* reqs,
                    const void* hip_stream);

/* ----------------------------------------------------------- estimator --- */

/* The a posteriori error estimator of eq. est-res (Sec. 5) for k eigenpairs
 * (evals[j], column j of evecs) of level `level`: per triangle T
 *   eta_T^2 = h_T^2 lambda^2 |u|^2_{L2(T)}
 *           + 1/2 sum_{e in dT} |e| |[grad u . mu_e]|^2_{L2(e)}
 *           + |B_h grad u|^2_{L2(T)},
 * eta(u) = (sum_T eta_T^2)^(1/2).  h_T: longest edge of T; the jump is the
 * sum of the two outward conormal derivatives across e (mu_e in the plane of
 * each triangle, normal to e); B_h = A_h - P_h, the geometric error of the
 * Dirichlet form under the lift onto the exact surface, is taken for the
 * sphere (radial lift: A_h = c P_h + t t^T / c with nu = x/|x|, c = nu . n_T,
 * t = nu - c n_T; edge-midpoint rule) and is 0 for other surfaces.
 *   evals: host [k];  evecs: device, column-major [k][ld] (the layout
 *     bmg_solve writes with evecs_on_device = 1), ld >= N_level.
 *   eta: host [k];  parts: nullable host [3][k] (the sums of the three terms);
 *   eta2_T: nullable device [F_level], sum over the k pairs of eta_T^2.
 * The level's triangles are uploaded on first use and kept with the
 * hierarchy.  Blocks until eta is on the host.  BMG_EINVAL, BMG_ENOMEM,
 * BMG_EDEVICE. */
int bmg_estimate(bmg_hierarchy* h, int32_t level, int32_t k, const double* evals, const double* evecs,
                 int64_t ld, double* eta, double* parts, double* eta2_T, void* stream);

/* ------------------------------------------------------------ two-grid --- */

/* The two-grid eigensolver with a spectral shift (Alg. 1) applied in a cascade
 * between neighbouring levels (Remark 3.1), the fine source problem of
 * eq. (pb-f-s) relaxed by Kaczmarz sweeps (Sec. 5.3; the remark after Alg. 1).
 * All eigenpairs of (A_H, M_H) on level_H are computed (at most 12288
 * vertices; kept with the hierarchy); the pairs idx (host [n], indices into
 * that ascending spectrum) are followed.  On each level k = level_H + 1..top,
 * for every pair c: u = P u_c, then nu multicolour Kaczmarz sweeps
 * (alternating directions, forward first; FP64) on
 *   (A_k - theta_c M_k) x = M_k u   from x = u,
 * theta_c the pair's value on level k - 1 (on level_H its coarse eigenvalue;
 * the fixed shift mu of Alg. 1 cancels, since the fine problem uses
 * mu + lambda_H); theta_c <- x^T A_k x / x^T M_k x and u_c <- x / |x|_M.
 * A coarse mesh too coarse for an eigenfunction's wavelength sends it to
 * another eigenvalue (the loss of spectra of Sec. 5.1).
 *   level_H in [0, L]; top in [level_H, L] or -1 for L; n in [1, 512];
 *   nu in [0, 64] (the paper uses 5).
 *   evals: host [L + 1][n]; row l (level_H <= l <= top) receives the values
 *     on level l in the order of idx; other rows are not written.
 *   evecs: NULL, or host column-major [n][N_top] (column c = pair c), unit
 *     M_top-norm.
 * Blocks until done; allocates its work buffers per call (4 N_top n doubles).
 * BMG_EINVAL on a bad argument, BMG_ENOMEM, BMG_EDEVICE. */
int bmg_two_grid(bmg_hierarchy* h, int32_t level_H, int32_t n, const int32_t* idx, int32_t top,
                 int32_t nu, double* evals, double* evecs, void* stream);

/* ------------------------------------------------ single-operator hook --- */

typedef enum {
  BMG_OP_A = 0,          /* y = A_l x                         (FP64)            */
  BMG_OP_M = 1,          /* y = M_l x                         (FP64)            */
  BMG_OP_SHIFTED = 2,    /* y = (A_l - sigma M_l) x           (dtype)           */
  BMG_OP_RESIDUAL = 3,   /* y = f - (A_l - sigma M_l) x       (dtype)           */
  BMG_OP_SMOOTH_FWD = 4, /* y <- one smoothing sweep of (A_l - sigma M_l) y = f,
                            colours ascending (GS) / one Jacobi step (dtype)      */
  BMG_OP_SMOOTH_BWD = 5, /* as above, colours descending                        */
  BMG_OP_RESTRICT = 6,   /* y [N_{l-1}][m] = P_l^T x [N_l][m]     (dtype)       */
  BMG_OP_PROLONG_ADD = 7,/* y [N_l][m] += P_l x [N_{l-1}][m]      (dtype)       */
  BMG_OP_VCYCLE = 8,     /* y = B_sigma x: one correction V-cycle from level l to
                            l_c (the solver's cycle, dtype)                      */
  BMG_OP_GAUSSIAN = 9,   /* y [N_l][m] = seeded N(0,1) block (FP64)             */
  BMG_OP_GRAM = 10,      /* y [m][m2] = x^T f with x [N_l][m], f [N_l][m2] (FP64,
                            matrix-core reduction over rows)                     */
  BMG_OP_SYEV = 11,      /* x: symmetric [m][m] FP64; y: [m] eigenvalues ascending
                            followed by [m][m] row-major orthonormal eigenvectors
                            (column j = vector j); one-workgroup Jacobi, m <= 96 */
  BMG_OP_EIGRES = 12,    /* y = A_l x - (M_l x) diag(f), f: device [m] doubles;
                            (FP64 in, output in dtype)                           */
  BMG_OP_UPDATE = 13,    /* y [N_l][m] <- [x | y] f in place: x [N_l][m2] (NULL if
                            m2 = 0), f = Y [m2 + m][m] row-major; the Ritz update
                            U <- [W_c, U'] Y (FP64, matrix cores, m2 + m <= 96)  */
  BMG_OP_GRAM_AM = 14,   /* y [m2 + m][2m] = [x | f]^T [A_l f | M_l f]: x [N_l][m2]
                            (NULL if m2 = 0), f [N_l][m], m even; the Gram blocks
                            of the enriched pencil with the products formed on the
                            fly (FP64, matrix cores, m2 + m <= 96)               */
  BMG_OP_COARSE_SOLVE = 15, /* y [N_l][m] = Phi diag(g) Phi^T x: the SHIFTED scheme's
                            coarse solve, the truncated spectral inverse of
                            A_l - sigma M_l (g = 1 / (lambda - sigma), 0 within
                            1e-2 max(1, |sigma|)); builds (and keeps) the level's
                            eigendecomposition on first use; N_l <= 12288, m a
                            multiple of 4 up to 96 (dtype)                       */
  BMG_OP_SHIFT_OFFSETS = 16 /* y [level + 1] doubles: y[j] = sigma + mean_c(x_c^T A_j
                            x_c / x_c^T M_j x_c - f_c) over the first N_j rows of
                            x, for l_c <= j < level, and y[level] = sigma (the
                            SHIFTED scheme's adaptive shifts); x FP64 [N_level][m],
                            f device [m] Ritz values, m even up to 96; other
                            entries of y are not written                         */
} bmg_op;

typedef struct {
  int32_t level;     /* level the operator acts on */
  int32_t op;        /* bmg_op */
  int32_t dtype;     /* 0 = FP64 blocks, 1 = FP32 blocks (where the op allows) */
  int32_t m;         /* columns of the interleaved x / y blocks */
  int32_t m2;        /* columns of f for BMG_OP_GRAM */
  int32_t smoother;  /* bmg_smoother for the smoothing ops and BMG_OP_VCYCLE */
  int32_t nu1, nu2;  /* BMG_OP_VCYCLE sweeps */
  int32_t l_c;       /* BMG_OP_VCYCLE coarsest level (-1: Weyl rule as in bmg_solve) */
  int32_t reserved;
  double sigma;      /* shift of the shifted operator */
  double omega;      /* Jacobi weight */
  uint64_t seed;     /* BMG_OP_GAUSSIAN */
} bmg_apply_args;

/* Enqueue one operator of the solver on `stream` with caller-owned device
 * blocks x, f, y (sizes as listed per op; f may be NULL where unused).  For
 * checking each kernel against an independent implementation and for
 * composing custom cycles.  Returns without synchronising. */
int bmg_apply(const bmg_hierarchy* h, const bmg_apply_args* args, const void* x, const void* f,
              void* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * Gram of bmg_apply(BMG_OP_GRAM_AM), G [m2 + m][2m] = [w | u]^T [A_l u | M_l u]
 * with w device [N_l][m2] (NULL if m2 = 0), u device [N_l][m], m even,
 * m2 + m <= 96, G device, all FP64, enqueued on `stream`.  It calls no
 * hipMalloc, hipFree or allocating library routine: the kernel's partial sums
 * live in a static 16 MiB device array (one per device, held until the process
 * ends); the row-block count is reduced where the planner's would not fit, so
 * results agree with bmg_apply's to rounding (a different summation split),
 * not bit for bit.  Calls that overlap on one device share that array and
 * race: serialise them (one stream, or events).  Errors: BMG_EINVAL for
 * invalid sizes or a block whose partial sums exceed the array, BMG_EDEVICE
 * if the array's device address cannot be obtained. */
int bmg_gram_am_noalloc(const bmg_hierarchy* h, int32_t level, const double* w, int32_t m2,
                        const double* u, int32_t m, double* G, void* stream);

/* ------------------------------------------------------------- serving --- */

typedef struct bmg_server bmg_server;

/* A continuous-batching server for many independent eigenproblems (the
 * request-level form of bmg_solve).  Requests wait in arrival order and are
 * admitted while fewer than max_slots run and the device memory they need (an
 * upper bound of the solve's workspace, plus the hierarchy if it is not yet
 * resident) fits in hbm_budget_bytes beside the resident hierarchies, their
 * pooled workspaces and the running requests.  A smaller request may start
 * before a waiting larger one; once the oldest waiting request has been passed
 * 4 * max_slots times, nothing else starts before it.  Admitted requests run
 * concurrently, each on a stream of its own, so their kernels overlap on the
 * device.  Hierarchies are built on first use and cached per surface and
 * level; idle workspaces, then idle hierarchies (least recently used first),
 * are freed when the budget needs their memory.
 * Requests on the same surface and level, at the same shift, that run the
 * enriched scheme with the same precision, smoother, nu1, nu2, omega, n_c and
 * l_c, and wait together, run as one grouped solve (bmg_solve_group; up to 8
 * requests and 512 block columns) in one slot.  A request that ran alone gets
 * bit-for-bit the result of bmg_solve with the same arguments (the kernels
 * are deterministic and requests share only read-only hierarchy data); a
 * grouped one gets it to rounding (stats.group_size > 1).  A server created
 * while the environment variable BMG_NO_GROUP is set groups nothing.
 * Uses the current device; BMG_EDEVICE if there is none.
 * BMG_EINVAL if hbm_budget_bytes <= 0 or max_slots is outside [1, 64].
 * Ownership: *out belongs to the caller until bmg_server_destroy. */
int bmg_server_create(int64_t hbm_budget_bytes, int32_t max_slots, bmg_server** out);

/* Queue one request.  The descriptor (and a custom mesh's arrays) and opts are
 * copied; opts->initial_block and opts->timed_kernel are ignored; opts == NULL
 * means bmg_solve_opts_default.  *request_id gets its id.  BMG_EINVAL on the
 * arguments bmg_build_hierarchy or bmg_solve would reject (those detected only
 * while building are reported by bmg_server_poll), BMG_ENOMEM if the request
 * alone exceeds the budget. */
int bmg_server_submit(bmg_server* s, const bmg_surface_desc* desc, int32_t n_refine, int32_t k,
                      double sigma, double tol, const bmg_solve_opts* opts, uint64_t* request_id);

/* BMG_EBUSY while the request is queued or running.  Otherwise its final status
 * (BMG_OK, BMG_ENOCONV, BMG_ECANCELED, a build or solve error) after copying
 * evals (nullable host [k]), evecs (nullable host column-major [k][ld],
 * ld >= N_L, else BMG_EINVAL and the request is kept), stats (nullable; its
 * rho / delta pointers, if set, receive [k] doubles) and latency_ms (nullable:
 * milliseconds from submit to completion, hierarchy build included).  A
 * finished request is forgotten once polled; BMG_EINVAL for an unknown id. */
int bmg_server_poll(bmg_server* s, uint64_t request_id, double* evals, double* evecs, int64_t ld,
                    bmg_solve_stats* stats, double* latency_ms);

/* A queued request finishes at once with BMG_ECANCELED; a running one stops
 * with BMG_ECANCELED at the end of its current cycle; a finished one is not
 * changed.  BMG_EINVAL for an unknown id. */
int bmg_server_cancel(bmg_server* s, uint64_t request_id);

/* Cancels the queued requests, waits for the running ones, frees every
 * hierarchy and workspace of the server. */
void bmg_server_destroy(bmg_server* s);

/* ---------------------------------------------------------------- misc --- */

const char* bmg_status_string(int status);
/* Text of the last HIP / validation error seen by the calling thread. */
const char* bmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BMG_H */
