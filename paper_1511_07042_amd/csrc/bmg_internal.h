// Internal declarations of the BMG library: host-side hierarchy data, device
// level data, per-solve workspace and the kernel launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bmg.h"

namespace bmg {

// ------------------------------------------------------------------ tracing --
// A named host-time range for rocprofv3's marker trace (roctx): open while the
// object lives.  The solve, its level ramp, its start, its cycle loop, a
// hierarchy build and a level's dense eigendecomposition are marked.
class TraceRange {
 public:
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// ------------------------------------------------------------------ errors --
void set_error(const char* fmt, ...);
const char* get_error();

#define BMG_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::bmg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      return BMG_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

#define BMG_CHECK(cond, ...)          \
  do {                                \
    if (!(cond)) {                    \
      ::bmg::set_error(__VA_ARGS__);  \
      return BMG_EINVAL;              \
    }                                 \
  } while (0)

#define BMG_TRY(expr)          \
  do {                         \
    int s_ = (expr);           \
    if (s_ != BMG_OK) return s_; \
  } while (0)

// ------------------------------------------------------------- host level --
struct HostLevel {
  int64_t n = 0, n_prev = 0, n_tri = 0;
  std::vector<double> xyz;        // [n][3]
  std::vector<int32_t> tri;       // [n_tri][3]
  std::vector<int32_t> parents;   // [n - n_prev][2], a < b
  int32_t W = 0;                  // ELL row width (diagonal first)
  std::vector<int32_t> cols;      // [n][W], padding repeats the row index
  std::vector<double> a, mm;      // [n][W] values of A and M, padding 0
  std::vector<double> lumped;     // [n] row sums of M
  std::vector<int32_t> colour;    // [n]
  int32_t n_colours = 0;
  std::vector<int32_t> colour_ptr;   // [n_colours + 1]
  std::vector<int32_t> colour_rows;  // [n] rows grouped by colour, ascending inside
  // distance-2 colouring (Kaczmarz): no two vertices within two edges share a colour
  std::vector<int32_t> colour2;
  int32_t n_colours2 = 0;
  std::vector<int32_t> colour2_ptr;   // [n_colours2 + 1]
  std::vector<int32_t> colour2_rows;  // [n]
  int32_t RW = 0;                    // children per coarse vertex (restriction gather width)
  std::vector<int32_t> rtab;         // [n_prev][RW] new vertices adjacent to coarse vertex i, -1 pad
  double area = 0.0;
  double hmax = 0.0;                 // longest edge
  int64_t nnz = 0;
};

// Mesh construction (mesh.cpp).  Returns BMG_OK or BMG_EINVAL (+ set_error).
int build_host_levels(const bmg_surface_desc* d, int n_refine, std::vector<HostLevel>& out);
// P1 assembly to ELL + colouring + restriction tables (assemble.cpp).
int assemble_level(HostLevel& lv, const HostLevel* coarser);
// Setup-time dense generalized symmetric-definite eigensolver (dense_host.cpp):
// A x = lambda M x, n x n row-major; lam ascending; X row-major, column j = x_j,
// X^T M X = I.  Cholesky reduction + cyclic Jacobi.
int dense_sygv(int n, const std::vector<double>& A, const std::vector<double>& M,
               std::vector<double>& lam, std::vector<double>& X);
// Row visiting orders (order.cpp): the vertices along a Morton curve through
// xyz ([n][3]), a permutation of 0..n-1; and the same over 16-row chunks placed
// at their centroids (a permutation of the chunk indices).
std::vector<int32_t> morton_order(const std::vector<double>& xyz);
std::vector<int32_t> chunk_morton_order(const HostLevel& H);

// ----------------------------------------------------------- device level --
struct DevLevel {
  int64_t n = 0, n_prev = 0;
  int32_t W = 0, RW = 0, n_colours = 0;
  int32_t* cols = nullptr;
  double* a64 = nullptr;
  double* m64 = nullptr;
  float* a32 = nullptr;
  float* m32 = nullptr;
  double* dinv = nullptr;         // 1 / lumped mass
  // Storage order: large levels keep their rows permuted along a Morton curve
  // (storage row r is vertex perm[r], vertex i is storage row iperm[i]); both
  // null when the level is stored in vertex order.  Row blocks on the device
  // use the storage order; the API converts at its boundary.
  int32_t* perm = nullptr;        // [n]
  int32_t* iperm = nullptr;       // [n]
  std::vector<int32_t> perm_h;    // host copy of perm (empty when null)
  // Transfers to and from the level below, in both levels' storage rows.
  // Nested form (par_nc = n_prev, rself null): fine row i < n_prev is coarse
  // vertex i, parents [n - n_prev][2] are those of the new vertices.  General
  // form (par_nc = 0): parents [n][2] for every fine row (a coarse vertex's
  // copy names it twice), rself [n_prev] the fine row of each coarse vertex.
  int64_t par_nc = 0;
  int32_t* parents = nullptr;
  int32_t* rself = nullptr;
  int32_t* rtab = nullptr;        // [n_prev][RW] fine rows of the new vertices adjacent to coarse row i, -1 pad
  int32_t* colour_rows = nullptr; // [n]
  int32_t* chunk_order = nullptr; // [ceil(n / 16)] 16-row chunks by Morton code of their centroid (large levels stored in vertex order), else null
  int32_t* colour2_rows = nullptr; // [n] rows grouped by distance-2 colour
  std::vector<int32_t> colour_ptr;
  int32_t n_colours2 = 0;
  std::vector<int32_t> colour2_ptr;
  int64_t bytes = 0;
};

// Triangles of one level on the device for the a posteriori estimator:
// tri [F][3], nbr [F][3] = 4 t' + j for the neighbour t' across edge i
// (opposite vertex i) and that edge's index j in t', xyz [N][3].
struct EstLevel {
  int level = -1;
  int64_t F = 0;
  int32_t* tri = nullptr;
  int32_t* nbr = nullptr;
  double* xyz = nullptr;
  int64_t bytes = 0;
};

// All generalized eigenpairs of one level (Alg. 2 step 1 taken at a finer
// coarse level; the interior-shift scheme's coarse solve and start block).
// Built on first use and kept with the hierarchy: it does not depend on the
// shift.  Eigenvectors one per row: phi[j][i] = x_j(i), M_l-orthonormal.
struct LevelEig {
  int level = -1;
  int n = 0;
  std::vector<double> lam;   // host [n] ascending
  double* d_lam = nullptr;   // [n]
  double* d_phi64 = nullptr; // [n][n]
  float* d_phi32 = nullptr;  // [n][n]
  int64_t bytes = 0;
  double setup_ms = 0.0;     // wall time of the eigensolve and upload
};

}  // namespace bmg

struct bmg_hierarchy {
  int device = 0;
  std::vector<bmg::HostLevel> host;
  std::vector<bmg::DevLevel> dev;
  // level-0 generalized eigendecomposition (Alg. 2 step 1)
  int64_t n0 = 0;
  std::vector<double> lam0;  // [n0] ascending
  std::vector<double> phi0;  // [n0][n0] row-major, column j = eigenvector j
  double* d_phi0_64 = nullptr;   // [n0][n0]
  double* d_phi0t_64 = nullptr;  // transpose
  float* d_phi0_32 = nullptr;
  float* d_phi0t_32 = nullptr;
  std::mutex ws_mutex;
  std::vector<struct bmg_workspace*> ws_pool;
  // per-level eigendecompositions of the interior-shift scheme (by level)
  std::mutex eig_mutex;
  std::vector<std::unique_ptr<bmg::LevelEig>> level_eig;
  // the surface (bmg_surface_kind) the hierarchy was built for
  int kind = -1;
  // per-level triangle data of the a posteriori estimator (by level)
  std::mutex est_mutex;
  std::vector<std::unique_ptr<bmg::EstLevel>> est;
};

namespace bmg {

// Level-0 generalized eigensolvers (Alg. 2 step 1): host Jacobi up to
// kHostEigMax vertices, rocSOLVER on the device up to kDeviceEigMax.
constexpr int kHostEigMax = 1024;
constexpr int kDeviceEigMax = 4096;
int device_sygv(int n, const std::vector<double>& A, const std::vector<double>& M,
                std::vector<double>& lam, std::vector<double>& X, hipStream_t s);
// The same solve leaving the eigenvectors on the device: *vecs [n][n] with
// row j the M-orthonormal eigenvector j (the caller frees it with hipFree).
int device_sygv_keep(int n, const std::vector<double>& A, const std::vector<double>& M,
                     std::vector<double>& lam, double** vecs, hipStream_t s);
// Largest level the interior-shift scheme eigendecomposes densely.
constexpr int kLevelEigMax = 12288;

// A device-wide synchronisation (hipFree, hipDeviceSynchronize, the dense
// eigensolver's set-up and teardown) on one thread while another thread's
// stream is capturing a graph fails and leaves a sticky error on the calling
// thread, which then fails its next launch.  Graph captures therefore hold a
// process-wide lock shared and such calls hold it exclusively; the exclusive
// side is re-entrant on one thread.  Captures only enqueue kernels.
struct DeviceSyncGuard {
  DeviceSyncGuard();
  ~DeviceSyncGuard();
  DeviceSyncGuard(const DeviceSyncGuard&) = delete;
  DeviceSyncGuard& operator=(const DeviceSyncGuard&) = delete;
};
struct CaptureGuard {
  CaptureGuard();
  ~CaptureGuard();
  CaptureGuard(const CaptureGuard&) = delete;
  CaptureGuard& operator=(const CaptureGuard&) = delete;
};
// hipFree under DeviceSyncGuard (null is ignored)
void dev_free(void* p);
// The eigendecomposition of level l (built on first use; thread-safe).
int level_eig(bmg_hierarchy* h, int l, hipStream_t s, const LevelEig** out);
void free_level_eigs(bmg_hierarchy* h);
int upload_hierarchy(bmg_hierarchy* h, hipStream_t s);
void free_device(bmg_hierarchy* h);
// Solve workspaces pooled per hierarchy (solver.cpp): bytes held by the idle
// ones, and freeing them.
void free_workspaces(bmg_hierarchy* h);
int64_t idle_workspace_bytes(bmg_hierarchy* h);
void trim_idle_workspaces(bmg_hierarchy* h);
// Defaults shared by the solver and the server's footprint estimates.
int default_block_width(int k, double sigma);
// The widest block the solver gives a request that names no width: at most
// 96 - n_c columns, half the finest level's rows and (interior scheme) half
// of level l_c's.
int block_width_cap(const bmg_hierarchy* h, int n_c, bool shifted, int l_c);
int default_coarse_vectors(const bmg_hierarchy* h);
int solve(bmg_hierarchy* h, int k, double sigma, double tol, const bmg_solve_opts* opts,
          double* evals, double* evecs, int64_t ld, int evecs_on_device, void* stream,
          bmg_solve_stats* stats);
// Grouped solve (solver.cpp); see bmg_solve_group in bmg.h.  cancel: nullable
// per-request flags (a request whose flag reads nonzero stops with
// BMG_ECANCELED at the end of the current cycle).
int solve_group(bmg_hierarchy* h, double sigma, int n, bmg_group_request* reqs, void* stream,
                const std::atomic<int>* const* cancel = nullptr);
// A posteriori estimator of eq. est-res (estimate.cpp); see bmg_estimate in bmg.h.
int estimate(bmg_hierarchy* h, int level, int k, const double* evals, const double* evecs, int64_t ld,
             double* eta, double* parts, double* eta2_T, hipStream_t s);
void free_est_levels(bmg_hierarchy* h);
// Per-triangle kernel and the fixed-order reduction of its per-block sums
// (kernels_estimate.hip): part [nblk][k][3], out [3][k].
int est_blocks(int64_t F);
int launch_estimate(const EstLevel& E, int k, const double* U, int64_t ld, const double* lam,
                    int sphere, double* eta2_T, double* part, double* out, hipStream_t s);
// Two-grid cascade of Alg. 1 (twogrid.cpp); see bmg_two_grid in bmg.h.
int two_grid(bmg_hierarchy* h, int level_H, int n, const int32_t* idx, int top, int nu, double* evals,
             double* evecs, hipStream_t s);

// ------------------------------------------------------------- launchers --
// Kernel timing: a caller that wants the next launch timed sets `start` and
// `stop`; the launcher consumes them and records them at the kernel's own
// start and end (hipExtLaunchKernelGGL), so the elapsed time excludes the
// queueing around it.  A class of two kernels takes start on the first and
// stop on the second.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;
// Set by a serving worker around a solve: the cycle loop stops with
// BMG_ECANCELED when it reads nonzero.
extern thread_local const std::atomic<int>* g_cancel;

#define BMG_LAUNCH(kernel, grid, block, shmem, stream, ...)                                  \
  do {                                                                                       \
    const ::bmg::LaunchEvents ev_ = ::bmg::g_launch_events;                                  \
    ::bmg::g_launch_events = ::bmg::LaunchEvents{};                                          \
    if (ev_.start || ev_.stop)                                                               \
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), (shmem), (stream), ev_.start,   \
                            ev_.stop, 0, __VA_ARGS__);                                       \
    else                                                                                     \
      kernel<<<(grid), (block), (shmem), (stream)>>>(__VA_ARGS__);                           \
  } while (0)

// Interleaved blocks [n][m]; T = double or float.  All launchers enqueue on s
// and return BMG_OK or BMG_EDEVICE.
enum RowMode { ROW_SHIFTED = 0, ROW_RESIDUAL = 1 };

// S = A - sigma M in precision T (same expression as the smoothers use)
template <typename T>
int launch_shift(const DevLevel& L, double sigma, T* S, hipStream_t s);
template <typename T>
int launch_shifted(const DevLevel& L, const T* S, int mode, const T* x, const T* f, T* y, int m,
                   hipStream_t s);
int launch_spmm_am(const DevLevel& L, const double* x, double* ya, double* ym, int m,
                   hipStream_t s);
// y = A x - (M x) diag(theta) (FP64) stored as T with sign `sgn` (+1 or -1),
// rho2_part[b][m] = per-block partial sums of r^2 / lumped (FP64) if non-null.
template <typename T>
int launch_eigres(const DevLevel& L, const double* x, const double* theta, double sgn, T* y,
                  double* rho2_part, int nblk, int m, hipStream_t s);
int eigres_blocks(const DevLevel& L, int m);
// out[c] = sum_b part[c][b]; with mirror set (host-mapped [theta m][rho2 m][8
// status words]) theta and the status words are copied from src (the device
// buffer of that layout, out = src + m) and the sums written there as well.
int launch_colsum(const double* part, int nblk, int m, double* out, hipStream_t s,
                  const double* src = nullptr, double* mirror = nullptr);

template <typename T>
// u_add != nullptr: the sweep's result is added to the FP64 block u_add
// (n x m) instead of being written to y (the cycle's last sweep of the finest
// level adds its correction to the iterate directly).
int launch_jacobi(const DevLevel& L, const T* S, double omega, const T* x, const T* f, T* y,
                  bool x_is_zero, int m, hipStream_t s, double* u_add = nullptr);
template <typename T>
int launch_gs_colour(const DevLevel& L, const T* S, int colour, T* x, const T* f, int m,
                     hipStream_t s);
// Kaczmarz projections of the rows of one distance-2 colour, in place.
template <typename T>
int launch_kaczmarz_colour(const DevLevel& L, const T* S, int colour, T* x, const T* f, int m,
                           hipStream_t s);
// The same in FP64 with a shift per column: column c relaxes
// (A - shifts[c] M) x_c = f_c (shifts: device [m]; m even).
int launch_kaczmarz_shifts_colour(const DevLevel& L, int colour, const double* shifts, double* x,
                                  const double* f, int m, hipStream_t s);
// Per column: rq[c] = u_c^T A u_c / u_c^T M u_c over the level's rows, then
// u_c scaled in place to unit M-norm (a zero column stays zero, rq[c] = 0).
// part: [kRqBlocks][2m] doubles; rq: device [2m] (rq, then 1 / M-norms).
int launch_rq_normalise(const DevLevel& L, double* U, int m, double* part, double* rq, hipStream_t s);
// Fused cycle kernels (identical results to the unfused sequences):
// two Jacobi sweeps from zero; residual + restriction; prolongation + one
// Jacobi sweep.
template <typename T>
int launch_jacobi2z(const DevLevel& L, const T* S, double omega, const T* f, T* y, int m,
                    hipStream_t s);
template <typename T>
int launch_resrestrict(const DevLevel& fine, const T* S, const T* e, const T* f, T* fc, int m,
                       hipStream_t s);
template <typename T>
int launch_prolong_jacobi(const DevLevel& fine, const T* S, double omega, const T* e, const T* ec,
                          const T* f, T* y, int m, hipStream_t s);
template <typename T>
int launch_restrict(const DevLevel& fine, const T* x, T* y, int m, hipStream_t s);
template <typename T>
int launch_prolong_add(const DevLevel& fine, const T* x, T* y, int m, hipStream_t s);
template <typename T>
int launch_fill(T* y, int64_t count, T value, hipStream_t s);
template <typename T>
int launch_dense_apply(int n, const T* mat, const T* g, const T* x, T* y, int m, hipStream_t s);
// U (FP64) += e (T)
template <typename T>
int launch_add_to(double* u, const T* e, int64_t count, hipStream_t s);
template <typename T>
int launch_convert(const double* x, T* y, int64_t count, hipStream_t s);
// element (r, j) from counter perm[r] m + j (perm null: r m + j), so the block
// in a permuted storage order holds the same numbers per vertex
int launch_gaussian(double* y, int64_t n, int m, uint64_t seed, hipStream_t s, const int* perm = nullptr);

// Gram: G[nz][ny] = Z^T Y with Z = [z1 (w1 cols) | z2 (w2 cols)], Y = [y1 | y2]
// (v1, v2 cols), all FP64 [n][w] blocks.  part: [nblk][nzp][nyp].
struct GramPlan {
  int nz, ny, nzp, nyp, nblk;
  int64_t per_block;  // doubles of partial sums per block (the larger of the two layouts)
};
GramPlan gram_plan(int64_t n, int nz, int ny);
int64_t sym_tile_doubles(int w1, int m);
// G = [w | u]^T [A_L u | M_L u] with the products formed in LDS (fused SpMM
// and Gram; w1 columns of w, m of u; plan for nz = w1 + m, ny = 2 m).
// uperm (nullable): w and u are in vertex order and storage row r reads row uperm[r];
// ldu: row stride of u (0: m), so u may be a column slice of a wider block;
// nreq > 1: that many equal-width requests side by side in u (request r's
// columns start r m further), partials and G of request r at r part_stride
// and r g_stride, in one launch
int launch_gram_am(const GramPlan& p, const DevLevel& L, const double* w, int w1, const double* u,
                   int m, double* part, double* G, hipStream_t s, const int* uperm = nullptr, int ldu = 0,
                   int nreq = 1, int64_t part_stride = 0, int64_t g_stride = 0);
int launch_gram(const GramPlan& p, int64_t n, const double* z1, int w1, const double* z2, int w2,
                const double* y1, int v1, const double* y2, int v2, double* part, double* G,
                hipStream_t s);
// U[n][m] = Z Y, Z = [z1 (w1) | z2 (w2)], Y [w1+w2][m] device; ldz2, ldu: row
// strides of z2 and U (0: w2 and m), so both may be column slices of a wider block
// nreq > 1: that many equal-width requests side by side (request r's columns
// of z2 and U start r w2 and r m further, its Y at r (w1 + w2) m), one launch
int launch_update_zy(int64_t n, const double* z1, int w1, const double* z2, int w2,
                     const double* Y, double* U, int m, hipStream_t s, int ldz2 = 0, int ldu = 0,
                     int nreq = 1);

// Coarse end of the correction cycle in one workgroup, in LDS (kernels_tail.hip).
constexpr int kTailMaxLevels = 12;
constexpr int kTailMaxColours = 32;
constexpr int kTailLdsBudget = 152 * 1024;
struct TailLevel {  // byte offsets into the kernel's dynamic LDS
  int n, n_prev, W, RW, n_colours;
  int off_S, off_cols, off_crow, off_par, off_rtab, off_e, off_f, off_t;
  int colour_ptr[kTailMaxColours + 1];
};
struct alignas(16) TailArgs {
  int lo, hi, m, smoother, nu1, nu2;
  int m_full;  // columns of the global blocks; workgroup g takes columns [g m, (g + 1) m)
  double omega;
  const void* image;  // packed static arrays, copied to LDS offset 0
  int image_bytes;
  int off_phi, off_phit, off_g;  // level-0 spectral inverse (-1: smoothing at lo)
  const void* f_top;  // f of level hi (global)
  void* e_top;        // e of level hi (global)
  TailLevel lv[kTailMaxLevels];
};
template <typename T>
int launch_tail(const TailArgs* dev_args, int lds_bytes, int groups, hipStream_t s);

// One-workgroup Ritz step (see kernels_dense.hip).
struct RitzArgs {
  int n_c, m, nz;        // nz = n_c + m
  double sigma;
  double rtol2;          // squared significance threshold of a Jacobi rotation
  int warm;              // 1: start from the coarse-block basis the previous call left in scratch
  const double* G;       // [nz][2m]: Z^T [A U | M U]
  const double* GW;      // [n_c][2 n_c]: W^T [A W | M W] (constant during a solve)
  double* Y;             // out [nz][m]
  double* theta;         // out [m] ascending
  double* scratch;       // [ritz_scratch_doubles(nz)]; its tail persists between calls
  int* status;           // out: 0 ok, 1 rank loss below m, 2 Jacobi did not converge
  const double* rho2 = nullptr;  // [m] residual norms of the previous block (with theta on
                                 // entry): the Jacobi threshold follows them; null: rtol2
};
int launch_ritz(const RitzArgs& a, hipStream_t s);
// The Ritz steps of several requests in one launch (one workgroup each).
constexpr int kRitzBatchMax = 16;
struct RitzBatch {
  int n, n_c;
  double sigma, rtol2;
  const double* GW;
  int m[kRitzBatchMax];
  const double* G[kRitzBatchMax];
  double* Y[kRitzBatchMax];
  double* theta[kRitzBatchMax];
  double* scratch[kRitzBatchMax];
  int* status[kRitzBatchMax];
  const double* rho2[kRitzBatchMax];  // as RitzArgs::rho2
};
int launch_ritz_batch(const RitzBatch& b, int warm, hipStream_t s);
// Significance threshold (squared) of a rotation in the Ritz step.  An
// off-diagonal a_pq left below 1e-11 of the diagonal scale moves a Ritz vector
// by ~1e-11 relative and adds ~1e-11 ||C|| to its residual: far below what the
// stopping certificate asks (rho / delta <= 1e-7) for the shifted Ritz
// matrices of these problems (||C|| of order 1e2), and the certificate is
// computed from the true residuals, so a looser threshold cannot pass a pair
// that is not accurate.  Ritz values change at second order (~1e-22).
constexpr double kRitzRtol2 = 1e-22;
int launch_syev(int n, const double* A, double* w, double* V, int* status, hipStream_t s);
int ritz_scratch_doubles(int nz);

// Interior-shift scheme (kernels_coarse.hip).
// e = Phi^T diag(g) Phi f with phi [n][n] (row j = eigenvector j), f, e [n][m];
// t [n][m] and part [spec_slices(n)][n][m] are scratch.
int spec_slices(int n);
template <typename T>
int launch_spec_apply(int n, const T* phi, const T* g, const T* f, T* t, T* part, T* e, int m,
                      hipStream_t s);
// g[i] = 1 / (lam[i] - *shift), 0 where |lam[i] - *shift| < tau
template <typename T>
int launch_spec_g(int n, const double* lam, const double* shift, double tau, T* g, hipStream_t s);
// S = A - (*shift) M, the shift read from device memory
template <typename T>
int launch_shift_dev(const DevLevel& L, const double* shift, T* S, hipStream_t s);
// blk [n][m]: blk[i][c] = phi[sel[c]][i]
int launch_gather_rows(int n, int m, const double* phi, const int* sel, double* blk, hipStream_t s);
// Per-level shifts from the block U (FP64 [N_top][m]) and its Ritz values
// theta: shifts[l] = sigma + mean_c(U_c^T A_l U_c / U_c^T M_l U_c - theta_c)
// over the first N_l rows, lo <= l < top; shifts[top] = sigma.  part holds
// [top][kRqBlocks][2m] doubles.
constexpr int kRqBlocks = 64;
int launch_offsets(const std::vector<DevLevel>& dev, int lo, int top, const double* U, int m,
                   double sigma, const double* theta, double* part, double* shifts, hipStream_t s);

// column-wise argmax |U[:, sel_j]| (lowest row on ties) and output writer
// signs and output of the selected columns in vertex order (iperm: the
// storage row of each vertex, null when the storage is in vertex order)
int launch_signs(int64_t n, const double* U, int m, const int* sel, int k, const int* iperm, double* sign_out,
                 double* part_val, int* part_idx, int nblk, hipStream_t s);
int launch_write_evecs(int64_t n, const double* U, int m, const int* sel, const double* sign,
                       int k, const int* iperm, double* out, int64_t ld, hipStream_t s);
// y[r] = x[map[r]] for an [n][m] block
template <typename T>
int launch_permute_rows(int64_t n, int m, const int* map, const T* x, T* y, hipStream_t s);

}  // namespace bmg
