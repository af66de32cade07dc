// BMG solve driver: the cycle of Alg. 2/3 iterated on the finest level with a
// fixed shift, all device work on the caller's stream.
//
// Per cycle (paper Alg. 3 steps 2-5, Remark 3.2):
//   H1  R = A U - M U Theta (FP64), stored as -R in the correction precision,
//       and rho_i^2 = ||r_i||^2_{D^-1}; O(m) values are read back to decide
//       convergence (the paper runs fixed cycles; the certificate is ours).
//   H2  E = B_sigma(-R): one V(nu1, nu2) cycle for (A_l - sigma M_l) on levels
//       L..l_c with restriction P^T and prolongation P (Sec. 3), smoothing by
//       multicolour Gauss-Seidel or weighted Jacobi (Sec. 5.3 methods 2/4).
//   H3  U' = U + E.
//   H4  Gram matrices of Z = [W_c, U'] with A and M (enriched pencil,
//       eq. pb-c-aux-mat, Galerkin evaluation on the finest level).
//   H5  SVQB M-orthonormalisation and the shifted Ritz problem (one workgroup).
//   H6  U <- Z Y.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "bmg_internal.h"

struct bmg_workspace {
  int64_t N = 0;
  int m = 0, n_c = 0, prec = 0, nl = 0;
  bool busy = false;
  double *W = nullptr, *AW = nullptr, *MW = nullptr;
  double *U = nullptr, *AU = nullptr, *MU = nullptr;
  std::vector<void*> e, f, t;  // per level, correction precision
  void* ctmp = nullptr;        // [N0][m]
  void* gco = nullptr;         // [N0]
  double *gpart = nullptr, *G = nullptr, *GW = nullptr, *Y = nullptr, *theta = nullptr;
  double *rho2part = nullptr, *rho2 = nullptr, *rscratch = nullptr;
  int* status = nullptr;
  int* sel = nullptr;
  double *sign = nullptr, *argv = nullptr;
  int* argi = nullptr;
  double* hbuf = nullptr;  // pinned host: theta[m], rho2[m], status
  int nblk_res = 0, nblk_arg = 0;
  bmg::GramPlan gp{}, gpw{};
  std::vector<void*> allocs;
};

namespace bmg {
namespace {

int dalloc(bmg_workspace* w, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of %zu bytes failed", bytes);
    return BMG_ENOMEM;
  }
  w->allocs.push_back(*p);
  return BMG_OK;
}

void free_workspace(bmg_workspace* w) {
  for (void* p : w->allocs) (void)hipFree(p);
  if (w->hbuf) (void)hipHostFree(w->hbuf);
  delete w;
}

int make_workspace(bmg_hierarchy* h, int m, int n_c, int prec, bmg_workspace** out) {
  auto* w = new bmg_workspace();
  const int nl = int(h->dev.size());
  const int64_t N = h->dev[nl - 1].n;
  w->N = N;
  w->m = m;
  w->n_c = n_c;
  w->prec = prec;
  w->nl = nl;
  const size_t vb = prec == BMG_MIXED ? sizeof(float) : sizeof(double);
  auto A = [&](void** p, size_t bytes) { return dalloc(w, p, bytes); };
  int st = BMG_OK;
#define AL(ptr, bytes)                                           \
  do {                                                           \
    st = A(reinterpret_cast<void**>(&(ptr)), (bytes));           \
    if (st != BMG_OK) {                                          \
      free_workspace(w);                                         \
      return st;                                                 \
    }                                                            \
  } while (0)
  AL(w->W, sizeof(double) * N * n_c);
  AL(w->AW, sizeof(double) * N * n_c);
  AL(w->MW, sizeof(double) * N * n_c);
  AL(w->U, sizeof(double) * N * m);
  AL(w->AU, sizeof(double) * N * m);
  AL(w->MU, sizeof(double) * N * m);
  w->e.resize(nl);
  w->f.resize(nl);
  w->t.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const size_t b = vb * h->dev[l].n * m;
    AL(w->e[l], b);
    AL(w->f[l], b);
    AL(w->t[l], b);
  }
  AL(w->ctmp, vb * h->n0 * m);
  AL(w->gco, vb * h->n0);
  const int nz = n_c + m;
  w->gp = gram_plan(N, nz, 2 * m);
  w->gpw = gram_plan(N, n_c, 2 * n_c);
  const size_t gpb = std::max(size_t(w->gp.nblk) * w->gp.nzp * w->gp.nyp,
                              size_t(w->gpw.nblk) * w->gpw.nzp * w->gpw.nyp);
  AL(w->gpart, sizeof(double) * gpb);
  AL(w->G, sizeof(double) * nz * 2 * m);
  AL(w->GW, sizeof(double) * n_c * 2 * n_c);
  AL(w->Y, sizeof(double) * nz * m);
  AL(w->theta, sizeof(double) * m);
  w->nblk_res = eigres_blocks(h->dev[nl - 1], m);
  AL(w->rho2part, sizeof(double) * w->nblk_res * m);
  AL(w->rho2, sizeof(double) * m);
  AL(w->rscratch, sizeof(double) * ritz_scratch_doubles(nz));
  AL(w->status, sizeof(int) * 4);
  AL(w->sel, sizeof(int) * m);
  AL(w->sign, sizeof(double) * m);
  w->nblk_arg = int(std::min<int64_t>(256, (N + 255) / 256));
  AL(w->argv, sizeof(double) * w->nblk_arg * m);
  AL(w->argi, sizeof(int) * w->nblk_arg * m);
#undef AL
  if (hipHostMalloc(reinterpret_cast<void**>(&w->hbuf), sizeof(double) * (2 * m + 4)) != hipSuccess) {
    (void)hipGetLastError();
    free_workspace(w);
    set_error("hipHostMalloc failed");
    return BMG_ENOMEM;
  }
  *out = w;
  return BMG_OK;
}

int acquire_workspace(bmg_hierarchy* h, int m, int n_c, int prec, bmg_workspace** out) {
  {
    std::lock_guard<std::mutex> g(h->ws_mutex);
    for (auto* w : h->ws_pool)
      if (!w->busy && w->m == m && w->n_c == n_c && w->prec == prec) {
        w->busy = true;
        *out = w;
        return BMG_OK;
      }
  }
  bmg_workspace* w = nullptr;
  BMG_TRY(make_workspace(h, m, n_c, prec, &w));
  w->busy = true;
  std::lock_guard<std::mutex> g(h->ws_mutex);
  h->ws_pool.push_back(w);
  *out = w;
  return BMG_OK;
}

void release_workspace(bmg_hierarchy* h, bmg_workspace* w) {
  std::lock_guard<std::mutex> g(h->ws_mutex);
  w->busy = false;
}

}  // namespace

void free_workspaces(bmg_hierarchy* h) {
  std::lock_guard<std::mutex> g(h->ws_mutex);
  for (auto* w : h->ws_pool) free_workspace(w);
  h->ws_pool.clear();
}

// ----------------------------------------------------------- kernel timer --
// Brackets the launches of one kernel class (finest level only) with HIP events
// on the solve's stream; durations are summed after the final synchronisation.
struct KTimer {
  int which = -1;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double bytes = 0.0;
  int64_t units = 0;
  int begin(int k) {
    if (k != which) return BMG_OK;
    if (2 * used + 2 > ev.size()) {
      hipEvent_t a, b;
      BMG_HIP(hipEventCreate(&a));
      BMG_HIP(hipEventCreate(&b));
      ev.push_back(a);
      ev.push_back(b);
    }
    BMG_HIP(hipEventRecord(ev[2 * used], s));
    return BMG_OK;
  }
  int end(int k) {
    if (k != which) return BMG_OK;
    BMG_HIP(hipEventRecord(ev[2 * used + 1], s));
    ++used;
    return BMG_OK;
  }
  void add(int k, double b, int64_t u) {
    if (k != which) return;
    bytes += b;
    units += u;
  }
  double total_ms() {
    double t = 0.0;
    for (size_t i = 0; i < used; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) t += ms;
    }
    return t;
  }
  ~KTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// ------------------------------------------------------- correction cycle --
struct CycleCfg {
  int m, nu1, nu2, smoother, l_c;
  double sigma, omega;
};

template <typename T>
struct Cycle {
  bmg_hierarchy* h;
  CycleCfg c;
  std::vector<T*> e, f, t;
  T* ctmp;
  const T* g0;  // truncated inverse spectrum at level 0
  hipStream_t s;
  KTimer* kt = nullptr;  // timing of finest-level launches (level L)
  int L = -1;

  int kclass(int l, int k) const { return (kt && l == L) ? k : -2; }

  int sweep(int l, bool forward, bool from_zero) {
    const DevLevel& D = h->dev[l];
    const int kc = kclass(l, BMG_K_SMOOTH);
    const double b = sizeof(T);
    if (kt) kt->add(kc, (4 + 2 * b) * double(h->host[l].nnz) + 4.0 * D.n + 3 * b * D.n * c.m, 1);
    if (c.smoother == BMG_SMOOTH_JACOBI) {
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_jacobi<T>(D, c.sigma, c.omega, e[l], f[l], t[l], from_zero, c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
      std::swap(e[l], t[l]);
      return BMG_OK;
    }
    if (from_zero) BMG_TRY(launch_fill<T>(e[l], D.n * c.m, T(0), s));
    for (int k = 0; k < D.n_colours; ++k) {
      const int col = forward ? k : D.n_colours - 1 - k;
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_gs_colour<T>(D, col, c.sigma, e[l], f[l], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
    }
    return BMG_OK;
  }

  // e[l] <- B_sigma f[l]
  int vcycle(int l) {
    const DevLevel& D = h->dev[l];
    if (l == c.l_c) {
      if (l == 0) {
        const int n0 = int(h->n0);
        const T* pt = std::is_same<T, float>::value ? (const T*)h->d_phi0t_32 : (const T*)h->d_phi0t_64;
        const T* p = std::is_same<T, float>::value ? (const T*)h->d_phi0_32 : (const T*)h->d_phi0_64;
        BMG_TRY(launch_dense_apply<T>(n0, pt, nullptr, f[0], ctmp, c.m, s));
        BMG_TRY(launch_dense_apply<T>(n0, p, g0, ctmp, e[0], c.m, s));
        return BMG_OK;
      }
      for (int k = 0; k < 8; ++k) BMG_TRY(sweep(l, k % 2 == 0, k == 0));
      return BMG_OK;
    }
    for (int k = 0; k < c.nu1; ++k) BMG_TRY(sweep(l, true, k == 0));
    if (c.nu1 == 0) BMG_TRY(launch_fill<T>(e[l], D.n * c.m, T(0), s));
    const double b = sizeof(T);
    const double nnz = double(h->host[l].nnz), n = double(D.n), nc = double(D.n_prev);
    int kc = kclass(l, BMG_K_RESIDUAL);
    if (kt) kt->add(kc, (4 + 2 * b) * nnz + 3 * b * n * c.m, 1);
    if (kt) BMG_TRY(kt->begin(kc));
    BMG_TRY(launch_shifted<T>(D, ROW_RESIDUAL, c.sigma, e[l], f[l], t[l], c.m, s));
    if (kt) BMG_TRY(kt->end(kc));
    kc = kclass(l, BMG_K_RESTRICT);
    if (kt) kt->add(kc, b * n * c.m + b * nc * c.m + 4.0 * nc * D.RW, 1);
    if (kt) BMG_TRY(kt->begin(kc));
    BMG_TRY(launch_restrict<T>(D, t[l], f[l - 1], c.m, s));
    if (kt) BMG_TRY(kt->end(kc));
    BMG_TRY(vcycle(l - 1));
    kc = kclass(l, BMG_K_PROLONG);
    if (kt) kt->add(kc, b * nc * c.m + 2 * b * n * c.m + 8.0 * (n - nc), 1);
    if (kt) BMG_TRY(kt->begin(kc));
    BMG_TRY(launch_prolong_add<T>(D, e[l - 1], e[l], c.m, s));
    if (kt) BMG_TRY(kt->end(kc));
    for (int k = 0; k < c.nu2; ++k) BMG_TRY(sweep(l, false, false));
    return BMG_OK;
  }
};

int weyl_coarsest(const bmg_hierarchy* h, double sigma) {
  const int nl = int(h->host.size());
  const double nw = h->host[nl - 1].area * std::max(sigma, 0.0) / (4.0 * M_PI);
  for (int l = 0; l < nl; ++l)
    if (double(h->host[l].n) >= 8.0 * nw) return l;
  return nl - 1;
}

namespace {

// k nearest sigma among values (ties: value, then index)
std::vector<int> nearest(const std::vector<double>& v, double sigma, int k) {
  std::vector<int> idx(v.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const double da = std::fabs(v[a] - sigma), db = std::fabs(v[b] - sigma);
    if (da != db) return da < db;
    if (v[a] != v[b]) return v[a] < v[b];
    return a < b;
  });
  idx.resize(std::min<size_t>(k, idx.size()));
  return idx;
}

struct Cert {
  bool ok = false;
  double max_dk = 0, max_kt = 0;
  std::vector<double> rho, delta;
  std::vector<int> ret;
};

Cert certify(const std::vector<double>& theta, const std::vector<double>& rho2, double sigma,
             int k, double tol, double angle_tol) {
  Cert c;
  const int m = int(theta.size());
  std::vector<int> cid(m, 0);
  for (int j = 1; j < m; ++j) {
    const double gap = theta[j] - theta[j - 1];
    const double sc = std::max({std::fabs(theta[j]), std::fabs(theta[j - 1]), 1.0});
    cid[j] = cid[j - 1] + (gap < 1e-2 * sc ? 0 : 1);
  }
  c.ret = nearest(theta, sigma, k);
  bool kt_ok = true;
  for (int i : c.ret) {
    double d = INFINITY;
    for (int j = 0; j < m; ++j)
      if (cid[j] != cid[i]) d = std::min(d, std::fabs(theta[j] - theta[i]));
    if (!std::isfinite(d)) d = 1e-2 * std::max(std::fabs(theta[i]), 1.0);
    const double r = 2.0 * std::sqrt(std::max(rho2[i], 0.0));
    c.rho.push_back(r);
    c.delta.push_back(d);
    const double kt = r * r / d;
    const double sc = std::max(std::fabs(theta[i]), 1.0);
    if (!(kt <= 0.1 * tol * sc)) kt_ok = false;
    c.max_kt = std::max(c.max_kt, kt / sc);
    c.max_dk = std::max(c.max_dk, r / d);
  }
  c.ok = kt_ok && (c.max_dk <= angle_tol);
  return c;
}

template <typename T>
int run_solve(bmg_hierarchy* h, bmg_workspace* w, int k, double sigma, double tol,
              const bmg_solve_opts& o, int l_c, double* evals, double* evecs, int64_t ld,
              int evecs_on_device, hipStream_t s, bmg_solve_stats* stats) {
  const int nl = int(h->dev.size());
  const int L = nl - 1;
  const DevLevel& DL = h->dev[L];
  const int64_t N = DL.n;
  const int m = o.m, n_c = o.n_c, nz = n_c + m;
  const int64_t n0 = h->n0;
  hipEvent_t ev0, ev1;
  BMG_HIP(hipEventCreate(&ev0));
  BMG_HIP(hipEventCreate(&ev1));
  BMG_HIP(hipEventRecord(ev0, s));

  // ---- S2: W_c = P_{0->L} Phi_c, its Gram blocks, and the level-0 inverse
  {
    std::vector<int> idx = nearest(h->lam0, sigma, n_c);
    std::sort(idx.begin(), idx.end());
    std::vector<double> phic(size_t(n0) * n_c);
    for (int64_t i = 0; i < n0; ++i)
      for (int j = 0; j < n_c; ++j) phic[size_t(i) * n_c + j] = h->phi0[size_t(i) * n0 + idx[j]];
    std::vector<T> g(n0);
    for (int64_t i = 0; i < n0; ++i) {
      const double x = h->lam0[i] - sigma;
      g[i] = std::fabs(x) >= 1e-2 * std::max(1.0, std::fabs(sigma)) ? T(1.0 / x) : T(0);
    }
    double* cur = (L % 2 == 0) ? w->W : w->AW;  // ping-pong so the last lands in W
    BMG_HIP(hipMemcpyAsync(cur, phic.data(), sizeof(double) * phic.size(), hipMemcpyHostToDevice, s));
    BMG_HIP(hipMemcpyAsync(w->gco, g.data(), sizeof(T) * n0, hipMemcpyHostToDevice, s));
    for (int l = 1; l <= L; ++l) {
      double* nxt = (cur == w->W) ? w->AW : w->W;
      BMG_TRY(launch_fill<double>(nxt, h->dev[l].n * n_c, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(h->dev[l], cur, nxt, n_c, s));
      cur = nxt;
    }
    BMG_HIP(hipStreamSynchronize(s));  // phic / g are host locals
  }
  BMG_TRY(launch_spmm_am(DL, w->W, w->AW, w->MW, n_c, s));
  BMG_TRY(launch_gram(w->gpw, N, w->W, n_c, nullptr, 0, w->AW, n_c, w->MW, n_c, w->gpart, w->GW, s));

  // ---- S3: test vectors and the first Rayleigh-Ritz step
  if (o.initial_block)
    BMG_HIP(hipMemcpyAsync(w->U, o.initial_block, sizeof(double) * N * m, hipMemcpyHostToDevice, s));
  else
    BMG_TRY(launch_gaussian(w->U, N, m, o.seed, s));

  KTimer kt;
  kt.which = o.timed_kernel;
  kt.s = s;
  const double nnzL = double(h->host[L].nnz), Nd = double(N);
  int ritz_sweeps_max = 0, ritz_fallbacks = 0;
  RitzArgs ra;
  ra.n_c = n_c;
  ra.m = m;
  ra.nz = nz;
  ra.sigma = sigma;
  ra.G = w->G;
  ra.GW = w->GW;
  ra.Y = w->Y;
  ra.theta = w->theta;
  ra.scratch = w->rscratch;
  ra.status = w->status;
  auto ritz_step = [&]() -> int {
    kt.add(BMG_K_SPMM_AM, 20 * nnzL + 24 * Nd * m, 1);
    BMG_TRY(kt.begin(BMG_K_SPMM_AM));
    BMG_TRY(launch_spmm_am(DL, w->U, w->AU, w->MU, m, s));
    BMG_TRY(kt.end(BMG_K_SPMM_AM));
    kt.add(BMG_K_GRAM, 4.0 * Nd * nz * m, 1);
    BMG_TRY(kt.begin(BMG_K_GRAM));
    BMG_TRY(launch_gram(w->gp, N, w->W, n_c, w->U, m, w->AU, m, w->MU, m, w->gpart, w->G, s));
    BMG_TRY(kt.end(BMG_K_GRAM));
    kt.add(BMG_K_RITZ, 0.0, 1);
    BMG_TRY(kt.begin(BMG_K_RITZ));
    BMG_TRY(launch_ritz(ra, s));
    BMG_TRY(kt.end(BMG_K_RITZ));
    kt.add(BMG_K_UPDATE, 2.0 * Nd * nz * m, 1);
    BMG_TRY(kt.begin(BMG_K_UPDATE));
    BMG_TRY(launch_update_zy(N, w->W, n_c, w->U, m, w->Y, w->U, m, s));  // in place
    BMG_TRY(kt.end(BMG_K_UPDATE));
    return BMG_OK;
  };
  BMG_TRY(ritz_step());

  Cycle<T> cyc;
  cyc.h = h;
  cyc.c = CycleCfg{m, o.nu1, o.nu2, o.smoother, l_c, sigma, o.omega};
  cyc.e.resize(nl);
  cyc.f.resize(nl);
  cyc.t.resize(nl);
  for (int l = 0; l < nl; ++l) {
    cyc.e[l] = static_cast<T*>(w->e[l]);
    cyc.f[l] = static_cast<T*>(w->f[l]);
    cyc.t[l] = static_cast<T*>(w->t[l]);
  }
  cyc.ctmp = static_cast<T*>(w->ctmp);
  cyc.g0 = static_cast<const T*>(w->gco);
  cyc.s = s;
  cyc.kt = o.timed_kernel >= 0 ? &kt : nullptr;
  cyc.L = L;

  std::vector<double> theta(m), rho2(m);
  Cert cert;
  int cycles = 0;
  int status = BMG_OK;
  for (;;) {
    // H1: -R in the correction precision and rho^2
    kt.add(BMG_K_EIGRES, 20 * nnzL + (8.0 + sizeof(T)) * Nd * m + 8 * Nd, 1);
    BMG_TRY(kt.begin(BMG_K_EIGRES));
    BMG_TRY(launch_eigres<T>(DL, w->U, w->theta, -1.0, cyc.f[L], w->rho2part, w->nblk_res, m, s));
    BMG_TRY(kt.end(BMG_K_EIGRES));
    BMG_TRY(launch_colsum(w->rho2part, w->nblk_res, m, w->rho2, s));
    BMG_HIP(hipMemcpyAsync(w->hbuf, w->theta, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    BMG_HIP(hipMemcpyAsync(w->hbuf + m, w->rho2, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    BMG_HIP(hipMemcpyAsync(w->hbuf + 2 * m, w->status, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    BMG_HIP(hipStreamSynchronize(s));
    std::memcpy(theta.data(), w->hbuf, sizeof(double) * m);
    std::memcpy(rho2.data(), w->hbuf + m, sizeof(double) * m);
    int rs3[3] = {0, 0, 0};
    std::memcpy(rs3, w->hbuf + 2 * m, 3 * sizeof(int));
    const int rstat = rs3[0];
    ritz_sweeps_max = std::max(ritz_sweeps_max, rs3[1]);
    ritz_fallbacks += rs3[2];
    if (rstat == 1) {
      set_error("enriched space lost rank below m");
      status = BMG_ENOCONV;
      break;
    }
    bool finite = true;
    for (int j = 0; j < m; ++j) finite = finite && std::isfinite(theta[j]) && std::isfinite(rho2[j]);
    if (!finite) {
      set_error("non-finite Ritz value or residual at cycle %d", cycles);
      status = BMG_ENOCONV;
      cert = certify(theta, rho2, sigma, k, tol, o.angle_tol);
      break;
    }
    cert = certify(theta, rho2, sigma, k, tol, o.angle_tol);
    if (cert.ok) break;
    if (cycles >= o.max_cycles) {
      status = BMG_ENOCONV;
      set_error("no convergence in %d cycles", o.max_cycles);
      break;
    }
    // H2 + H3
    BMG_TRY(cyc.vcycle(L));
    BMG_TRY(launch_add_to<T>(w->U, cyc.e[L], N * m, s));
    // H4-H6
    BMG_TRY(ritz_step());
    ++cycles;
  }

  // ---- output: k pairs nearest sigma, ascending, signs normalised
  std::vector<int> sel = cert.ret;
  std::sort(sel.begin(), sel.end());  // theta is ascending
  for (int j = 0; j < k; ++j) evals[j] = theta[sel[j]];
  if (evecs) {
    BMG_HIP(hipMemcpyAsync(w->sel, sel.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
    BMG_TRY(launch_signs(N, w->U, m, w->sel, k, w->sign, w->argv, w->argi, w->nblk_arg, s));
    if (evecs_on_device) {
      BMG_TRY(launch_write_evecs(N, w->U, m, w->sel, w->sign, k, evecs, ld, s));
    } else {
      BMG_TRY(launch_write_evecs(N, w->U, m, w->sel, w->sign, k, w->AU, N, s));
      BMG_HIP(hipMemcpy2DAsync(evecs, sizeof(double) * ld, w->AU, sizeof(double) * N,
                               sizeof(double) * N, k, hipMemcpyDeviceToHost, s));
    }
  }
  BMG_HIP(hipEventRecord(ev1, s));
  BMG_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  BMG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (stats) {
    stats->cycles = cycles;
    stats->converged = cert.ok ? 1 : 0;
    stats->m = m;
    stats->n_c = n_c;
    stats->l_c = l_c;
    stats->t_solve_ms = ms;
    stats->max_rho_over_delta = cert.max_dk;
    stats->max_kato_temple = cert.max_kt;
    stats->timed_kernel_ms = kt.total_ms();
    stats->timed_kernel_bytes = kt.bytes;
    stats->timed_kernel_units = kt.units;
    stats->ritz_sweeps_max = ritz_sweeps_max;
    stats->ritz_fallbacks = ritz_fallbacks;
    // report in the output order (ascending)
    for (int j = 0; j < k && j < int(cert.ret.size()); ++j) {
      const int pos = int(std::find(cert.ret.begin(), cert.ret.end(), sel[j]) - cert.ret.begin());
      if (stats->rho) stats->rho[j] = cert.rho[pos];
      if (stats->delta) stats->delta[j] = cert.delta[pos];
    }
  }
  return status;
}

}  // namespace

int solve(bmg_hierarchy* h, int k, double sigma, double tol, const bmg_solve_opts* opts,
          double* evals, double* evecs, int64_t ld, int evecs_on_device, void* stream,
          bmg_solve_stats* stats) {
  BMG_CHECK(h != nullptr && evals != nullptr, "hierarchy and evals must be non-NULL");
  bmg_solve_opts o;
  bmg_solve_opts_default(&o);
  if (opts) o = *opts;
  const int nl = int(h->dev.size());
  const int64_t N = h->dev[nl - 1].n;
  BMG_CHECK(k >= 1, "k must be >= 1");
  BMG_CHECK(std::isfinite(sigma), "sigma must be finite");
  BMG_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive and finite");
  if (o.m <= 0) {
    const double fac = sigma == 0.0 ? 1.25 : 1.5;
    o.m = 4 * int(std::ceil(fac * k / 4.0));
  }
  if (o.n_c <= 0) o.n_c = int(std::min<int64_t>(h->n0, 32)) & ~1;
  BMG_CHECK(o.m % 4 == 0, "m = %d must be a multiple of 4", o.m);
  BMG_CHECK(o.m >= k, "m = %d must be >= k = %d", o.m, k);
  BMG_CHECK(int64_t(o.m) <= N / 2, "m = %d must be <= N_L / 2", o.m);
  BMG_CHECK(o.n_c % 2 == 0 && o.n_c >= 2 && o.n_c <= h->n0, "n_c must be even and in [2, N_0]");
  BMG_CHECK(o.n_c + o.m <= 96, "n_c + m = %d exceeds 96", o.n_c + o.m);
  BMG_CHECK(o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 <= 64 && o.nu2 <= 64, "nu1, nu2 must be in [0, 64]");
  BMG_CHECK(o.smoother == BMG_SMOOTH_GS || o.smoother == BMG_SMOOTH_JACOBI, "unknown smoother");
  BMG_CHECK(o.precision == BMG_FP64 || o.precision == BMG_MIXED, "unknown precision");
  BMG_CHECK(o.max_cycles >= 0, "max_cycles must be >= 0");
  BMG_CHECK(o.omega > 0 && o.omega < 2, "omega must be in (0, 2)");
  BMG_CHECK(o.angle_tol > 0, "angle_tol must be positive");
  BMG_CHECK(evecs == nullptr || ld >= N, "ld must be >= N_L");
  const int l_c = o.l_c < 0 ? weyl_coarsest(h, sigma) : o.l_c;
  BMG_CHECK(l_c >= 0 && l_c < nl, "l_c out of range");
  BMG_HIP(hipSetDevice(h->device));
  bmg_workspace* w = nullptr;
  BMG_TRY(acquire_workspace(h, o.m, o.n_c, o.precision, &w));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = (o.precision == BMG_MIXED)
               ? run_solve<float>(h, w, k, sigma, tol, o, l_c, evals, evecs, ld, evecs_on_device, s, stats)
               : run_solve<double>(h, w, k, sigma, tol, o, l_c, evals, evecs, ld, evecs_on_device, s, stats);
  if (st == BMG_EDEVICE || st == BMG_EINVAL) (void)hipStreamSynchronize(s);
  release_workspace(h, w);
  return st;
}

// V-cycle for bmg_apply: uses a temporary workspace.
int apply_vcycle(bmg_hierarchy* h, int level, int dtype, int m, double sigma, int smoother,
                 int nu1, int nu2, int l_c, double omega, const void* x, void* y, hipStream_t s) {
  const int lc = l_c < 0 ? weyl_coarsest(h, sigma) : l_c;
  BMG_CHECK(lc >= 0 && lc <= level, "l_c must be in [0, level]");
  bmg_workspace* w = nullptr;
  const int prec = dtype == 1 ? BMG_MIXED : BMG_FP64;
  const int n_c = int(std::min<int64_t>(h->n0, 32)) & ~1;
  BMG_TRY(make_workspace(h, m, n_c, prec, &w));
  const size_t vb = dtype == 1 ? sizeof(float) : sizeof(double);
  int st = BMG_OK;
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    std::vector<T> g(h->n0);
    for (int64_t i = 0; i < h->n0; ++i) {
      const double xx = h->lam0[i] - sigma;
      g[i] = std::fabs(xx) >= 1e-2 * std::max(1.0, std::fabs(sigma)) ? T(1.0 / xx) : T(0);
    }
    BMG_HIP(hipMemcpyAsync(w->gco, g.data(), sizeof(T) * h->n0, hipMemcpyHostToDevice, s));
    BMG_HIP(hipMemcpyAsync(w->f[level], x, vb * h->dev[level].n * m, hipMemcpyDeviceToDevice, s));
    Cycle<T> cyc;
    cyc.h = h;
    cyc.c = CycleCfg{m, nu1, nu2, smoother, lc, sigma, omega};
    const int nl = int(h->dev.size());
    cyc.e.resize(nl);
    cyc.f.resize(nl);
    cyc.t.resize(nl);
    for (int l = 0; l < nl; ++l) {
      cyc.e[l] = static_cast<T*>(w->e[l]);
      cyc.f[l] = static_cast<T*>(w->f[l]);
      cyc.t[l] = static_cast<T*>(w->t[l]);
    }
    cyc.ctmp = static_cast<T*>(w->ctmp);
    cyc.g0 = static_cast<const T*>(w->gco);
    cyc.s = s;
    BMG_TRY(cyc.vcycle(level));
    BMG_HIP(hipMemcpyAsync(y, cyc.e[level], vb * h->dev[level].n * m, hipMemcpyDeviceToDevice, s));
    BMG_HIP(hipStreamSynchronize(s));
    return BMG_OK;
  };
  st = dtype == 1 ? run(float(0)) : run(double(0));
  free_workspace(w);
  return st;
}

}  // namespace bmg
