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
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <type_traits>

#include "bmg_internal.h"

struct bmg_workspace {
  int64_t N = 0;
  int m = 0, n_c = 0, prec = 0, nl = 0;
  int gram_m = 0;  // widest block the Gram / Ritz buffers serve (m, or less in a grouped solve)
  bool busy = false;
  double *W = nullptr, *AW = nullptr, *MW = nullptr;
  double *U = nullptr, *AU = nullptr, *MU = nullptr;
  std::vector<void*> e, f, t;  // per level, correction precision
  std::vector<void*> S;        // per level: A_l - sigma M_l in the correction precision
  void* tail_img = nullptr;    // packed static arrays of the LDS tail
  std::vector<char> tail_host; // host staging of the image
  void* ctmp = nullptr;        // [N0][m]
  void* gco = nullptr;         // [N0]
  double *gpart = nullptr, *G = nullptr, *GW = nullptr, *Y = nullptr, *theta = nullptr;
  double *rho2part = nullptr, *rho2 = nullptr, *rscratch = nullptr;
  int* status = nullptr;
  int* sel = nullptr;
  double *sign = nullptr, *argv = nullptr;
  int* argi = nullptr;
  double* hbuf = nullptr;  // pinned host: theta[m], rho2[m], status
  double* hbuf_d = nullptr;  // its device-side address (written by k_colsum)
  bmg::TailArgs* tail_h = nullptr;  // pinned host staging of the tail descriptor
  bmg::TailArgs* tail_d = nullptr;  // device copy
  hipStream_t stream = nullptr;     // internal stream (capturable), joined to the caller's
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // cached graph of one cycle (V-cycle, update, Ritz step, next residual)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  double g_sigma = 0, g_omega = 0;
  int g_smoother = -1, g_nu1 = -1, g_nu2 = -1, g_lc = -1, g_tail = -2, g_timed = -1, g_fuse = -1, g_warm = -1;
  int nblk_res = 0, nblk_arg = 0;
  bmg::GramPlan gp{}, gpw{};
  // interior-shift scheme: per-level shifts, the quadratic-form partials they
  // come from, and the coarse solve's scratch (sized for sh_n coarse rows)
  int g_scheme = -1;
  int64_t sh_n = -1;
  double* shifts = nullptr;   // [nl]
  double* rqpart = nullptr;   // [nl][kRqBlocks][2m]
  void* spec_g = nullptr;     // [sh_n] correction precision
  void* spec_t = nullptr;     // [sh_n][m]
  void* spec_part = nullptr;  // [spec_slices(sh_n)][sh_n][m]
  int* csel = nullptr;        // [m] coarse eigenvectors of the start block
  std::vector<void*> allocs;
  int64_t bytes = 0;  // device bytes held by allocs
};

namespace bmg {

thread_local LaunchEvents g_launch_events;
thread_local const std::atomic<int>* g_cancel = nullptr;

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
  w->bytes += int64_t(bytes);
  return BMG_OK;
}

void free_workspace(bmg_workspace* w) {
  DeviceSyncGuard sync;  // stream, graph and pinned-memory teardown synchronise
  if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
  if (w->graph) (void)hipGraphDestroy(w->graph);
  if (w->ev_in) (void)hipEventDestroy(w->ev_in);
  if (w->ev_out) (void)hipEventDestroy(w->ev_out);
  if (w->stream) (void)hipStreamDestroy(w->stream);
  for (void* p : w->allocs) dev_free(p);
  if (w->hbuf) (void)hipHostFree(w->hbuf);
  if (w->tail_h) (void)hipHostFree(w->tail_h);
  delete w;
}

int make_workspace(bmg_hierarchy* h, int m, int n_c, int prec, bmg_workspace** out, int gram_m = 0) {
  auto* w = new bmg_workspace();
  if (gram_m <= 0) gram_m = m;
  w->gram_m = gram_m;
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
  w->S.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const size_t b = vb * h->dev[l].n * m;
    AL(w->e[l], b);
    AL(w->f[l], b);
    AL(w->t[l], b);
    AL(w->S[l], vb * h->dev[l].n * h->dev[l].W);
  }
  AL(w->tail_img, size_t(kTailLdsBudget));
  AL(w->ctmp, vb * h->n0 * m);
  AL(w->gco, vb * h->n0);
  // Gram and Ritz buffers for blocks up to gram_m wide: every plan of a width
  // w <= gram_m fits the partial-sum buffer
  const int nz = n_c + gram_m;
  w->gp = gram_plan(N, nz, 2 * gram_m);
  w->gpw = gram_plan(N, n_c, 2 * n_c);
  size_t gpb = std::max(size_t(w->gp.nblk) * w->gp.per_block, size_t(w->gpw.nblk) * w->gpw.per_block);
  for (int gw = 2; gw < gram_m; gw += 2) {
    const GramPlan q = gram_plan(N, n_c + gw, 2 * gw);
    gpb = std::max(gpb, size_t(q.nblk) * q.per_block);
  }
  AL(w->gpart, sizeof(double) * gpb);
  AL(w->G, sizeof(double) * nz * 2 * gram_m);
  AL(w->GW, sizeof(double) * n_c * 2 * n_c);
  AL(w->Y, sizeof(double) * nz * gram_m);
  // theta [m], rho2 [m] and the Ritz status words [16] are contiguous: one
  // device-to-host copy per cycle reads all three
  AL(w->theta, sizeof(double) * (2 * m + 8));
  w->rho2 = w->theta + m;
  w->status = reinterpret_cast<int*>(w->theta + 2 * m);
  w->nblk_res = eigres_blocks(h->dev[nl - 1], m);
  AL(w->rho2part, sizeof(double) * w->nblk_res * m);
  AL(w->rscratch, sizeof(double) * ritz_scratch_doubles(nz));
  AL(w->sel, sizeof(int) * m);
  AL(w->sign, sizeof(double) * m);
  w->nblk_arg = int(std::min<int64_t>(256, (N + 255) / 256));
  AL(w->argv, sizeof(double) * w->nblk_arg * m);
  AL(w->argi, sizeof(int) * w->nblk_arg * m);
  AL(w->tail_d, sizeof(TailArgs));
#undef AL
  DeviceSyncGuard sync;  // stream, events and pinned memory
  if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    free_workspace(w);
    set_error("stream/event creation failed");
    return BMG_EDEVICE;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&w->tail_h), sizeof(TailArgs)) != hipSuccess) {
    (void)hipGetLastError();
    free_workspace(w);
    set_error("hipHostMalloc failed");
    return BMG_ENOMEM;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&w->hbuf), sizeof(double) * (2 * m + 8)) != hipSuccess) {
    (void)hipGetLastError();
    free_workspace(w);
    set_error("hipHostMalloc failed");
    return BMG_ENOMEM;
  }
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&w->hbuf_d), w->hbuf, 0) != hipSuccess) {
    (void)hipGetLastError();
    w->hbuf_d = nullptr;  // the results are then copied back instead
  }
  *out = w;
  return BMG_OK;
}

int acquire_workspace(bmg_hierarchy* h, int m, int n_c, int prec, bmg_workspace** out, int gram_m = 0) {
  if (gram_m <= 0) gram_m = m;
  {
    std::lock_guard<std::mutex> g(h->ws_mutex);
    for (auto* w : h->ws_pool)
      if (!w->busy && w->m == m && w->n_c == n_c && w->prec == prec && w->gram_m == gram_m) {
        w->busy = true;
        *out = w;
        return BMG_OK;
      }
  }
  bmg_workspace* w = nullptr;
  BMG_TRY(make_workspace(h, m, n_c, prec, &w, gram_m));
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

int64_t idle_workspace_bytes(bmg_hierarchy* h) {
  std::lock_guard<std::mutex> g(h->ws_mutex);
  int64_t b = 0;
  for (auto* w : h->ws_pool)
    if (!w->busy) b += w->bytes;
  return b;
}

void trim_idle_workspaces(bmg_hierarchy* h) {
  std::lock_guard<std::mutex> g(h->ws_mutex);
  std::vector<bmg_workspace*> keep;
  for (auto* w : h->ws_pool) {
    if (w->busy)
      keep.push_back(w);
    else
      free_workspace(w);
  }
  h->ws_pool.swap(keep);
}

// ----------------------------------------------------------- kernel timer --
// Times the launches of one kernel class with HIP events that the launcher
// records at the kernel's own start and end (no queueing inside the interval).
// Eager launches record fresh event pairs; harvest() runs after each
// synchronisation of the solve.
struct KTimer {
  int which = -1;
  int level = -1;  // time only launches on this level (-1: every level)
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double ms = 0.0, bytes = 0.0;
  int64_t units = 0;
  double pend_bytes = 0.0, body_bytes = 0.0;
  int64_t pend_units = 0, body_units = 0;
  bool frozen = false;  // event pairs baked into a graph
  int begin(int k) {
    if (k != which) return BMG_OK;
    if (2 * used + 2 > ev.size()) {
      hipEvent_t a, b;
      BMG_HIP(hipEventCreate(&a));
      BMG_HIP(hipEventCreate(&b));
      ev.push_back(a);
      ev.push_back(b);
    }
    g_launch_events = LaunchEvents{ev[2 * used], ev[2 * used + 1]};
    return BMG_OK;
  }
  int end(int k) {
    if (k != which) return BMG_OK;
    g_launch_events = LaunchEvents{};
    ++used;
    return BMG_OK;
  }
  void add(int k, double b, int64_t u) {
    if (k != which) return;
    pend_bytes += b;
    pend_units += u;
  }
  // the pending amounts and event pairs now belong to a captured graph body
  void freeze() {
    frozen = true;
    body_bytes = pend_bytes;
    body_units = pend_units;
    pend_bytes = 0.0;
    pend_units = 0;
  }
  // drop what a failed capture recorded
  void discard(size_t keep_used) {
    used = keep_used;
    pend_bytes = 0.0;
    pend_units = 0;
  }
  // after a synchronisation: add the completed launches (or graph replay)
  void harvest(bool replayed) {
    if (which < 0) return;
    for (size_t i = 0; i < used; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess)
        ms += t;
      else
        (void)hipGetLastError();  // not a launch error: keep it out of later checks
    }
    if (frozen) {
      if (replayed) {
        bytes += body_bytes;
        units += body_units;
      }
    } else {
      bytes += pend_bytes;
      units += pend_units;
      pend_bytes = 0.0;
      pend_units = 0;
      used = 0;
    }
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
  std::vector<const T*> S;  // A_l - sigma M_l
  T* ctmp;
  const T* g0;  // truncated inverse spectrum at level 0
  hipStream_t s;
  KTimer* kt = nullptr;  // timing of finest-level launches (level L)
  int L = -1;
  int tail_hi = -1;  // levels l_c..tail_hi run in one workgroup, in LDS
  const TailArgs* tail_d = nullptr;
  int tail_lds = 0;
  int tail_groups = 1;  // workgroups of the tail (column groups)
  // set by the caller: the final Jacobi post-sweep of level add_level adds its
  // result to add_u (FP64 n x m); added reports whether that happened
  double* add_u = nullptr;
  int add_level = -1;
  bool added = false;
  bool fuse_ok = std::getenv("BMG_NO_FUSE") == nullptr;  // fused Jacobi cycle kernels
  // coarse solve at l_c by the truncated spectral inverse of a dense level
  // (the interior-shift scheme): eigenvectors one per row, inverse spectrum g
  const T* lc_phi = nullptr;
  const T* lc_g = nullptr;
  T* lc_t = nullptr;
  T* lc_part = nullptr;
  int lc_n = 0;

  // Pack the LDS image of levels l_c..hi (the largest hi whose image and work
  // blocks fit the budget) and upload it with its descriptor.  phi0 and gh are
  // the level-0 eigenvectors and the truncated inverse spectrum (host, FP64).
  int setup_tail(TailArgs* th, TailArgs* td, void* img_d, std::vector<char>& img,
                 const std::vector<double>& phi0, const std::vector<double>& gh, int top) {
    tail_hi = -1;
    if (std::getenv("BMG_NO_TAIL")) return BMG_OK;
    if (c.smoother == BMG_SMOOTH_KACZMARZ) return BMG_OK;  // the LDS tail runs Jacobi and GS
    const int nl = top + 1;
    if (nl > kTailMaxLevels) return BMG_OK;
    auto al = [](size_t x) { return (x + 15) / 16 * 16; };
    const size_t vt = sizeof(T);
    const size_t n0 = size_t(h->n0);
    const bool spectral = c.l_c == 0;
    const size_t stat0 = spectral ? 2 * al(n0 * n0 * vt) + al(n0 * vt) : 0;
    // the highest level whose arrays fit LDS with mc columns per workgroup
    auto top_level = [&](int mc, size_t& stat_out) {
      size_t stat = stat0, work = 0;
      int hi = -1;
      for (int l = c.l_c; l < nl; ++l) {
        const HostLevel& H = h->host[l];
        if (H.n > 32767 || H.n_colours > kTailMaxColours) break;  // 16-bit tables
        const size_t n = size_t(H.n), np = size_t(H.n_prev);
        const size_t st = al(n * H.W * vt) + al(n * H.W * 2) + al(n * 2) + al((n - np) * 4) +
                          al(np * H.RW * 2);
        const size_t wk = 3 * al(n * size_t(mc) * vt);
        if (stat + st + work + wk > size_t(kTailLdsBudget)) break;
        stat += st;
        work += wk;
        hi = l;
      }
      stat_out = stat;
      return hi;
    };
    // columns per workgroup: the most groups (each on its own CU, each phase
    // with fewer items per thread) among those that reach the highest level
    const int vw = int(16 / vt);
    int hi = -1, groups = 1;
    size_t stat = 0;
    for (int g = 1; g <= c.m / vw; g *= 2) {
      if (c.m % g != 0 || (c.m / g) % vw != 0) break;
      size_t st_g = 0;
      const int hg = top_level(c.m / g, st_g);
      if (hg >= hi) {
        hi = hg;
        groups = g;
        stat = st_g;
      }
    }
    if (hi < 0) return BMG_OK;
    const int mc = c.m / groups;
    std::memset(th, 0, sizeof(TailArgs));
    th->lo = c.l_c;
    th->hi = hi;
    th->m = mc;
    th->m_full = c.m;
    th->smoother = c.smoother;
    th->nu1 = c.nu1;
    th->nu2 = c.nu2;
    th->omega = c.omega;
    img.assign(stat, 0);
    size_t pos = 0;
    auto put = [&](const void* src, size_t bytes) {
      const size_t off = pos;
      if (src && bytes) std::memcpy(img.data() + off, src, bytes);
      pos += al(bytes);
      return int(off);
    };
    for (int l = c.l_c; l <= hi; ++l) {
      const HostLevel& H = h->host[l];
      TailLevel& t = th->lv[l];
      t.n = int(H.n);
      t.n_prev = int(H.n_prev);
      t.W = H.W;
      t.RW = H.RW;
      t.n_colours = H.n_colours;
      for (int k = 0; k <= H.n_colours; ++k) t.colour_ptr[k] = H.colour_ptr[k];
      t.off_S = put(nullptr, size_t(H.n) * H.W * vt);  // filled on the device
      std::vector<uint16_t> u16(H.cols.begin(), H.cols.end());
      t.off_cols = put(u16.data(), u16.size() * 2);
      u16.assign(H.colour_rows.begin(), H.colour_rows.end());
      t.off_crow = put(u16.data(), u16.size() * 2);
      u16.assign(H.parents.begin(), H.parents.end());
      t.off_par = put(u16.data(), u16.size() * 2);
      std::vector<int16_t> i16(H.rtab.begin(), H.rtab.end());
      t.off_rtab = put(i16.data(), i16.size() * 2);
    }
    th->off_phi = th->off_phit = th->off_g = -1;
    if (spectral) {
      std::vector<T> p(n0 * n0), pt(n0 * n0), g(n0);
      for (size_t i = 0; i < n0; ++i)
        for (size_t j = 0; j < n0; ++j) {
          p[i * n0 + j] = T(phi0[i * n0 + j]);
          pt[j * n0 + i] = T(phi0[i * n0 + j]);
        }
      for (size_t i = 0; i < n0; ++i) g[i] = T(gh[i]);
      th->off_phi = put(p.data(), p.size() * vt);
      th->off_phit = put(pt.data(), pt.size() * vt);
      th->off_g = put(g.data(), g.size() * vt);
    }
    th->image_bytes = int(pos);
    for (int l = c.l_c; l <= hi; ++l) {
      const size_t b = al(size_t(h->host[l].n) * mc * vt);
      TailLevel& t = th->lv[l];
      t.off_e = int(pos);
      pos += b;
      t.off_f = int(pos);
      pos += b;
      t.off_t = int(pos);
      pos += b;
    }
    th->image = img_d;
    th->f_top = f[hi];
    th->e_top = e[hi];
    tail_lds = int(pos);
    BMG_HIP(hipMemcpyAsync(img_d, img.data(), img.size(), hipMemcpyHostToDevice, s));
    for (int l = c.l_c; l <= hi; ++l)
      BMG_HIP(hipMemcpyAsync(static_cast<char*>(img_d) + th->lv[l].off_S, S[l],
                             size_t(h->host[l].n) * h->host[l].W * vt, hipMemcpyDeviceToDevice, s));
    BMG_HIP(hipMemcpyAsync(td, th, sizeof(TailArgs), hipMemcpyHostToDevice, s));
    // img and th are host staging reused by the next solve
    BMG_HIP(hipStreamSynchronize(s));
    tail_hi = hi;
    tail_groups = groups;
    tail_d = td;
    return BMG_OK;
  }

  // the class to time for a launch on level l (-2: not timed)
  int kclass(int k, int l) const { return kt && (kt->level < 0 || kt->level == l) ? k : -2; }

  // last: the cycle's final post-sweep on its top level, which (Jacobi, with
  // add_u set) adds its result to add_u instead of writing e[l]
  int sweep(int l, bool forward, bool from_zero, bool last = false) {
    const DevLevel& D = h->dev[l];
    const HostLevel& H = h->host[l];
    const double b = sizeof(T), n = double(D.n);
    if (c.smoother == BMG_SMOOTH_JACOBI) {
      const bool fold = last && !from_zero && add_u != nullptr && l == add_level;
      const int kc = from_zero ? -2 : kclass(fold ? BMG_K_SMOOTH_ADD : BMG_K_SMOOTH, l);
      if (kt)
        kt->add(kc, fold ? (4 + b) * double(H.nnz) + 2 * b * n * c.m + 16.0 * n * c.m
                         : (4 + b) * double(H.nnz) + 3 * b * n * c.m, 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_jacobi<T>(D, S[l], c.omega, e[l], f[l], t[l], from_zero, c.m, s, fold ? add_u : nullptr));
      if (kt) BMG_TRY(kt->end(kc));
      // the roles swap as after any sweep (with fold, e[l] then holds no
      // result: the correction is in add_u), so a cycle's swaps stay even
      std::swap(e[l], t[l]);
      if (fold) added = true;
      return BMG_OK;
    }
    if (from_zero) BMG_TRY(launch_fill<T>(e[l], D.n * c.m, T(0), s));
    const int kc = kclass(BMG_K_SMOOTH, l);
    if (c.smoother == BMG_SMOOTH_KACZMARZ) {
      for (int k = 0; k < D.n_colours2; ++k) {
        const int col = forward ? k : D.n_colours2 - 1 - k;
        const double nk = double(H.colour2_ptr[col + 1] - H.colour2_ptr[col]);
        // ELL row (index + value) of each row of the colour, f and the gathered
        // neighbour rows of x, and the neighbour rows written back
        if (kt) kt->add(kc, (4 + b) * H.W * nk + b * c.m * nk * (1 + 2 * H.W), 1);
        if (kt) BMG_TRY(kt->begin(kc));
        BMG_TRY(launch_kaczmarz_colour<T>(D, S[l], col, e[l], f[l], c.m, s));
        if (kt) BMG_TRY(kt->end(kc));
      }
      return BMG_OK;
    }
    for (int k = 0; k < D.n_colours; ++k) {
      const int col = forward ? k : D.n_colours - 1 - k;
      const double nk = double(H.colour_ptr[col + 1] - H.colour_ptr[col]);
      if (kt) kt->add(kc, (4 + b) * H.W * nk + b * c.m * (n + 2 * nk), 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_gs_colour<T>(D, S[l], col, e[l], f[l], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
    }
    return BMG_OK;
  }

  // e[l] <- B_sigma f[l]
  int vcycle(int l) {
    const DevLevel& D = h->dev[l];
    if (l == tail_hi) return launch_tail<T>(tail_d, tail_lds, tail_groups, s);
    if (l == c.l_c) {
      if (lc_phi) return launch_spec_apply<T>(lc_n, lc_phi, lc_g, f[l], lc_t, lc_part, e[l], c.m, s);
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
    const double b = sizeof(T);
    const double nnz = double(h->host[l].nnz), n = double(D.n), nc = double(D.n_prev);
    constexpr double kFuseMaxBlock = 24.0 * (1 << 20);
    // weighted Jacobi: the zero-start pair of pre-sweeps, the residual with its
    // restriction, and the prolongation with the first post-sweep each run as
    // one fused kernel (same arithmetic, identical results).  Fusion saves
    // launches and block round trips but recomputes residual rows and gathers
    // the coarse correction per neighbour, so it pays while the level's blocks
    // are small (launch- and latency-bound) and is skipped on levels whose
    // blocks exceed kFuseMaxBlock bytes (bandwidth-bound).
    const bool fuse = c.smoother == BMG_SMOOTH_JACOBI && fuse_ok &&
                      double(D.n) * c.m * b <= kFuseMaxBlock;
    int k0 = 0;
    if (fuse && c.nu1 >= 2) {
      const int kc = kclass(BMG_K_SMOOTH_PAIR, l);
      if (kt) kt->add(kc, (4 + b) * nnz + 2 * b * n * c.m, 1);
      if (kt) BMG_TRY(kt->begin(kc));
      // reads only f, so it writes the iterate in place (no buffer swap)
      BMG_TRY(launch_jacobi2z<T>(D, S[l], c.omega, f[l], e[l], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
      k0 = 2;
    }
    for (int k = k0; k < c.nu1; ++k) BMG_TRY(sweep(l, true, k == 0));
    if (c.nu1 == 0) BMG_TRY(launch_fill<T>(e[l], D.n * c.m, T(0), s));
    if (fuse) {
      const int kc = kclass(BMG_K_RESTRICT_RES, l);
      if (kt) kt->add(kc, (4 + b) * nnz + 2 * b * n * c.m + b * nc * c.m + 4.0 * nc * D.RW, 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_resrestrict<T>(D, S[l], e[l], f[l], f[l - 1], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
    } else {
      int kc = kclass(BMG_K_RESIDUAL, l);
      if (kt) kt->add(kc, (4 + b) * nnz + 3 * b * n * c.m, 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_shifted<T>(D, S[l], ROW_RESIDUAL, e[l], f[l], t[l], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
      kc = kclass(BMG_K_RESTRICT, l);
      if (kt) kt->add(kc, b * n * c.m + b * nc * c.m + 4.0 * nc * D.RW, 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_restrict<T>(D, t[l], f[l - 1], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
    }
    BMG_TRY(vcycle(l - 1));
    if (fuse && c.nu2 >= 1) {
      const int kc = kclass(BMG_K_PROLONG_SMOOTH, l);
      if (kt) kt->add(kc, (4 + b) * nnz + 3 * b * n * c.m + b * nc * c.m + 8.0 * (n - nc), 1);
      if (kt) BMG_TRY(kt->begin(kc));
      BMG_TRY(launch_prolong_jacobi<T>(D, S[l], c.omega, e[l], e[l - 1], f[l], t[l], c.m, s));
      if (kt) BMG_TRY(kt->end(kc));
      std::swap(e[l], t[l]);
      for (int k = 1; k < c.nu2; ++k) BMG_TRY(sweep(l, false, false, k == c.nu2 - 1));
      return BMG_OK;
    }
    const int kc = kclass(BMG_K_PROLONG, l);
    if (kt) kt->add(kc, b * nc * c.m + 2 * b * n * c.m + 8.0 * (n - nc), 1);
    if (kt) BMG_TRY(kt->begin(kc));
    BMG_TRY(launch_prolong_add<T>(D, e[l - 1], e[l], c.m, s));
    if (kt) BMG_TRY(kt->end(kc));
    for (int k = 0; k < c.nu2; ++k) BMG_TRY(sweep(l, false, false, k == c.nu2 - 1));
    return BMG_OK;
  }
};

// Truncated inverse spectrum of the level-0 pencil (Alg. 2 step 1, with the
// near-singular modes dropped): g_i = 1/(lambda_i - sigma), 0 when
// |lambda_i - sigma| < 1e-2 max(1, |sigma|).
std::vector<double> coarse_inverse(const bmg_hierarchy* h, double sigma) {
  std::vector<double> g(h->n0);
  for (int64_t i = 0; i < h->n0; ++i) {
    const double x = h->lam0[i] - sigma;
    g[i] = std::fabs(x) >= 1e-2 * std::max(1.0, std::fabs(sigma)) ? 1.0 / x : 0.0;
  }
  return g;
}

// Bind a cycle to the workspace buffers, form S_l = A_l - sigma M_l on every
// level up to `top`, upload the level-0 inverse and set up the LDS tail.
template <typename T>
int init_cycle(Cycle<T>& cyc, bmg_hierarchy* h, bmg_workspace* w, const CycleCfg& cfg, int top,
               hipStream_t s, bool allow_tail = true) {
  const int nl = int(h->dev.size());
  cyc.h = h;
  cyc.c = cfg;
  cyc.s = s;
  cyc.e.resize(nl);
  cyc.f.resize(nl);
  cyc.t.resize(nl);
  cyc.S.resize(nl);
  for (int l = 0; l < nl; ++l) {
    cyc.e[l] = static_cast<T*>(w->e[l]);
    cyc.f[l] = static_cast<T*>(w->f[l]);
    cyc.t[l] = static_cast<T*>(w->t[l]);
    cyc.S[l] = static_cast<const T*>(w->S[l]);
  }
  for (int l = 0; l <= top; ++l) BMG_TRY(launch_shift<T>(h->dev[l], cfg.sigma, static_cast<T*>(w->S[l]), s));
  cyc.ctmp = static_cast<T*>(w->ctmp);
  cyc.g0 = static_cast<const T*>(w->gco);
  const std::vector<double> gh = coarse_inverse(h, cfg.sigma);
  std::vector<T> g(gh.begin(), gh.end());
  BMG_HIP(hipMemcpyAsync(w->gco, g.data(), sizeof(T) * g.size(), hipMemcpyHostToDevice, s));
  if (allow_tail) BMG_TRY(cyc.setup_tail(w->tail_h, w->tail_d, w->tail_img, w->tail_host, h->phi0, gh, top));
  BMG_HIP(hipStreamSynchronize(s));  // g is a host local
  return BMG_OK;
}

int default_block_width(int k, double sigma) {
  const double fac = sigma == 0.0 ? 1.25 : 1.5;
  return 4 * int(std::ceil(fac * k / 4.0));
}

int default_coarse_vectors(const bmg_hierarchy* h) { return int(std::min<int64_t>(h->n0, 32)) & ~1; }

// The block must hold whole clusters of the spectrum plus overlap (Sec. 4,
// the choice of Lambda: multiplicities and the gap between clusters).  Given
// a coarse level's eigenvalues lam, which place the clusters near sigma, the
// default width m is widened until the first eigenvalue left out lies at
// least 1.25 times as far from sigma as the k-th nearest: the block then
// converges the k-th pair at a ratio of at most 0.8 per cycle even when k
// cuts a cluster (the sphere's multiplets, a nearly round ellipsoid's split
// ones), where a block ending inside the cluster barely converges at all.
// A multiple of 4, at most m_cap; unchanged if the coarse spectrum does not
// reach past the window.
int widen_block_width(const std::vector<double>& lam, int k, double sigma, int m, int m_cap) {
  if (k < 1 || int(lam.size()) <= k) return m;
  std::vector<double> d(lam.size());
  for (size_t i = 0; i < lam.size(); ++i) d[i] = std::fabs(lam[i] - sigma);
  std::sort(d.begin(), d.end());
  const double dk = d[size_t(k) - 1];
  size_t c = 0;
  while (c < d.size() && d[c] < 1.25 * dk) ++c;
  if (c >= d.size()) return m;
  const int want = 4 * ((int(c) + 3) / 4);
  return std::max(m, std::min(want, m_cap));
}

int block_width_cap(const bmg_hierarchy* h, int n_c, bool shifted, int l_c) {
  int64_t cap = std::min<int64_t>(96 - n_c, h->host.back().n / 2);
  if (shifted) cap = std::min<int64_t>(cap, h->host[l_c].n / 2);
  return int(cap / 4 * 4);
}

// The default width widened by widen_block_width on the spectrum of level l_c
// (interior scheme: the level it eigendecomposes anyway) or of the coarsest
// level with at least max(4 m, 96) vertices (enriched scheme: it places the
// clusters up to a few times the default width, and a new hierarchy pays for
// only a small dense eigensolve); kept as it is if no such level fits the
// dense eigensolve.
int widened_default_width(bmg_hierarchy* h, int k, double sigma, bool shifted, int l_c, int n_c,
                          hipStream_t s, int* m) {
  const int nl = int(h->host.size());
  int g = -1;
  if (shifted) {
    g = l_c;
  } else {
    const int64_t need = std::max(4 * int64_t(*m), int64_t(96));
    for (int l = 0; l < nl && g < 0; ++l)
      if (h->host[l].n >= need && h->host[l].n <= kLevelEigMax) g = l;
  }
  const int cap = block_width_cap(h, n_c, shifted, l_c);
  if (g < 0 || cap <= *m) return BMG_OK;
  const LevelEig* le = nullptr;
  BMG_TRY(level_eig(h, g, s, &le));
  *m = widen_block_width(le->lam, k, sigma, *m, cap);
  return BMG_OK;
}

// Coarse level of the interior-shift scheme.  The P1 eigenvalue error of an
// eigenfunction near sigma on level l is O(sigma^2 h^2) (the a priori estimate
// of Sec. 2.2, Lemma 2.2) with h the mesh size along it, and a block of m vectors spans a
// window of about 2 pi m / |Gamma_h| around sigma; the coarse solve must place
// the eigenvalues near sigma within a fixed multiple of that window.  With the
// longest edge h_max,l (which bounds the spread over directions on stretched
// grids such as the torus's) the rule is: the coarsest l with
//   sigma^2 h_max,l^2 |Gamma_h| / m <= 60   and   N_l >= 2 m
// (the level must hold twice the start block's eigenpairs).  The constant was
// measured: the ellipsoid (1, 1.5, 2) at sigma = 40..100 and the 64 x 32 torus
// grid at sigma = 84..138 converge in 18-41 cycles at values 39-80, weighted
// Jacobi on the torus grid slows to 127-155 cycles at 79, and the cycle
// stalls at 156 and above.  Levels above kLevelEigMax vertices are not
// eigendecomposed: if the rule needs one, the finest level within the cap is
// used and, when m was not given, m is raised to meet the rule there (a
// multiple of 4, at most 96).
constexpr double kShiftResolution = 60.0;

int shifted_coarse_level(const bmg_hierarchy* h, double sigma, int& m, bool m_given) {
  const int nl = int(h->host.size());
  const double area = h->host[nl - 1].area;
  auto q = [&](int l, int mm) {
    const double hm = h->host[l].hmax;
    return sigma * sigma * hm * hm * area / mm;
  };
  int cap = 0;
  for (int l = 0; l < nl; ++l)
    if (h->host[l].n <= kLevelEigMax) cap = l;
  for (int l = 0; l < nl; ++l)
    if (q(l, m) <= kShiftResolution && h->host[l].n >= 2 * m) {
      if (l <= cap) return l;
      break;
    }
  if (!m_given && cap < nl - 1) {
    const double hm = h->host[cap].hmax;
    const int want = 4 * int(std::ceil(sigma * sigma * hm * hm * area / kShiftResolution / 4.0));
    m = std::min({96, std::max(m, want), int(h->host[cap].n / 2) / 4 * 4});
  }
  return cap;
}

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
              const bmg_solve_opts& o, int l_c, const LevelEig* lce, const LevelEig* lre, double* evals,
              double* evecs, int64_t ld, int evecs_on_device, hipStream_t s, bmg_solve_stats* stats) {
  const int nl = int(h->dev.size());
  const int L = nl - 1;
  const DevLevel& DL = h->dev[L];
  const int64_t N = DL.n;
  const int m = o.m, n_c = o.n_c, nz = n_c + m;
  const int64_t n0 = h->n0;
  // interior-shift scheme: no fixed coarse vectors, per-level shifts, the
  // spectral inverse of level l_c as the coarse solve, coarse start block
  const bool shifted = lce != nullptr;
  hipEvent_t ev0, ev1;
  BMG_HIP(hipEventCreate(&ev0));
  BMG_HIP(hipEventCreate(&ev1));
  BMG_HIP(hipEventRecord(ev0, s));
  if (shifted && w->sh_n < lce->n) {
    // scratch of the coarse solve and the shift estimates (kept by the
    // workspace for later solves)
    const size_t vb = sizeof(T);
    const size_t n = size_t(lce->n);
    if (dalloc(w, reinterpret_cast<void**>(&w->shifts), sizeof(double) * nl) != BMG_OK ||
        dalloc(w, reinterpret_cast<void**>(&w->rqpart), sizeof(double) * nl * kRqBlocks * 2 * m) != BMG_OK ||
        dalloc(w, &w->spec_g, vb * n) != BMG_OK || dalloc(w, &w->spec_t, vb * n * m) != BMG_OK ||
        dalloc(w, &w->spec_part, vb * n * m * spec_slices(int(n))) != BMG_OK ||
        dalloc(w, reinterpret_cast<void**>(&w->csel), sizeof(int) * m) != BMG_OK)
      return BMG_ENOMEM;
    w->sh_n = lce->n;
  }

  // ---- S2: W_c = P_{0->top} Phi_c and its Gram blocks on level top (top = L
  // but for the levels of a ramp)
  auto build_wc = [&](int top) -> int {
    std::vector<int> idx = nearest(h->lam0, sigma, n_c);
    std::sort(idx.begin(), idx.end());
    std::vector<double> phic(size_t(n0) * n_c);
    for (int64_t i = 0; i < n0; ++i)
      for (int j = 0; j < n_c; ++j) phic[size_t(i) * n_c + j] = h->phi0[size_t(i) * n0 + idx[j]];
    double* cur = (top % 2 == 0) ? w->W : w->AW;  // ping-pong so the last lands in W
    BMG_HIP(hipMemcpyAsync(cur, phic.data(), sizeof(double) * phic.size(), hipMemcpyHostToDevice, s));
    for (int l = 1; l <= top; ++l) {
      double* nxt = (cur == w->W) ? w->AW : w->W;
      BMG_TRY(launch_fill<double>(nxt, h->dev[l].n * n_c, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(h->dev[l], cur, nxt, n_c, s));
      cur = nxt;
    }
    const DevLevel& D = h->dev[top];
    BMG_TRY(launch_spmm_am(D, w->W, w->AW, w->MW, n_c, s));
    const GramPlan gpw = top == L ? w->gpw : gram_plan(D.n, n_c, 2 * n_c);
    BMG_TRY(launch_gram(gpw, D.n, w->W, n_c, nullptr, 0, w->AW, n_c, w->MW, n_c, w->gpart, w->GW, s));
    BMG_HIP(hipStreamSynchronize(s));  // phic is a host local
    return BMG_OK;
  };
  const bool ramp = lre != nullptr;
  if (!shifted && !ramp) BMG_TRY(build_wc(L));

  // ---- S3: test vectors and the first Rayleigh-Ritz step (the interior
  // scheme starts from coarse eigenvectors further below unless a block is given)
  if (ramp) {
    // the ramp below fills U
  } else if (o.initial_block) {
    // the caller's block is in vertex order; the level's storage may not be
    double* dst = DL.perm != nullptr ? w->AU : w->U;
    BMG_HIP(hipMemcpyAsync(dst, o.initial_block, sizeof(double) * N * m, hipMemcpyHostToDevice, s));
    if (DL.perm != nullptr) BMG_TRY(launch_permute_rows<double>(N, m, DL.perm, w->AU, w->U, s));
  } else if (!shifted) {
    BMG_TRY(launch_gaussian(w->U, N, m, o.seed, s, DL.perm));
  }

  KTimer kt;
  // timed_kernel = class, or class + 256 (l + 1) for the launches on level l only
  kt.which = o.timed_kernel < 0 ? -1 : (o.timed_kernel & 255);
  kt.level = o.timed_kernel < 0 ? -1 : (o.timed_kernel >> 8) - 1;
  kt.s = s;
  const double nnzL = double(h->host[L].nnz), Nd = double(N);
  int ritz_sweeps_max = 0, ritz_fallbacks = 0;
  RitzArgs ra;
  ra.n_c = n_c;
  ra.m = m;
  ra.nz = nz;
  ra.sigma = sigma;
  ra.rtol2 = kRitzRtol2;
  if (const char* e = std::getenv("BMG_RITZ_RTOL")) ra.rtol2 = std::atof(e) * std::atof(e);
  // U += E in the cycle's last Jacobi sweep (BMG_NO_FUSE keeps it separate)
  const bool fold_add = std::getenv("BMG_NO_FUSE") == nullptr;
  // the first Ritz step of a solve starts cold; later ones may reuse the
  // coarse-block basis the previous step left (BMG_NO_WARM turns this off)
  const int warm_ok = std::getenv("BMG_NO_WARM") ? 0 : 1;
  ra.warm = 0;
  ra.G = w->G;
  ra.GW = w->GW;
  ra.Y = w->Y;
  ra.theta = w->theta;
  ra.scratch = w->rscratch;
  ra.status = w->status;
  auto ritz_step = [&]() -> int {
    // H4: A U', M U' and the Gram blocks of Z = [W_c, U'] in one fused pass
    // flops of the needed outputs: W^T [A U', M U'] and one triangle of each
    // symmetric block (U'^T A U', U'^T M U')
    kt.add(BMG_K_GRAM, 2.0 * Nd * (2.0 * n_c * m + double(m) * (m + 1)), 1);
    BMG_TRY(kt.begin(BMG_K_GRAM));
    BMG_TRY(launch_gram_am(w->gp, DL, w->W, n_c, w->U, m, w->gpart, w->G, s));
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
  if (!ramp && (!shifted || o.initial_block)) BMG_TRY(ritz_step());
  ra.warm = warm_ok;

  Cycle<T> cyc;
  BMG_TRY(init_cycle<T>(cyc, h, w, CycleCfg{m, o.nu1, o.nu2, o.smoother, l_c, sigma, o.omega}, L, s,
                        !shifted));
  cyc.kt = o.timed_kernel >= 0 ? &kt : nullptr;
  cyc.L = L;
  // truncation of the coarse inverse spectrum (as at level 0)
  const double spec_tau = 1e-2 * std::max(1.0, std::fabs(sigma));
  if (shifted) {
    cyc.lc_phi = std::is_same<T, float>::value ? reinterpret_cast<const T*>(lce->d_phi32)
                                               : reinterpret_cast<const T*>(lce->d_phi64);
    cyc.lc_g = static_cast<const T*>(w->spec_g);
    cyc.lc_t = static_cast<T*>(w->spec_t);
    cyc.lc_part = static_cast<T*>(w->spec_part);
    cyc.lc_n = lce->n;
  }
  // shifts of levels l_c..L from the current block (Remark 4.1), the shifted
  // operators and the coarse inverse spectrum that depend on them
  auto adapt_shifts = [&]() -> int {
    BMG_TRY(launch_offsets(h->dev, l_c, L, w->U, m, sigma, w->theta, w->rqpart, w->shifts, s));
    for (int l = l_c + 1; l <= L; ++l)
      BMG_TRY(launch_shift_dev<T>(h->dev[l], w->shifts + l, static_cast<T*>(w->S[l]), s));
    BMG_TRY(launch_spec_g<T>(lce->n, lce->d_lam, w->shifts + l_c, spec_tau, static_cast<T*>(w->spec_g), s));
    return BMG_OK;
  };
  std::vector<double> shifts_h(nl, sigma);
  if (shifted) {
    BMG_HIP(hipMemcpyAsync(w->shifts, shifts_h.data(), sizeof(double) * nl, hipMemcpyHostToDevice, s));
    BMG_TRY(launch_spec_g<T>(lce->n, lce->d_lam, w->shifts + l_c, spec_tau, static_cast<T*>(w->spec_g), s));
    BMG_HIP(hipStreamSynchronize(s));  // shifts_h is read by the copy
  }
  // Start of the interior scheme (Alg. 2 steps 2-4, Alg. 4 step 1): the m
  // level-l_c eigenvectors nearest sigma + off (off: the level's offset),
  // prolongated to level L, one relaxation of the source problem with their
  // eigenvalues shifted back by off as Theta, and a Ritz step in their span.
  std::vector<double> theta0(m);
  std::vector<int> csel;
  auto start = [&](double off) -> int {
    csel = nearest(lce->lam, sigma + off, m);
    BMG_CHECK(int(csel.size()) == m, "level %d has fewer than m = %d eigenpairs", l_c, m);
    std::sort(csel.begin(), csel.end());
    for (int j = 0; j < m; ++j) theta0[j] = lce->lam[csel[j]] - off;
    BMG_HIP(hipMemcpyAsync(w->csel, csel.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
    BMG_HIP(hipMemcpyAsync(w->theta, theta0.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    double* cur = ((L - l_c) % 2 == 0) ? w->U : w->AU;  // ping-pong so the last lands in U
    BMG_TRY(launch_gather_rows(lce->n, m, lce->d_phi64, w->csel, cur, s));
    for (int l = l_c + 1; l <= L; ++l) {
      double* nxt = (cur == w->U) ? w->AU : w->U;
      BMG_TRY(launch_fill<double>(nxt, h->dev[l].n * m, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(h->dev[l], cur, nxt, m, s));
      cur = nxt;
    }
    if (l_c < L) {
      BMG_TRY(launch_eigres<T>(DL, w->U, w->theta, -1.0, cyc.f[L], w->rho2part, w->nblk_res, m, s));
      cyc.add_u = nullptr;
      cyc.added = false;
      BMG_TRY(cyc.vcycle(L));
      BMG_TRY(launch_add_to<T>(w->U, cyc.e[L], N * m, s));
    }
    BMG_TRY(ritz_step());
    BMG_HIP(hipStreamSynchronize(s));  // csel and theta0 are read by the copies
    return BMG_OK;
  };
  // ---- Level ramp (BFMG, Alg. 4): the exact pairs of level l0 nearest sigma
  // (step 1), then on every level l0 < lev < L the block prolongated from the
  // level below, a Ritz step and ramp_cycles cycles of the level's own cycle
  // (step 2: the V-cycle between level lev and the coarse end), recording the
  // k values nearest sigma after each level (step 3); level L then continues
  // as the solve's own loop.  Plain launches; the Ritz warm start is off.
  std::vector<double> ramp_rows;
  int ramp_l0 = -1;
  if (ramp) {
    TraceRange trace("bmg_solve: level ramp");
    ramp_l0 = lre->level;
    ramp_rows.assign(size_t(nl) * k, std::nan(""));
    const int warm_saved = ra.warm;
    ra.warm = 0;
    auto ritz_on = [&](int lev) -> int {
      const DevLevel& D = h->dev[lev];
      const GramPlan gp = lev == L ? w->gp : gram_plan(D.n, nz, 2 * m);
      BMG_TRY(launch_gram_am(gp, D, w->W, n_c, w->U, m, w->gpart, w->G, s));
      BMG_TRY(launch_ritz(ra, s));
      BMG_TRY(launch_update_zy(D.n, w->W, n_c, w->U, m, w->Y, w->U, m, s));
      return BMG_OK;
    };
    auto record = [&](int lev) -> int {
      std::vector<double> buf(2 * m + 8);
      BMG_HIP(hipMemcpyAsync(buf.data(), w->theta, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, s));
      BMG_HIP(hipStreamSynchronize(s));
      int rs0 = 0;
      std::memcpy(&rs0, buf.data() + 2 * m, sizeof(int));
      if (rs0 == 1) {
        set_error("the block lost rank below m on level %d of the ramp", lev);
        return BMG_ENOCONV;
      }
      std::vector<double> th(buf.begin(), buf.begin() + m);
      std::vector<int> sel = nearest(th, sigma, k);
      std::sort(sel.begin(), sel.end());
      for (int j = 0; j < k && j < int(sel.size()); ++j) ramp_rows[size_t(lev) * k + j] = th[sel[j]];
      return BMG_OK;
    };
    // step 1: level l0's own eigenpairs nearest sigma
    {
      std::vector<int> sel = nearest(lre->lam, sigma, m);
      BMG_CHECK(int(sel.size()) == m, "level %d has fewer than m = %d eigenpairs", ramp_l0, m);
      std::sort(sel.begin(), sel.end());
      BMG_HIP(hipMemcpyAsync(w->sel, sel.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
      BMG_TRY(launch_gather_rows(lre->n, m, lre->d_phi64, w->sel, w->U, s));
      BMG_HIP(hipStreamSynchronize(s));  // sel is a host local
    }
    for (int lev = ramp_l0; lev < L; ++lev) {
      const DevLevel& D = h->dev[lev];
      if (lev > ramp_l0) {
        // prolongate the block from level lev - 1
        BMG_TRY(launch_fill<double>(w->AU, D.n * m, 0.0, s));
        BMG_TRY(launch_prolong_add<double>(D, w->U, w->AU, m, s));
        BMG_HIP(hipMemcpyAsync(w->U, w->AU, sizeof(double) * D.n * m, hipMemcpyDeviceToDevice, s));
      }
      if (!shifted) BMG_TRY(build_wc(lev));
      BMG_TRY(ritz_on(lev));
      for (int c = 0; lev > ramp_l0 && c < o.ramp_cycles; ++c) {
        if (shifted) {
          BMG_TRY(launch_offsets(h->dev, l_c, lev, w->U, m, sigma, w->theta, w->rqpart, w->shifts, s));
          for (int l = l_c + 1; l <= lev; ++l)
            BMG_TRY(launch_shift_dev<T>(h->dev[l], w->shifts + l, static_cast<T*>(w->S[l]), s));
          BMG_TRY(launch_spec_g<T>(lce->n, lce->d_lam, w->shifts + l_c, spec_tau, static_cast<T*>(w->spec_g), s));
        }
        BMG_TRY(launch_eigres<T>(D, w->U, w->theta, -1.0, cyc.f[lev], w->rho2part, eigres_blocks(D, m), m, s));
        cyc.add_u = fold_add ? w->U : nullptr;
        cyc.add_level = lev;
        cyc.added = false;
        BMG_TRY(cyc.vcycle(lev));
        if (!cyc.added) BMG_TRY(launch_add_to<T>(w->U, cyc.e[lev], D.n * m, s));
        BMG_TRY(ritz_on(lev));
      }
      BMG_TRY(record(lev));
    }
    // on to level L: prolongate, the fine coarse vectors, a Ritz step
    if (ramp_l0 < L) {
      BMG_TRY(launch_fill<double>(w->AU, N * m, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(DL, w->U, w->AU, m, s));
      BMG_HIP(hipMemcpyAsync(w->U, w->AU, sizeof(double) * N * m, hipMemcpyDeviceToDevice, s));
    }
    if (!shifted) BMG_TRY(build_wc(L));
    if (shifted) {
      // the shifts and operators of the finest level's cycles start from sigma again
      BMG_HIP(hipMemcpyAsync(w->shifts, shifts_h.data(), sizeof(double) * nl, hipMemcpyHostToDevice, s));
      for (int l = l_c + 1; l <= L; ++l)
        BMG_TRY(launch_shift_dev<T>(h->dev[l], w->shifts + l, static_cast<T*>(w->S[l]), s));
      BMG_TRY(launch_spec_g<T>(lce->n, lce->d_lam, w->shifts + l_c, spec_tau, static_cast<T*>(w->spec_g), s));
      BMG_HIP(hipStreamSynchronize(s));
    }
    BMG_TRY(ritz_step());
    ra.warm = warm_saved;
  } else if (shifted && !o.initial_block) {
    TraceRange trace("bmg_solve: start");
    BMG_TRY(start(0.0));
    if (l_c < L) {
      BMG_TRY(adapt_shifts());
      BMG_HIP(hipMemcpyAsync(shifts_h.data(), w->shifts, sizeof(double) * nl, hipMemcpyDeviceToHost, s));
      BMG_HIP(hipStreamSynchronize(s));
      BMG_TRY(start(shifts_h[l_c] - sigma));
    }
  }

  std::vector<double> theta(m), rho2(m);
  Cert cert;
  int cycles = 0;
  int status = BMG_OK;
  // H1: -R in the correction precision and rho^2 (feeds the next decision)
  auto residual_step = [&]() -> int {
    kt.add(BMG_K_EIGRES, 20 * nnzL + (8.0 + sizeof(T)) * Nd * m + 8 * Nd, 1);
    BMG_TRY(kt.begin(BMG_K_EIGRES));
    BMG_TRY(launch_eigres<T>(DL, w->U, w->theta, -1.0, cyc.f[L], w->rho2part, w->nblk_res, m, s));
    BMG_TRY(kt.end(BMG_K_EIGRES));
    BMG_TRY(launch_colsum(w->rho2part, w->nblk_res, m, w->rho2, s, w->theta, w->hbuf_d));
    return BMG_OK;
  };
  // H2-H6 followed by the next H1: the same launches every cycle
  auto cycle_body = [&]() -> int {
    if (shifted) BMG_TRY(adapt_shifts());
    // U += E: folded into the cycle's last sweep when that is a Jacobi sweep
    cyc.add_u = fold_add ? w->U : nullptr;
    cyc.add_level = L;
    cyc.added = false;
    BMG_TRY(cyc.vcycle(L));
    if (!cyc.added) BMG_TRY(launch_add_to<T>(w->U, cyc.e[L], N * m, s));
    BMG_TRY(ritz_step());
    BMG_TRY(residual_step());
    return BMG_OK;
  };
  // Graph replay of cycle_body: not while timing kernels, and only if the
  // body leaves the buffer roles as it found them.
  // graphs replay the cycle; kernel timing uses plain launches (event pairs
  // recorded per launch)
  bool use_graph = o.timed_kernel < 0 && !std::getenv("BMG_NO_GRAPH");
  const bool debug = std::getenv("BMG_DEBUG") != nullptr;
  if (use_graph && !(w->gexec && o.timed_kernel < 0 && w->g_timed < 0 && w->g_sigma == sigma &&
                     w->g_scheme == int(shifted) && w->g_omega == o.omega &&
                     w->g_smoother == o.smoother && w->g_nu1 == o.nu1 && w->g_nu2 == o.nu2 &&
                     w->g_lc == l_c && w->g_tail == cyc.tail_hi && w->g_fuse == int(cyc.fuse_ok) &&
                     w->g_warm == ra.warm)) {
    if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
    if (w->graph) (void)hipGraphDestroy(w->graph);
    w->gexec = nullptr;
    w->graph = nullptr;
  }
  auto launch_body = [&]() -> int {
    if (!use_graph) return cycle_body();
    if (!w->gexec) {
      const std::vector<T*> e0 = cyc.e, t0 = cyc.t;
      const size_t kt_used = kt.used;
      int cst = BMG_OK;
      hipGraph_t g = nullptr;
      hipError_t ce = hipSuccess;
      {
        CaptureGuard cg;  // no device-wide synchronisation meanwhile
        BMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        cst = cycle_body();
        ce = hipStreamEndCapture(s, &g);
      }
      const bool swapped = cyc.e != e0 || cyc.t != t0;  // odd number of Jacobi swaps
      if (cst != BMG_OK || ce != hipSuccess || swapped) {
        // capture impossible here: run this and later cycles as plain launches
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        cyc.e = e0;
        cyc.t = t0;
        kt.discard(kt_used);
        use_graph = false;
        return cycle_body();
      }
      BMG_HIP(hipGraphInstantiate(&w->gexec, g, nullptr, nullptr, 0));
      w->graph = g;
      w->g_timed = o.timed_kernel;
      if (o.timed_kernel >= 0) kt.freeze();
      w->g_sigma = sigma;
      w->g_omega = o.omega;
      w->g_smoother = o.smoother;
      w->g_nu1 = o.nu1;
      w->g_nu2 = o.nu2;
      w->g_lc = l_c;
      w->g_tail = cyc.tail_hi;
      w->g_fuse = int(cyc.fuse_ok);
      w->g_warm = ra.warm;
      w->g_scheme = int(shifted);
    }
    BMG_HIP(hipGraphLaunch(w->gexec, s));
    return BMG_OK;
  };
  TraceRange trace_cycles("bmg_solve: cycles");
  BMG_TRY(residual_step());
  // from here on every Ritz step finds the previous block's residual norms
  // in w->rho2 and its Jacobi threshold follows them; a level ramp (the
  // paper's fixed-cycle runs, whose values are compared level by level) keeps
  // the exact threshold
  ra.rho2 = ramp ? nullptr : w->rho2;
  for (;;) {
    // theta, rho2 and the Ritz status words: written to the pinned host buffer
    // by the cycle's last kernel (k_colsum), else copied back here
    if (w->hbuf_d == nullptr)
      BMG_HIP(hipMemcpyAsync(w->hbuf, w->theta, sizeof(double) * (2 * m + 8), hipMemcpyDeviceToHost, s));
    BMG_HIP(hipStreamSynchronize(s));
    kt.harvest(cycles > 0 && use_graph);
    std::memcpy(theta.data(), w->hbuf, sizeof(double) * m);
    std::memcpy(rho2.data(), w->hbuf + m, sizeof(double) * m);
    int rs3[16] = {0};
    std::memcpy(rs3, w->hbuf + 2 * m, 16 * sizeof(int));
    if (debug) {
      fprintf(stderr, "[bmg] cycle %d ritz: sweeps %d rounds %d fallback %d dropped %d warm %d/%d | phases (us) "
              "assemble %.1f chol %.1f products %.1f jacobi %.1f select %.1f\n", cycles, rs3[1], rs3[9], rs3[2],
              rs3[3], rs3[10], rs3[11], rs3[4] * 0.01, rs3[5] * 0.01, rs3[6] * 0.01, rs3[7] * 0.01, rs3[8] * 0.01);
    }
    const int rstat = rs3[0];
    ritz_sweeps_max = std::max(ritz_sweeps_max, rs3[1]);
    ritz_fallbacks += rs3[2];
    if (rstat == 1) {
      // no m pairs exist: nothing is certified and no pair is written
      set_error("enriched space lost rank below m after %d cycles", cycles);
      status = BMG_ENOCONV;
      cert = Cert();
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
    if (g_cancel && g_cancel->load(std::memory_order_relaxed)) {
      status = BMG_ECANCELED;
      set_error("canceled after %d cycles", cycles);
      break;
    }
    if (cycles >= o.max_cycles) {
      status = BMG_ENOCONV;
      set_error("no convergence in %d cycles", o.max_cycles);
      break;
    }
    BMG_TRY(launch_body());
    ++cycles;
  }

  // ---- output: k pairs nearest sigma, ascending, signs normalised (none
  // when the Ritz step lost rank: evals and evecs are then left untouched)
  std::vector<int> sel = cert.ret;
  std::sort(sel.begin(), sel.end());  // theta is ascending
  const bool have_pairs = int(sel.size()) == k;
  if (have_pairs)
    for (int j = 0; j < k; ++j) evals[j] = theta[sel[j]];
  if (evecs && have_pairs) {
    BMG_HIP(hipMemcpyAsync(w->sel, sel.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
    BMG_TRY(launch_signs(N, w->U, m, w->sel, k, DL.iperm, w->sign, w->argv, w->argi, w->nblk_arg, s));
    if (evecs_on_device) {
      BMG_TRY(launch_write_evecs(N, w->U, m, w->sel, w->sign, k, DL.iperm, evecs, ld, s));
    } else {
      BMG_TRY(launch_write_evecs(N, w->U, m, w->sel, w->sign, k, DL.iperm, w->AU, N, s));
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
    stats->group_size = 1;
    stats->m = m;
    stats->n_c = n_c;
    stats->l_c = l_c;
    stats->t_solve_ms = ms;
    stats->max_rho_over_delta = cert.max_dk;
    stats->max_kato_temple = cert.max_kt;
    stats->timed_kernel_ms = kt.ms;
    stats->timed_kernel_bytes = kt.bytes;
    stats->timed_kernel_units = kt.units;
    stats->ritz_sweeps_max = ritz_sweeps_max;
    stats->ritz_fallbacks = ritz_fallbacks;
    stats->scheme = shifted ? BMG_SCHEME_SHIFTED : BMG_SCHEME_ENRICHED;
    stats->ramp_start = ramp_l0;
    if (ramp && stats->ramp_evals) {
      for (int j = 0; j < k; ++j) ramp_rows[size_t(L) * k + j] = have_pairs ? evals[j] : std::nan("");
      for (int l = ramp_l0; l <= L; ++l)
        for (int j = 0; j < k; ++j) stats->ramp_evals[size_t(l) * k + j] = ramp_rows[size_t(l) * k + j];
    }
    stats->coarse_eig_ms = shifted ? lce->setup_ms : 0.0;
    stats->lc_shift = shifted ? shifts_h[l_c] : sigma;
    if (shifted && l_c < L) {
      // final shift of level l_c (the adaptive shift after the last cycle)
      double v = sigma;
      if (hipMemcpy(&v, w->shifts + l_c, sizeof(double), hipMemcpyDeviceToHost) == hipSuccess)
        stats->lc_shift = v;
      else
        (void)hipGetLastError();
    }
    // report in the output order (ascending)
    for (int j = 0; j < k && j < int(cert.ret.size()); ++j) {
      const int pos = int(std::find(cert.ret.begin(), cert.ret.end(), sel[j]) - cert.ret.begin());
      if (stats->rho) stats->rho[j] = cert.rho[pos];
      if (stats->delta) stats->delta[j] = cert.delta[pos];
    }
  }
  return status;
}

// One request of a grouped solve: its slice of the concatenated block and
// its own Ritz state.
struct GroupItem {
  bmg_group_request* r = nullptr;
  bmg_solve_opts o{};
  int m = 0, off = 0;
  double* rscratch = nullptr;  // [ritz_scratch_doubles(n_c + m)], persists between Ritz steps
  int* status = nullptr;       // [16] Ritz status words
  double *gpart = nullptr, *G = nullptr, *Y = nullptr;  // this request's Gram partials, Gram, Ritz Y
  GramPlan gp{};
  const std::atomic<int>* cancel = nullptr;
  bool done = false;
  int cycles = 0;
};

// Grouped enriched solve (bmg_solve_group): the workspace w is M = sum m_i
// columns wide; request i owns columns [off_i, off_i + m_i) of U, of the
// correction blocks and of theta / rho2.
template <typename T>
int run_group(bmg_hierarchy* h, bmg_workspace* w, double sigma, std::vector<GroupItem>& items,
              const bmg_solve_opts& o, int l_c, hipStream_t s) {
  const int nl = int(h->dev.size());
  const int L = nl - 1;
  const DevLevel& DL = h->dev[L];
  const int64_t N = DL.n;
  const int M = w->m, n_c = o.n_c;
  const int64_t n0 = h->n0;
  const auto t0 = std::chrono::steady_clock::now();
  // S2: W_c = P_{0->L} Phi_c (the n_c level-0 eigenvectors nearest sigma) and
  // its Gram blocks, shared by the group
  {
    std::vector<int> idx = nearest(h->lam0, sigma, n_c);
    std::sort(idx.begin(), idx.end());
    std::vector<double> phic(size_t(n0) * n_c);
    for (int64_t i = 0; i < n0; ++i)
      for (int j = 0; j < n_c; ++j) phic[size_t(i) * n_c + j] = h->phi0[size_t(i) * n0 + idx[j]];
    double* cur = (L % 2 == 0) ? w->W : w->AW;
    BMG_HIP(hipMemcpyAsync(cur, phic.data(), sizeof(double) * phic.size(), hipMemcpyHostToDevice, s));
    for (int l = 1; l <= L; ++l) {
      double* nxt = (cur == w->W) ? w->AW : w->W;
      BMG_TRY(launch_fill<double>(nxt, h->dev[l].n * n_c, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(h->dev[l], cur, nxt, n_c, s));
      cur = nxt;
    }
    BMG_TRY(launch_spmm_am(DL, w->W, w->AW, w->MW, n_c, s));
    BMG_TRY(launch_gram(w->gpw, N, w->W, n_c, nullptr, 0, w->AW, n_c, w->MW, n_c, w->gpart, w->GW, s));
    BMG_HIP(hipStreamSynchronize(s));  // phic is a host local
  }
  // S3: each request's seeded block (the same numbers as its solo solve),
  // drawn into scratch and copied into its columns
  for (GroupItem& it : items) {
    BMG_TRY(launch_gaussian(w->AU, N, it.m, it.o.seed, s, DL.perm));
    BMG_HIP(hipMemcpy2DAsync(w->U + it.off, sizeof(double) * M, w->AU, sizeof(double) * it.m,
                             sizeof(double) * it.m, size_t(N), hipMemcpyDeviceToDevice, s));
  }
  // H4-H6 per request on its slice: the fused Gram and the update per
  // request (own Gram, Y and partial buffers), the Ritz steps of all requests
  // in one launch (one workgroup each, side by side on different CUs)
  // equal widths: one Gram launch and one update launch for the whole group
  // (their buffers are contiguous, see solve_group)
  bool equal = items.size() > 1;
  for (const GroupItem& it : items) equal = equal && it.m == items[0].m;
  auto ritz_steps = [&](int warm) -> int {
    const int nq = int(items.size());
    const int m0 = items[0].m, nz0 = n_c + m0;
    if (equal)
      BMG_TRY(launch_gram_am(items[0].gp, DL, w->W, n_c, w->U, m0, items[0].gpart, items[0].G, s, nullptr, M, nq,
                             int64_t(items[0].gp.nblk) * items[0].gp.per_block, int64_t(nz0) * 2 * m0));
    else
      for (GroupItem& it : items)
        BMG_TRY(launch_gram_am(it.gp, DL, w->W, n_c, w->U + it.off, it.m, it.gpart, it.G, s, nullptr, M));
    for (size_t b0 = 0; b0 < items.size(); b0 += kRitzBatchMax) {
      RitzBatch rb{};
      rb.n = int(std::min<size_t>(kRitzBatchMax, items.size() - b0));
      rb.n_c = n_c;
      rb.sigma = sigma;
      rb.rtol2 = kRitzRtol2;
      rb.GW = w->GW;
      for (int q = 0; q < rb.n; ++q) {
        GroupItem& it = items[b0 + q];
        rb.m[q] = it.m;
        rb.G[q] = it.G;
        rb.Y[q] = it.Y;
        rb.theta[q] = w->theta + it.off;
        rb.scratch[q] = it.rscratch;
        rb.status[q] = it.status;
        rb.rho2[q] = warm ? w->rho2 + it.off : nullptr;  // the residuals exist from the first cycle on
      }
      BMG_TRY(launch_ritz_batch(rb, warm, s));
    }
    if (equal) {
      BMG_TRY(launch_update_zy(N, w->W, n_c, w->U, m0, items[0].Y, w->U, m0, s, M, M, nq));
    } else {
      for (GroupItem& it : items) {
        double* u = w->U + it.off;
        BMG_TRY(launch_update_zy(N, w->W, n_c, u, it.m, it.Y, u, it.m, s, M, M));
      }
    }
    return BMG_OK;
  };
  BMG_TRY(ritz_steps(0));
  Cycle<T> cyc;
  BMG_TRY(init_cycle<T>(cyc, h, w, CycleCfg{M, o.nu1, o.nu2, o.smoother, l_c, sigma, o.omega}, L, s));
  cyc.L = L;
  const bool fold_add = std::getenv("BMG_NO_FUSE") == nullptr;
  // H1 over the whole block: -R and every column's rho^2
  auto residual_step = [&]() -> int {
    BMG_TRY(launch_eigres<T>(DL, w->U, w->theta, -1.0, cyc.f[L], w->rho2part, w->nblk_res, M, s));
    BMG_TRY(launch_colsum(w->rho2part, w->nblk_res, M, w->rho2, s, nullptr, nullptr));
    return BMG_OK;
  };
  auto cycle_body = [&]() -> int {
    cyc.add_u = fold_add ? w->U : nullptr;
    cyc.add_level = L;
    cyc.added = false;
    BMG_TRY(cyc.vcycle(L));
    if (!cyc.added) BMG_TRY(launch_add_to<T>(w->U, cyc.e[L], N * M, s));
    BMG_TRY(ritz_steps(1));
    BMG_TRY(residual_step());
    return BMG_OK;
  };
  // the cycle is replayed as a graph when it can be captured
  bool use_graph = !std::getenv("BMG_NO_GRAPH");
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  auto launch_body = [&]() -> int {
    if (!use_graph) return cycle_body();
    if (!gexec) {
      const std::vector<T*> e0 = cyc.e, t0v = cyc.t;
      int cst = BMG_OK;
      hipGraph_t g = nullptr;
      hipError_t ce = hipSuccess;
      {
        CaptureGuard cg;  // no device-wide synchronisation meanwhile
        BMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        cst = cycle_body();
        ce = hipStreamEndCapture(s, &g);
      }
      const bool swapped = cyc.e != e0 || cyc.t != t0v;
      if (cst != BMG_OK || ce != hipSuccess || swapped) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        cyc.e = e0;
        cyc.t = t0v;
        use_graph = false;
        return cycle_body();
      }
      if (hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        set_error("graph instantiation failed");
        return BMG_EDEVICE;
      }
      graph = g;
    }
    BMG_HIP(hipGraphLaunch(gexec, s));
    return BMG_OK;
  };
  struct GraphGuard {
    hipGraph_t& g;
    hipGraphExec_t& e;
    ~GraphGuard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } guard{graph, gexec};
  BMG_TRY(residual_step());
  const int n = int(items.size());
  int left = n, cycles = 0;
  // per-cycle readback into pinned memory (a copy to pageable memory can wait
  // for other streams' work): theta and rho2 of every column, then every
  // request's status words (contiguous, see solve_group)
  double* pin = nullptr;
  const size_t pin_bytes = sizeof(double) * 2 * M + sizeof(int) * 16 * size_t(n);
  {
    DeviceSyncGuard sync;
    BMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&pin), pin_bytes));
  }
  struct PinGuard {
    double* p;
    ~PinGuard() {
      DeviceSyncGuard sync;
      (void)hipHostFree(p);
    }
  } pin_guard{pin};
  const double* hb = pin;
  const int* hs = reinterpret_cast<const int*>(pin + 2 * M);
  const int* status_base = items[0].status;
  for (;;) {
    BMG_HIP(hipMemcpyAsync(pin, w->theta, sizeof(double) * 2 * M, hipMemcpyDeviceToHost, s));
    BMG_HIP(hipMemcpyAsync(pin + 2 * M, status_base, sizeof(int) * 16 * n, hipMemcpyDeviceToHost, s));
    BMG_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < n; ++q) {
      GroupItem& it = items[q];
      if (it.done) continue;
      bmg_group_request& r = *it.r;
      std::vector<double> theta(hb + it.off, hb + it.off + it.m);
      std::vector<double> rho2(hb + M + it.off, hb + M + it.off + it.m);
      const int rstat = hs[16 * q];
      int st = BMG_OK;
      Cert cert;
      bool finish = false;
      if (rstat == 1) {
        st = BMG_ENOCONV;
        finish = true;
      } else {
        bool finite = true;
        for (int j = 0; j < it.m; ++j) finite = finite && std::isfinite(theta[j]) && std::isfinite(rho2[j]);
        cert = certify(theta, rho2, sigma, r.k, r.tol, it.o.angle_tol);
        if (!finite) {
          st = BMG_ENOCONV;
          finish = true;
        } else if (cert.ok) {
          finish = true;
        } else if (it.cancel && it.cancel->load(std::memory_order_relaxed)) {
          st = BMG_ECANCELED;
          finish = true;
        } else if (cycles >= it.o.max_cycles) {
          st = BMG_ENOCONV;
          finish = true;
        }
      }
      if (!finish) continue;
      // output as in bmg_solve, from this request's columns of the block
      std::vector<int> sel = cert.ret;
      std::sort(sel.begin(), sel.end());
      const bool have_pairs = rstat != 1 && int(sel.size()) == r.k;
      if (have_pairs) {
        for (int j = 0; j < r.k; ++j) r.evals[j] = theta[sel[j]];
        if (r.evecs) {
          std::vector<int> gsel(sel);
          for (int& c : gsel) c += it.off;
          BMG_HIP(hipMemcpyAsync(w->sel, gsel.data(), sizeof(int) * r.k, hipMemcpyHostToDevice, s));
          BMG_TRY(launch_signs(N, w->U, M, w->sel, r.k, DL.iperm, w->sign, w->argv, w->argi, w->nblk_arg, s));
          if (r.evecs_on_device) {
            BMG_TRY(launch_write_evecs(N, w->U, M, w->sel, w->sign, r.k, DL.iperm, r.evecs, r.ld, s));
          } else {
            BMG_TRY(launch_write_evecs(N, w->U, M, w->sel, w->sign, r.k, DL.iperm, w->AU, N, s));
            BMG_HIP(hipMemcpy2DAsync(r.evecs, sizeof(double) * r.ld, w->AU, sizeof(double) * N,
                                     sizeof(double) * N, r.k, hipMemcpyDeviceToHost, s));
          }
          BMG_HIP(hipStreamSynchronize(s));  // gsel is a local
        }
      }
      if (r.stats) {
        bmg_solve_stats& t = *r.stats;
        t.cycles = cycles;
        t.converged = cert.ok && st == BMG_OK ? 1 : 0;
        t.group_size = n;
        t.m = it.m;
        t.n_c = n_c;
        t.l_c = l_c;
        t.t_solve_ms = ms;
        t.max_rho_over_delta = cert.max_dk;
        t.max_kato_temple = cert.max_kt;
        t.timed_kernel_ms = 0.0;
        t.timed_kernel_bytes = 0.0;
        t.timed_kernel_units = 0;
        t.ritz_sweeps_max = 0;
        t.ritz_fallbacks = 0;
        t.scheme = BMG_SCHEME_ENRICHED;
        t.coarse_eig_ms = 0.0;
        t.lc_shift = sigma;
        t.ramp_start = -1;
        for (int j = 0; j < r.k && have_pairs; ++j) {
          const int pos = int(std::find(cert.ret.begin(), cert.ret.end(), sel[j]) - cert.ret.begin());
          if (t.rho) t.rho[j] = cert.rho[pos];
          if (t.delta) t.delta[j] = cert.delta[pos];
        }
      }
      r.status = st;
      it.done = true;
      it.cycles = cycles;
      --left;
    }
    if (left == 0) break;
    BMG_TRY(launch_body());
    ++cycles;
  }
  return BMG_OK;
}

}  // namespace

int solve(bmg_hierarchy* h, int k, double sigma, double tol, const bmg_solve_opts* opts,
          double* evals, double* evecs, int64_t ld, int evecs_on_device, void* stream,
          bmg_solve_stats* stats) {
  TraceRange trace("bmg_solve");
  BMG_CHECK(h != nullptr && evals != nullptr, "hierarchy and evals must be non-NULL");
  bmg_solve_opts o;
  bmg_solve_opts_default(&o);
  if (opts) o = *opts;
  const int nl = int(h->dev.size());
  const int64_t N = h->dev[nl - 1].n;
  BMG_CHECK(k >= 1, "k must be >= 1");
  BMG_CHECK(std::isfinite(sigma), "sigma must be finite");
  BMG_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive and finite");
  BMG_CHECK(o.scheme >= BMG_SCHEME_AUTO && o.scheme <= BMG_SCHEME_SHIFTED, "unknown scheme %d", o.scheme);
  const bool shifted = o.scheme == BMG_SCHEME_SHIFTED || (o.scheme == BMG_SCHEME_AUTO && sigma > 0.0);
  const bool m_given = o.m > 0;
  if (o.m <= 0) o.m = default_block_width(k, sigma);
  int l_c = o.l_c;
  if (shifted) {
    if (l_c < 0) l_c = shifted_coarse_level(h, sigma, o.m, m_given);
    o.n_c = 0;
  } else {
    if (o.n_c <= 0) o.n_c = default_coarse_vectors(h);
    if (l_c < 0) l_c = weyl_coarsest(h, sigma);
  }
  BMG_CHECK(o.m % 4 == 0, "m = %d must be a multiple of 4", o.m);
  BMG_CHECK(o.m >= k, "m = %d must be >= k = %d", o.m, k);
  BMG_CHECK(int64_t(o.m) <= N / 2, "m = %d must be <= N_L / 2", o.m);
  if (!shifted)
    BMG_CHECK(o.n_c % 2 == 0 && o.n_c >= 2 && o.n_c <= h->n0, "n_c must be even and in [2, N_0]");
  BMG_CHECK(o.n_c + o.m <= 96, "n_c + m = %d exceeds 96", o.n_c + o.m);
  BMG_CHECK(o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 <= 64 && o.nu2 <= 64, "nu1, nu2 must be in [0, 64]");
  BMG_CHECK(o.smoother == BMG_SMOOTH_GS || o.smoother == BMG_SMOOTH_JACOBI ||
                o.smoother == BMG_SMOOTH_KACZMARZ,
            "unknown smoother");
  BMG_CHECK(o.precision == BMG_FP64 || o.precision == BMG_MIXED, "unknown precision");
  BMG_CHECK(o.max_cycles >= 0, "max_cycles must be >= 0");
  BMG_CHECK(o.omega > 0 && o.omega < 2, "omega must be in (0, 2)");
  BMG_CHECK(o.angle_tol > 0, "angle_tol must be positive");
  BMG_CHECK(evecs == nullptr || ld >= N, "ld must be >= N_L");
  BMG_CHECK(l_c >= 0 && l_c < nl, "l_c out of range");
  if (shifted) {
    BMG_CHECK(h->host[l_c].n <= kLevelEigMax, "l_c = %d has %lld vertices; the interior scheme's dense "
              "eigensolve takes at most %d", l_c, (long long)h->host[l_c].n, kLevelEigMax);
    BMG_CHECK(h->host[l_c].n >= o.m, "l_c = %d has %lld vertices, fewer than the m = %d start vectors",
              l_c, (long long)h->host[l_c].n, o.m);
  }
  if (!m_given) {
    BMG_HIP(hipSetDevice(h->device));
    BMG_TRY(widened_default_width(h, k, sigma, shifted, l_c, o.n_c, static_cast<hipStream_t>(stream), &o.m));
  }
  BMG_CHECK(o.ramp_cycles >= 0 && o.ramp_cycles <= 64, "ramp_cycles must be in [0, 64]");
  int ramp_l0 = -1;
  if (o.ramp_cycles > 0) {
    ramp_l0 = o.ramp_level;
    if (ramp_l0 < 0) {
      // the coarsest level at or above l_c that holds 2 m eigenpairs
      ramp_l0 = nl - 1;
      for (int l = nl - 1; l >= l_c; --l)
        if (h->host[l].n >= 2 * int64_t(o.m)) ramp_l0 = l;
    }
    BMG_CHECK(ramp_l0 >= l_c && ramp_l0 < nl, "ramp_level %d outside [l_c = %d, %d]", ramp_l0, l_c, nl - 1);
    BMG_CHECK(h->host[ramp_l0].n >= o.m && h->host[ramp_l0].n <= kLevelEigMax,
              "the ramp's first level needs between m and %d vertices", kLevelEigMax);
  }
  BMG_HIP(hipSetDevice(h->device));
  const LevelEig* lce = nullptr;
  if (shifted) BMG_TRY(level_eig(h, l_c, static_cast<hipStream_t>(stream), &lce));
  const LevelEig* lre = nullptr;
  if (ramp_l0 >= 0) BMG_TRY(level_eig(h, ramp_l0, static_cast<hipStream_t>(stream), &lre));
  bmg_workspace* w = nullptr;
  BMG_TRY(acquire_workspace(h, o.m, o.n_c, o.precision, &w));
  // work runs on the workspace's own stream, ordered after the caller's
  // stream at entry and before it at exit
  hipStream_t cs = static_cast<hipStream_t>(stream);
  hipStream_t s = w->stream;
  int st = BMG_OK;
  if (hipEventRecord(w->ev_in, cs) != hipSuccess || hipStreamWaitEvent(s, w->ev_in, 0) != hipSuccess) {
    set_error("stream join failed");
    st = BMG_EDEVICE;
  } else {
    st = (o.precision == BMG_MIXED)
             ? run_solve<float>(h, w, k, sigma, tol, o, l_c, lce, lre, evals, evecs, ld, evecs_on_device, s, stats)
             : run_solve<double>(h, w, k, sigma, tol, o, l_c, lce, lre, evals, evecs, ld, evecs_on_device, s, stats);
  }
  (void)hipStreamSynchronize(s);
  if (hipEventRecord(w->ev_out, s) == hipSuccess) (void)hipStreamWaitEvent(cs, w->ev_out, 0);
  release_workspace(h, w);
  return st;
}

int solve_group(bmg_hierarchy* h, double sigma, int n, bmg_group_request* reqs, void* stream,
                const std::atomic<int>* const* cancel) {
  TraceRange trace("bmg_solve_group");
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy with device data required");
  BMG_CHECK(n >= 1 && reqs != nullptr, "n >= 1 requests required");
  BMG_CHECK(std::isfinite(sigma), "sigma must be finite");
  const int nl = int(h->dev.size());
  const int64_t N = h->dev[nl - 1].n;
  std::vector<GroupItem> items(n);
  int M = 0;
  for (int i = 0; i < n; ++i) {
    bmg_group_request& r = reqs[i];
    GroupItem& it = items[i];
    it.r = &r;
    bmg_solve_opts_default(&it.o);
    if (r.opts) it.o = *r.opts;
    bmg_solve_opts& o = it.o;
    BMG_CHECK(r.k >= 1 && r.evals != nullptr, "request %d: k >= 1 and evals required", i);
    BMG_CHECK(r.tol > 0 && std::isfinite(r.tol), "request %d: tol must be positive and finite", i);
    BMG_CHECK(o.scheme == BMG_SCHEME_ENRICHED || (o.scheme == BMG_SCHEME_AUTO && sigma <= 0.0),
              "request %d: a grouped solve runs the enriched scheme (sigma <= 0 or scheme ENRICHED)", i);
    BMG_CHECK(o.initial_block == nullptr && o.ramp_cycles == 0, "request %d: no initial block or ramp in a group", i);
    if (o.m <= 0) o.m = default_block_width(r.k, sigma);
    if (o.n_c <= 0) o.n_c = default_coarse_vectors(h);
    if (o.l_c < 0) o.l_c = weyl_coarsest(h, sigma);
    BMG_CHECK(o.m % 4 == 0 && o.m >= r.k && int64_t(o.m) <= N / 2, "request %d: m = %d invalid", i, o.m);
    BMG_CHECK(o.n_c % 2 == 0 && o.n_c >= 2 && o.n_c <= h->n0 && o.n_c + o.m <= 96,
              "request %d: n_c = %d invalid", i, o.n_c);
    BMG_CHECK(o.max_cycles >= 0 && o.angle_tol > 0, "request %d: max_cycles / angle_tol invalid", i);
    BMG_CHECK(r.evecs == nullptr || r.ld >= N, "request %d: ld must be >= N_L", i);
    const bmg_solve_opts& f = items[0].o;
    BMG_CHECK(o.precision == f.precision && o.smoother == f.smoother && o.nu1 == f.nu1 && o.nu2 == f.nu2 &&
                  o.omega == f.omega && o.n_c == f.n_c && o.l_c == f.l_c,
              "request %d: precision, smoother, nu1, nu2, omega, n_c and l_c must agree across the group", i);
    it.m = o.m;
    it.off = M;
    it.cancel = cancel ? cancel[i] : nullptr;
    M += o.m;
    r.status = BMG_EINVAL;
  }
  const bmg_solve_opts& o = items[0].o;
  BMG_CHECK(M <= 512, "the group's blocks are %d columns wide; at most 512", M);
  BMG_CHECK(o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 <= 64 && o.nu2 <= 64, "nu1, nu2 must be in [0, 64]");
  BMG_CHECK(o.smoother == BMG_SMOOTH_GS || o.smoother == BMG_SMOOTH_JACOBI || o.smoother == BMG_SMOOTH_KACZMARZ,
            "unknown smoother");
  BMG_CHECK(o.precision == BMG_FP64 || o.precision == BMG_MIXED, "unknown precision");
  BMG_CHECK(o.omega > 0 && o.omega < 2, "omega must be in (0, 2)");
  BMG_CHECK(o.l_c >= 0 && o.l_c < nl, "l_c out of range");
  BMG_HIP(hipSetDevice(h->device));
  // the requests' Gram and Ritz buffers are their own (below): the
  // workspace's serve only the shared W_c block
  bmg_workspace* w = nullptr;
  BMG_TRY(acquire_workspace(h, M, o.n_c, o.precision, &w, 2));
  hipStream_t cs = static_cast<hipStream_t>(stream);
  hipStream_t s = w->stream;
  // per-request Ritz scratch and status words (contiguous: one readback)
  std::vector<void*> bufs;
  int st = BMG_OK;
  auto dalloc_local = [&](void** p, size_t bytes) -> int {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of %zu bytes failed", bytes);
      return BMG_ENOMEM;
    }
    bufs.push_back(*p);
    return BMG_OK;
  };
  int* status_all = nullptr;
  st = dalloc_local(reinterpret_cast<void**>(&status_all), sizeof(int) * 16 * n);
  // per-request Gram partials, Gram and Y, one contiguous array each (the
  // layout the equal-width batched launches need)
  size_t n_part = 0, n_g = 0, n_y = 0;
  for (GroupItem& it : items) {
    const int nz = o.n_c + it.m;
    it.gp = gram_plan(N, nz, 2 * it.m);
    n_part += size_t(it.gp.nblk) * it.gp.per_block;
    n_g += size_t(nz) * 2 * it.m;
    n_y += size_t(nz) * it.m;
  }
  double *part_all = nullptr, *g_all = nullptr, *y_all = nullptr;
  if (st == BMG_OK) st = dalloc_local(reinterpret_cast<void**>(&part_all), sizeof(double) * n_part);
  if (st == BMG_OK) st = dalloc_local(reinterpret_cast<void**>(&g_all), sizeof(double) * n_g);
  if (st == BMG_OK) st = dalloc_local(reinterpret_cast<void**>(&y_all), sizeof(double) * n_y);
  for (int i = 0; i < n && st == BMG_OK; ++i) {
    GroupItem& it = items[i];
    const int nz = o.n_c + it.m;
    it.status = status_all + 16 * i;
    it.gpart = part_all;
    it.G = g_all;
    it.Y = y_all;
    part_all += size_t(it.gp.nblk) * it.gp.per_block;
    g_all += size_t(nz) * 2 * it.m;
    y_all += size_t(nz) * it.m;
    st = dalloc_local(reinterpret_cast<void**>(&it.rscratch), sizeof(double) * ritz_scratch_doubles(nz));
  }
  if (st == BMG_OK && hipMemsetAsync(status_all, 0, sizeof(int) * 16 * n, s) != hipSuccess) {
    set_error("status clear failed");
    st = BMG_EDEVICE;
  }
  if (st == BMG_OK) {
    if (hipEventRecord(w->ev_in, cs) != hipSuccess || hipStreamWaitEvent(s, w->ev_in, 0) != hipSuccess) {
      set_error("stream join failed");
      st = BMG_EDEVICE;
    } else {
      st = (o.precision == BMG_MIXED) ? run_group<float>(h, w, sigma, items, o, o.l_c, s)
                                      : run_group<double>(h, w, sigma, items, o, o.l_c, s);
    }
  }
  (void)hipStreamSynchronize(s);
  if (hipEventRecord(w->ev_out, s) == hipSuccess) (void)hipStreamWaitEvent(cs, w->ev_out, 0);
  for (void* p : bufs) dev_free(p);
  release_workspace(h, w);
  if (st != BMG_OK) {
    for (int i = 0; i < n; ++i)
      if (!items[i].done) reqs[i].status = st;
    return st;
  }
  for (int i = 0; i < n; ++i)
    if (reqs[i].status != BMG_OK) {
      set_error("request %d of the group ended with status %d", i, reqs[i].status);
      return reqs[i].status;
    }
  return BMG_OK;
}

// V-cycle for bmg_apply: uses a temporary workspace.
int apply_vcycle(bmg_hierarchy* h, int level, int dtype, int m, double sigma, int smoother,
                 int nu1, int nu2, int l_c, double omega, const void* x, void* y, hipStream_t s) {
  const int lc = l_c < 0 ? weyl_coarsest(h, sigma) : l_c;
  BMG_CHECK(lc >= 0 && lc <= level, "l_c must be in [0, level]");
  bmg_workspace* w = nullptr;
  const int prec = dtype == 1 ? BMG_MIXED : BMG_FP64;
  const int n_c = default_coarse_vectors(h);
  BMG_TRY(make_workspace(h, m, n_c, prec, &w));
  const size_t vb = dtype == 1 ? sizeof(float) : sizeof(double);
  int st = BMG_OK;
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    BMG_HIP(hipMemcpyAsync(w->f[level], x, vb * h->dev[level].n * m, hipMemcpyDeviceToDevice, s));
    Cycle<T> cyc;
    BMG_TRY(init_cycle<T>(cyc, h, w, CycleCfg{m, nu1, nu2, smoother, lc, sigma, omega}, level, s));
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
