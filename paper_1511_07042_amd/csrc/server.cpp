// Request-level continuous batching (serving).
//
// Independent eigenproblems (surface, refinement level, k, sigma, options) are
// admitted against a device-memory budget and a slot count and then run
// concurrently: every slot is a worker thread with its own HIP stream, and a
// solve runs on a pooled workspace of its hierarchy with a stream of its own,
// so the device interleaves the kernels of all active requests.  A request
// that arrives while others run is admitted as soon as a slot is free and its
// footprint fits beside the resident hierarchies, the pooled workspaces and
// the active requests; smaller requests may pass a waiting larger one, a
// bounded number of times.
//
// Requests for the same surface, level and shift that run the enriched scheme
// with the same cycle options are grouped: a worker that starts one takes the
// compatible requests waiting behind it (up to kMaxGroup, 512 columns) and runs
// them as one grouped solve (bmg_solve_group), whose correction cycle is a
// single set of launches over their concatenated blocks.  A grouped request's
// result equals its bmg_solve result to rounding; any other request's result
// is the result of bmg_solve with the same arguments, bit for bit: the kernels
// are deterministic and solves share only read-only hierarchy data.  Hierarchies are built on first use and cached by surface
// and level; idle workspaces and then idle hierarchies (least recently used
// first) are freed when the budget needs their memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "bmg_internal.h"

namespace {

using clk = std::chrono::steady_clock;

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
  uint64_t id = 0;
  bmg_surface_desc desc{};
  std::vector<double> xyz;
  std::vector<int32_t> tri;
  int32_t n_refine = 0, k = 0;
  double sigma = 0.0, tol = 0.0;
  bmg_solve_opts opts{};
  std::string key;
  bool groupable = false;  // enriched scheme, no ramp: may share a grouped solve
  int m_est = 0;           // block width the solver will use
  int64_t n_est = 0;   // finest-level vertices
  int64_t need = 0;    // workspace bytes reserved while running
  int64_t hier = 0;    // hierarchy bytes if it must be built
  int bypassed = 0;    // times a later request was admitted before it
  ReqState state = QUEUED;
  std::atomic<int> cancel{0};
  int status = BMG_OK;
  std::string error;
  int64_t N = 0;
  std::vector<double> evals, evecs, rho, delta;
  bmg_solve_stats stats{};
  clk::time_point t_submit, t_done;
};

struct Cached {
  bmg_hierarchy* h = nullptr;
  int64_t bytes = 0;   // device bytes of the levels (estimate while building)
  int users = 0;
  bool building = false;
  uint64_t last_use = 0;
};

// Coarse-mesh sizes (vertices, edges, triangles) of a surface description.
void coarse_counts(const bmg_surface_desc& d, int64_t* n, int64_t* e, int64_t* f) {
  if (d.kind == BMG_SPHERE || d.kind == BMG_ELLIPSOID) {
    *n = 12, *e = 30, *f = 20;
  } else if (d.kind == BMG_TORUS) {
    *n = int64_t(d.nu) * d.nv, *e = 3 * *n, *f = 2 * *n;
  } else {
    *n = d.n_vert, *f = d.n_tri, *e = int64_t(d.n_tri) * 3 / 2;
  }
}

// Per-level vertex counts of uniform refinement (every edge gains a midpoint,
// every triangle splits into four).
std::vector<int64_t> level_vertices(const bmg_surface_desc& d, int n_refine) {
  int64_t n, e, f;
  coarse_counts(d, &n, &e, &f);
  std::vector<int64_t> v{n};
  for (int l = 0; l < n_refine; ++l) {
    n += e;
    e = 2 * e + 3 * f;
    f *= 4;
    v.push_back(n);
  }
  return v;
}

// ELL row width assumed for footprints: valence 6 (+ diagonal) on the built-in
// surfaces; a custom mesh may have vertices of valence up to 30.
int ell_width(const bmg_surface_desc& d) { return d.kind == BMG_CUSTOM ? 31 : 7; }

// Device bytes of a hierarchy: per level FP64 and FP32 values of A and M,
// columns, lumped mass, colours and transfer tables; the level-0 eigenvectors
// and their transpose in FP64 and FP32.
int64_t hierarchy_estimate(const bmg_surface_desc& d, int n_refine) {
  const int W = ell_width(d);
  const std::vector<int64_t> lv = level_vertices(d, n_refine);
  int64_t b = 24 * lv[0] * lv[0];
  for (int64_t n : lv) b += n * (int64_t(W) * (2 * 8 + 2 * 4 + 4) + 64);
  return b + (1 << 20);
}

// Device bytes of one solve's workspace (an upper bound of what the solver
// allocates): FP64 W, AW, MW [N][n_c] and U, AU, MU [N][m]; per level e, f, t
// [n_l][m] and the shifted operator [n_l][W] in the correction precision;
// Gram partial sums (at most a quarter of the bytes the Gram kernel reads);
// the LDS-tail image and small buffers.
int64_t workspace_estimate(const bmg_surface_desc& d, int n_refine, int m, int n_c, int prec) {
  const std::vector<int64_t> lv = level_vertices(d, n_refine);
  const int64_t N = lv.back();
  const int64_t vb = prec == BMG_MIXED ? 4 : 8;
  int64_t b = 8 * N * (3 * int64_t(n_c) + 3 * int64_t(m));
  for (int64_t n : lv) b += vb * n * (3 * int64_t(m) + ell_width(d));
  b += 2 * N * (int64_t(n_c) + 3 * int64_t(m));
  return b + 2 * (1 << 20);
}

// Device bytes the interior-shift scheme adds for a request: the dense
// eigendecomposition of its coarse level (FP64 and FP32 eigenvectors, kept
// with the hierarchy) and the coarse solve's scratch.  The solver picks the
// level from the meshes' edge lengths, which are not known before the build,
// so this bound takes the finest level it may use (at most kLevelEigMax
// vertices) and, when m was not given, the widest block (96, or half that
// level's vertices).  *m_est receives the block width.
int64_t shifted_estimate(const bmg_surface_desc& d, int n_refine, int m, bool m_given, int prec,
                         int* m_est) {
  const std::vector<int64_t> lv = level_vertices(d, n_refine);
  int cap = 0;
  for (size_t l = 0; l < lv.size(); ++l)
    if (lv[l] <= bmg::kLevelEigMax) cap = int(l);
  const int64_t n = lv[cap];
  if (!m_given && cap < int(lv.size()) - 1) m = std::max(m, int(std::min<int64_t>(96, n / 2 / 4 * 4)));
  *m_est = m;
  const int64_t vb = prec == BMG_MIXED ? 4 : 8;
  return 12 * n * n + 8 * n + vb * n * (1 + int64_t(m) * (1 + bmg::spec_slices(int(n))));
}

// Finest-level vertex count and the device bytes of all levels.
void hierarchy_totals(const bmg_hierarchy* h, int64_t* n_finest, int64_t* bytes) {
  *n_finest = 0;
  *bytes = 0;
  bmg_level_info li{};
  if (bmg_hierarchy_info(h, 0, &li) != BMG_OK) return;
  const int nl = li.n_levels;
  for (int l = 0; l < nl; ++l) {
    if (bmg_hierarchy_info(h, l, &li) != BMG_OK) return;
    *bytes += li.device_bytes;
    *n_finest = li.n_vert;
  }
}

std::string surface_key(const Request& r) {
  std::ostringstream k;
  const bmg_surface_desc& d = r.desc;
  k.precision(17);
  k << d.kind << '/' << r.n_refine << '/';
  if (d.kind == BMG_ELLIPSOID) k << d.axes[0] << ',' << d.axes[1] << ',' << d.axes[2];
  if (d.kind == BMG_TORUS) k << d.R << ',' << d.r << ',' << d.nu << ',' << d.nv;
  if (d.kind == BMG_CUSTOM) {
    // FNV-1a of the arrays, plus the projection callback, identify a custom surface
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
      const unsigned char* c = static_cast<const unsigned char*>(p);
      for (size_t i = 0; i < n; ++i) hsh = (hsh ^ c[i]) * 1099511628211ull;
    };
    mix(r.xyz.data(), r.xyz.size() * sizeof(double));
    mix(r.tri.data(), r.tri.size() * sizeof(int32_t));
    k << std::hex << hsh << '/' << reinterpret_cast<uintptr_t>(d.project) << '/'
      << reinterpret_cast<uintptr_t>(d.ctx);
  }
  return k.str();
}

constexpr int kMaxGroup = 8;
constexpr int kMaxGroupColumns = 512;

// Whether b may join a grouped solve led by a: same hierarchy and shift, and
// the options a grouped solve requires to agree (bmg_solve_group).
bool group_compatible(const Request& a, const Request& b) {
  const bmg_solve_opts &x = a.opts, &y = b.opts;
  return a.groupable && b.groupable && a.key == b.key && a.sigma == b.sigma && x.precision == y.precision &&
         x.smoother == y.smoother && x.nu1 == y.nu1 && x.nu2 == y.nu2 && x.omega == y.omega &&
         x.n_c == y.n_c && x.l_c == y.l_c;
}

// Sets the calling thread's cancel flag for the duration of a solve.
struct CancelScope {
  explicit CancelScope(const std::atomic<int>* f) { bmg::g_cancel = f; }
  ~CancelScope() { bmg::g_cancel = nullptr; }
};

}  // namespace

struct bmg_server {
  int device = 0;
  int64_t budget = 0;
  int slots = 0;
  std::mutex mu;
  std::condition_variable cv;  // queue, admission, cache and completion changes
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::map<std::string, Cached> cache;
  int64_t active_bytes = 0;
  int running = 0;
  uint64_t next_id = 1, tick = 0;
  bool stopping = false;
  bool grouping = std::getenv("BMG_NO_GROUP") == nullptr;
  std::vector<std::thread> workers;

  // ---- everything below runs with mu held
  // Device bytes held now: cached hierarchies, their idle pooled workspaces,
  // and the workspaces reserved by running requests.
  int64_t resident() {
    int64_t b = active_bytes;
    for (auto& kv : cache) {
      b += kv.second.bytes;
      if (kv.second.h) b += bmg::idle_workspace_bytes(kv.second.h);
    }
    return b;
  }
  int64_t cost(const Request& r) const {
    return r.need + (cache.count(r.key) ? 0 : r.hier);
  }
  // Free idle workspaces, then idle hierarchies other than `keep` (least
  // recently used first), until `need` more bytes fit.
  void make_room(int64_t need, const std::string& keep) {
    if (resident() + need <= budget) return;
    for (auto& kv : cache)
      if (kv.second.h) bmg::trim_idle_workspaces(kv.second.h);
    while (resident() + need > budget) {
      auto victim = cache.end();
      for (auto it = cache.begin(); it != cache.end(); ++it)
        if (it->second.users == 0 && !it->second.building && it->first != keep &&
            (victim == cache.end() || it->second.last_use < victim->second.last_use))
          victim = it;
      if (victim == cache.end()) return;
      bmg_free_hierarchy(victim->second.h);
      cache.erase(victim);
    }
  }
  // The next request to start, or nullptr.  First fit in arrival order; once
  // the head of the queue has been passed 4 * slots times only it may start.
  Request* admit() {
    if (running >= slots || queue.empty()) return nullptr;
    Request& head = *reqs.at(queue.front());
    const bool head_only = head.bypassed >= 4 * slots;
    for (size_t i = 0; i < queue.size(); ++i) {
      Request& r = *reqs.at(queue[i]);
      const int64_t c = cost(r);
      make_room(c, r.key);
      if (resident() + c <= budget || running == 0) {
        if (i > 0) head.bypassed += 1;
        queue.erase(queue.begin() + i);
        return &r;
      }
      if (head_only) break;
    }
    return nullptr;
  }

  // Compatible requests waiting behind the leader that fit the budget: taken
  // off the queue and reserved (their workspaces' bytes) for one grouped solve.
  std::vector<Request*> take_group(Request* lead) {
    std::vector<Request*> g{lead};
    if (!grouping || !lead->groupable) return g;
    int cols = lead->m_est;
    for (size_t i = 0; i < queue.size() && int(g.size()) < kMaxGroup;) {
      Request& r = *reqs.at(queue[i]);
      if (group_compatible(*lead, r) && cols + r.m_est <= kMaxGroupColumns &&
          resident() + r.need <= budget) {
        cols += r.m_est;
        active_bytes += r.need;
        r.state = RUNNING;
        g.push_back(&r);
        queue.erase(queue.begin() + i);
      } else {
        ++i;
      }
    }
    return g;
  }

  void finish(Request* r, int st) {
    r->stats.rho = nullptr;
    r->stats.delta = nullptr;
    r->status = st;
    r->state = DONE;
    r->t_done = clk::now();
    cv.notify_all();
  }

  // Finds or builds the request's hierarchy; returns it with one more user.
  int acquire_hierarchy(Request* r, hipStream_t stream, std::unique_lock<std::mutex>& lk,
                        bmg_hierarchy** out) {
    for (;;) {
      auto it = cache.find(r->key);
      if (it != cache.end() && it->second.building) {
        cv.wait(lk);
        continue;
      }
      if (it != cache.end()) {
        it->second.users += 1;
        it->second.last_use = ++tick;
        *out = it->second.h;
        return BMG_OK;
      }
      Cached& c = cache[r->key];
      c.building = true;
      c.bytes = r->hier;
      lk.unlock();
      bmg_surface_desc d = r->desc;
      if (d.kind == BMG_CUSTOM) {
        d.xyz = r->xyz.data();
        d.tri = r->tri.data();
      }
      bmg_hierarchy* nh = nullptr;
      const int st = stream ? bmg_build_hierarchy(&d, r->n_refine, stream, &nh) : BMG_EDEVICE;
      const std::string err = st == BMG_OK ? "" : bmg_last_error();
      int64_t bytes = 0, nf = 0;
      if (st == BMG_OK) hierarchy_totals(nh, &nf, &bytes);
      lk.lock();
      Cached& c2 = cache[r->key];
      c2.building = false;
      cv.notify_all();
      if (st != BMG_OK) {
        cache.erase(r->key);
        r->error = err.empty() ? "hierarchy build failed" : err;
        return st;
      }
      c2.h = nh;
      c2.bytes = bytes;
    }
  }

  void worker_main() {
    hipStream_t stream = nullptr;
    {
      bmg::DeviceSyncGuard sync;
      if (hipSetDevice(device) != hipSuccess ||
          hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        stream = nullptr;
      }
    }
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Request* r = nullptr;
      while (!(stopping && queue.empty()) && (r = admit()) == nullptr) cv.wait(lk);
      if (r == nullptr) break;
      r->state = RUNNING;
      active_bytes += r->need;
      ++running;
      const std::vector<Request*> group = take_group(r);
      bmg_hierarchy* h = nullptr;
      int st = acquire_hierarchy(r, stream, lk, &h);
      std::vector<int> sts(group.size(), st);
      if (st == BMG_OK) {
        lk.unlock();
        int64_t nf = 0, hb = 0;
        hierarchy_totals(h, &nf, &hb);
        for (Request* q : group) {
          q->N = nf;
          q->evals.assign(q->k, 0.0);
          q->evecs.assign(size_t(q->N) * q->k, 0.0);
          q->rho.assign(q->k, 0.0);
          q->delta.assign(q->k, 0.0);
          q->stats.rho = q->rho.data();
          q->stats.delta = q->delta.data();
        }
        if (group.size() == 1) {
          CancelScope scope(&r->cancel);
          st = bmg::solve(h, r->k, r->sigma, r->tol, &r->opts, r->evals.data(), r->evecs.data(),
                          r->N, 0, stream, &r->stats);
          sts[0] = st;
          if (st != BMG_OK) r->error = bmg_last_error();
        } else {
          std::vector<bmg_group_request> gr(group.size());
          std::vector<const std::atomic<int>*> flags(group.size());
          for (size_t i = 0; i < group.size(); ++i) {
            Request* q = group[i];
            gr[i] = bmg_group_request{q->k, q->tol, &q->opts, q->evals.data(), q->evecs.data(), q->N, 0,
                                      BMG_OK, &q->stats};
            flags[i] = &q->cancel;
          }
          st = bmg::solve_group(h, r->sigma, int(group.size()), gr.data(), stream, flags.data());
          const std::string err = st == BMG_OK ? "" : bmg_last_error();
          for (size_t i = 0; i < group.size(); ++i) {
            sts[i] = gr[i].status;
            if (sts[i] != BMG_OK) group[i]->error = sts[i] == BMG_ECANCELED ? "canceled" : err;
          }
        }
        lk.lock();
        auto it = cache.find(r->key);
        if (it != cache.end()) {
          it->second.users -= 1;
          it->second.last_use = ++tick;
        }
      }
      --running;
      for (size_t i = 0; i < group.size(); ++i) {
        active_bytes -= group[i]->need;
        if (st != BMG_OK && group[i]->error.empty()) group[i]->error = r->error;
        finish(group[i], sts[i]);
      }
    }
    lk.unlock();
    if (stream) {
      bmg::DeviceSyncGuard sync;
      (void)hipStreamDestroy(stream);
    }
  }
};

extern "C" {

int bmg_server_create(int64_t hbm_budget_bytes, int32_t max_slots, bmg_server** out) {
  BMG_CHECK(out != nullptr, "out must be non-NULL");
  *out = nullptr;
  BMG_CHECK(hbm_budget_bytes > 0, "the memory budget must be positive");
  BMG_CHECK(max_slots >= 1 && max_slots <= 64, "max_slots must be in [1, 64]");
  int dev = 0, n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1 || hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    bmg::set_error("no HIP device");
    return BMG_EDEVICE;
  }
  auto* s = new (std::nothrow) bmg_server();
  if (!s) return BMG_ENOMEM;
  s->device = dev;
  s->budget = hbm_budget_bytes;
  s->slots = max_slots;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s] { s->worker_main(); });
  *out = s;
  return BMG_OK;
}

int bmg_server_submit(bmg_server* s, const bmg_surface_desc* desc, int32_t n_refine, int32_t k,
                      double sigma, double tol, const bmg_solve_opts* opts, uint64_t* request_id) {
  BMG_CHECK(s && desc && request_id, "NULL argument");
  BMG_CHECK(n_refine >= 0 && n_refine <= 10, "n_refine must be in [0, 10]");
  BMG_CHECK(k >= 1, "k must be >= 1");
  BMG_CHECK(std::isfinite(sigma), "sigma must be finite");
  BMG_CHECK(tol > 0 && std::isfinite(tol), "tol must be positive and finite");
  BMG_CHECK(desc->kind >= BMG_SPHERE && desc->kind <= BMG_CUSTOM, "unknown surface kind");
  if (desc->kind == BMG_TORUS) BMG_CHECK(desc->nu >= 3 && desc->nv >= 3, "torus grid too small");
  auto r = std::make_unique<Request>();
  r->desc = *desc;
  r->desc.xyz = nullptr;
  r->desc.tri = nullptr;
  if (desc->kind == BMG_CUSTOM) {
    BMG_CHECK(desc->xyz && desc->tri && desc->n_vert > 0 && desc->n_tri > 0,
              "custom mesh arrays missing");
    r->xyz.assign(desc->xyz, desc->xyz + 3 * int64_t(desc->n_vert));
    r->tri.assign(desc->tri, desc->tri + 3 * int64_t(desc->n_tri));
  }
  r->n_refine = n_refine;
  r->k = k;
  r->sigma = sigma;
  r->tol = tol;
  bmg_solve_opts_default(&r->opts);
  if (opts) r->opts = *opts;
  r->opts.initial_block = nullptr;  // not kept: the caller's pointer dies with the call
  r->opts.timed_kernel = -1;
  // the block width and the scheme are left to the solver (as in bmg_solve);
  // the footprint uses upper bounds of what it will choose
  BMG_CHECK(r->opts.scheme >= BMG_SCHEME_AUTO && r->opts.scheme <= BMG_SCHEME_SHIFTED, "unknown scheme");
  const bool shifted = r->opts.scheme == BMG_SCHEME_SHIFTED || (r->opts.scheme == BMG_SCHEME_AUTO && sigma > 0.0);
  int m_est = r->opts.m > 0 ? r->opts.m : bmg::default_block_width(k, sigma);
  int64_t n0, e0, f0;
  coarse_counts(r->desc, &n0, &e0, &f0);
  // the solver's default n_c (min(N_0, 32), rounded down to even)
  const int n_c = shifted ? 0 : (r->opts.n_c > 0 ? r->opts.n_c : int(std::min<int64_t>(n0, 32)) & ~1);
  r->key = surface_key(*r);
  r->n_est = level_vertices(r->desc, n_refine).back();
  r->hier = hierarchy_estimate(r->desc, n_refine);
  // a request that names no width may run wider than the default when it runs
  // alone (the solver widens the block to whole clusters of the spectrum), so
  // its footprint takes the widest block the solver can choose; grouping
  // keeps the default width (a grouped solve does not widen)
  int m_foot = m_est;
  if (r->opts.m <= 0)
    m_foot = std::max(m_est, int(std::min<int64_t>(96 - n_c, r->n_est / 2) / 4 * 4));
  int64_t extra = 0;
  if (shifted)
    extra = shifted_estimate(r->desc, n_refine, m_foot, r->opts.m > 0, r->opts.precision, &m_foot);
  r->need = workspace_estimate(r->desc, n_refine, m_foot, n_c, r->opts.precision) + extra;
  r->groupable = !shifted && r->opts.ramp_cycles == 0;
  r->m_est = m_est;
  BMG_CHECK(m_est >= k && int64_t(m_est) <= r->n_est / 2, "m must be in [k, N_L / 2]");
  std::lock_guard<std::mutex> g(s->mu);
  BMG_CHECK(!s->stopping, "the server is shutting down");
  if (r->need + r->hier > s->budget) {
    bmg::set_error("request needs about %lld bytes; the budget is %lld",
                   (long long)(r->need + r->hier), (long long)s->budget);
    return BMG_ENOMEM;
  }
  r->id = s->next_id++;
  r->t_submit = clk::now();
  *request_id = r->id;
  s->queue.push_back(r->id);
  s->reqs[r->id] = std::move(r);
  s->cv.notify_all();
  return BMG_OK;
}

int bmg_server_poll(bmg_server* s, uint64_t request_id, double* evals, double* evecs, int64_t ld,
                    bmg_solve_stats* stats, double* latency_ms) {
  BMG_CHECK(s != nullptr, "NULL server");
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(request_id);
    BMG_CHECK(it != s->reqs.end(), "unknown request id %llu", (unsigned long long)request_id);
    if (it->second->state != DONE) return BMG_EBUSY;
    Request& q = *it->second;
    if (evecs && !q.evecs.empty() && ld < q.N) {
      bmg::set_error("ld = %lld must be >= N_L = %lld", (long long)ld, (long long)q.N);
      return BMG_EINVAL;
    }
    r = std::move(it->second);
    s->reqs.erase(it);
  }
  if (evals && !r->evals.empty()) std::memcpy(evals, r->evals.data(), sizeof(double) * r->k);
  if (evecs && !r->evecs.empty())
    for (int j = 0; j < r->k; ++j)
      std::memcpy(evecs + int64_t(j) * ld, r->evecs.data() + int64_t(j) * r->N,
                  sizeof(double) * r->N);
  if (stats) {
    double* rho = stats->rho;
    double* delta = stats->delta;
    double* ramp = stats->ramp_evals;
    *stats = r->stats;
    stats->rho = rho;
    stats->delta = delta;
    stats->ramp_evals = ramp;  // not kept by the server: left untouched
    if (rho && !r->rho.empty()) std::memcpy(rho, r->rho.data(), sizeof(double) * r->k);
    if (delta && !r->delta.empty()) std::memcpy(delta, r->delta.data(), sizeof(double) * r->k);
  }
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (r->status != BMG_OK) bmg::set_error("%s", r->error.c_str());
  return r->status;
}

int bmg_server_cancel(bmg_server* s, uint64_t request_id) {
  BMG_CHECK(s != nullptr, "NULL server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(request_id);
  BMG_CHECK(it != s->reqs.end(), "unknown request id %llu", (unsigned long long)request_id);
  Request& r = *it->second;
  if (r.state == QUEUED) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), request_id), s->queue.end());
    r.error = "canceled before it started";
    s->finish(&r, BMG_ECANCELED);
  } else if (r.state == RUNNING) {
    r.cancel.store(1);
  }
  return BMG_OK;
}

void bmg_server_destroy(bmg_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
    for (uint64_t id : s->queue) {
      Request& r = *s->reqs.at(id);
      r.error = "server destroyed before the request started";
      s->finish(&r, BMG_ECANCELED);
    }
    s->queue.clear();
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->cache)
    if (kv.second.h) bmg_free_hierarchy(kv.second.h);
  delete s;
}

}  // extern "C"
