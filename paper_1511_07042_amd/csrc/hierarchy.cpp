// Device-resident hierarchy: upload of the host levels, the level-0
// eigendecomposition, sizes and export for inspection.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#include "bmg_internal.h"

#include <shared_mutex>

namespace bmg {

namespace {

template <typename T>
int upload(T** dst, const T* src, size_t count, hipStream_t s, int64_t& bytes) {
  *dst = nullptr;
  if (count == 0) return BMG_OK;
  if (hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(T)) != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed", count * sizeof(T));
    return BMG_ENOMEM;
  }
  bytes += int64_t(count * sizeof(T));
  BMG_HIP(hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  return BMG_OK;
}

// The Gram kernel's chunk order changes which rows a block's partial sums
// cover (and so their rounding): it is used on levels this large only.
constexpr int64_t kChunkOrderMinRows = 131072;

// Levels with at least this many rows are stored in a Morton order of their
// vertices (smaller levels stay in the caches in any order);
// BMG_ROW_ORDER_MIN_ROWS overrides it, down to kStorageOrderFloor.
constexpr int64_t kStorageOrderFloor = 16384;
static_assert(kStorageOrderFloor > kLevelEigMax, "levels with dense eigendecompositions stay in vertex order");
int64_t row_order_min_rows() {
  if (const char* e = std::getenv("BMG_ROW_ORDER_MIN_ROWS")) return std::atoll(e);
  return 131072;
}

}  // namespace

// Device copy of a level.  A large level is stored with its rows permuted
// along a Morton curve through the vertex positions: storage row r holds
// vertex perm[r] (iperm is the inverse), the ELL column indices, colour lists
// and transfer tables are renumbered to match, and every row keeps its slots
// in the same order, so each row's arithmetic is unchanged.  A row and its
// neighbours then sit close together in memory, and the neighbour rows a
// kernel gathers are still in the caches from the rows just before.  The
// transfer tables of a stored-permuted level take a general form: parents
// [n][2] gives both parents of every fine row in the coarse level's storage
// (a vertex of the coarse level names its copy twice: (x + x) / 2 = x
// exactly), with par_nc = 0; rself [n_prev] gives the storage row of each
// coarse vertex's own copy.  Other levels keep the nested numbering (fine
// rows below n_prev are the coarse vertices, par_nc = n_prev, rself null).
int upload_hierarchy(bmg_hierarchy* h, hipStream_t s) {
  const int nl = int(h->host.size());
  h->dev.resize(nl);
  std::vector<std::vector<float>> keep32;  // host staging must live until the stream syncs
  const int64_t min_ordered = row_order_min_rows();
  std::vector<int32_t> iperm_prev;  // storage row of each vertex of the level below (empty: identity)
  for (int l = 0; l < nl; ++l) {
    const HostLevel& H = h->host[l];
    DevLevel& D = h->dev[l];
    D.n = H.n;
    D.n_prev = H.n_prev;
    D.W = H.W;
    D.RW = H.RW;
    D.n_colours = H.n_colours;
    D.colour_ptr = H.colour_ptr;
    D.bytes = 0;
    const size_t nw = size_t(H.n) * H.W;
    // never a level small enough for the LDS tail or a dense level
    // eigendecomposition: those read the host tables in vertex order
    const bool permuted = H.n >= min_ordered && H.n >= kStorageOrderFloor;
    std::vector<int32_t> perm, iperm;
    if (permuted) {
      perm = morton_order(H.xyz);
      iperm.assign(size_t(H.n), 0);
      for (int64_t r = 0; r < H.n; ++r) iperm[size_t(perm[size_t(r)])] = int32_t(r);
    }
    auto snew = [&](int32_t q) { return permuted ? iperm[size_t(q)] : q; };        // this level
    auto cnew = [&](int32_t q) { return iperm_prev.empty() ? q : iperm_prev[size_t(q)]; };  // level below
    auto nat = [&](int64_t r) { return permuted ? int64_t(perm[size_t(r)]) : r; };
    std::vector<int32_t> cols(nw);
    std::vector<double> a(nw), mm(nw);
    for (int64_t r = 0; r < H.n; ++r) {
      const size_t q = size_t(nat(r));
      for (int k = 0; k < H.W; ++k) {
        cols[size_t(r) * H.W + k] = snew(H.cols[q * H.W + k]);
        a[size_t(r) * H.W + k] = H.a[q * H.W + k];
        mm[size_t(r) * H.W + k] = H.mm[q * H.W + k];
      }
    }
    BMG_TRY(upload(&D.cols, cols.data(), nw, s, D.bytes));
    BMG_TRY(upload(&D.a64, a.data(), nw, s, D.bytes));
    BMG_TRY(upload(&D.m64, mm.data(), nw, s, D.bytes));
    keep32.emplace_back(a.begin(), a.end());
    BMG_TRY(upload(&D.a32, keep32.back().data(), nw, s, D.bytes));
    keep32.emplace_back(mm.begin(), mm.end());
    BMG_TRY(upload(&D.m32, keep32.back().data(), nw, s, D.bytes));
    std::vector<double> dinv(H.n);
    for (int64_t r = 0; r < H.n; ++r) dinv[r] = 1.0 / H.lumped[size_t(nat(r))];
    BMG_TRY(upload(&D.dinv, dinv.data(), size_t(H.n), s, D.bytes));
    // transfer tables between this level and the one below
    std::vector<int32_t> par, rtab(H.rtab.size()), rself;
    if (l > 0) {
      if (permuted) {
        par.resize(size_t(H.n) * 2);
        for (int64_t r = 0; r < H.n; ++r) {
          const int64_t q = nat(r);
          if (q < H.n_prev) {
            par[2 * r] = par[2 * r + 1] = cnew(int32_t(q));
          } else {
            par[2 * r] = cnew(H.parents[size_t(2 * (q - H.n_prev))]);
            par[2 * r + 1] = cnew(H.parents[size_t(2 * (q - H.n_prev) + 1)]);
          }
        }
        // coarse storage row i is vertex c of the level below; its own copy
        // and its adjacent new vertices in this level's storage
        rself.resize(size_t(H.n_prev));
        std::vector<int32_t> cnat(size_t(H.n_prev));  // coarse storage row -> vertex
        for (int64_t c = 0; c < H.n_prev; ++c) cnat[size_t(cnew(int32_t(c)))] = int32_t(c);
        for (int64_t i = 0; i < H.n_prev; ++i) {
          const int32_t c = cnat[size_t(i)];
          rself[size_t(i)] = snew(c);
          for (int k = 0; k < H.RW; ++k) {
            const int32_t j = H.rtab[size_t(c) * H.RW + k];
            rtab[size_t(i) * H.RW + k] = j < 0 ? -1 : snew(j);
          }
        }
        D.par_nc = 0;
      } else {
        // nested numbering (the level below is then not permuted either)
        par = H.parents;
        rtab = H.rtab;
        D.par_nc = H.n_prev;
      }
    }
    BMG_TRY(upload(&D.parents, par.data(), par.size(), s, D.bytes));
    BMG_TRY(upload(&D.rtab, rtab.data(), rtab.size(), s, D.bytes));
    BMG_TRY(upload(&D.rself, rself.data(), rself.size(), s, D.bytes));
    std::vector<int32_t> crows(H.colour_rows.size()), c2rows(H.colour2_rows.size());
    for (size_t i = 0; i < crows.size(); ++i) crows[i] = snew(H.colour_rows[i]);
    for (size_t i = 0; i < c2rows.size(); ++i) c2rows[i] = snew(H.colour2_rows[i]);
    BMG_TRY(upload(&D.colour_rows, crows.data(), crows.size(), s, D.bytes));
    BMG_TRY(upload(&D.colour2_rows, c2rows.data(), c2rows.size(), s, D.bytes));
    D.n_colours2 = H.n_colours2;
    D.colour2_ptr = H.colour2_ptr;
    if (permuted) {
      BMG_TRY(upload(&D.perm, perm.data(), perm.size(), s, D.bytes));
      BMG_TRY(upload(&D.iperm, iperm.data(), iperm.size(), s, D.bytes));
      D.perm_h = perm;
    }
    // the fused Gram's chunk order: only where the storage is in index order
    std::vector<int32_t> cord;
    if (!permuted && H.n >= kChunkOrderMinRows) {
      cord = chunk_morton_order(H);
      BMG_TRY(upload(&D.chunk_order, cord.data(), cord.size(), s, D.bytes));
    }
    BMG_HIP(hipStreamSynchronize(s));  // the staging vectors are locals
    iperm_prev = std::move(iperm);
  }
  // level-0 eigendecomposition on the device (FP64 and FP32, with transposes)
  const int64_t n0 = h->n0;
  std::vector<double> t64(size_t(n0) * n0);
  for (int64_t i = 0; i < n0; ++i)
    for (int64_t j = 0; j < n0; ++j) t64[size_t(j) * n0 + i] = h->phi0[size_t(i) * n0 + j];
  std::vector<float> p32(h->phi0.begin(), h->phi0.end()), t32(t64.begin(), t64.end());
  int64_t b0 = 0;
  BMG_TRY(upload(&h->d_phi0_64, h->phi0.data(), h->phi0.size(), s, b0));
  BMG_TRY(upload(&h->d_phi0t_64, t64.data(), t64.size(), s, b0));
  BMG_TRY(upload(&h->d_phi0_32, p32.data(), p32.size(), s, b0));
  BMG_TRY(upload(&h->d_phi0t_32, t32.data(), t32.size(), s, b0));
  h->dev[0].bytes += b0;
  BMG_HIP(hipStreamSynchronize(s));
  return BMG_OK;
}

namespace {
std::shared_mutex g_capture_mu;
thread_local int t_sync_depth = 0;
}  // namespace

DeviceSyncGuard::DeviceSyncGuard() {
  if (t_sync_depth++ == 0) g_capture_mu.lock();
}
DeviceSyncGuard::~DeviceSyncGuard() {
  if (--t_sync_depth == 0) g_capture_mu.unlock();
}
CaptureGuard::CaptureGuard() { g_capture_mu.lock_shared(); }
CaptureGuard::~CaptureGuard() { g_capture_mu.unlock_shared(); }

void dev_free(void* p) {
  if (p == nullptr) return;
  DeviceSyncGuard g;
  (void)hipFree(p);
}

int level_eig(bmg_hierarchy* h, int l, hipStream_t s, const LevelEig** out) {
  TraceRange trace("bmg_level_eig");
  std::lock_guard<std::mutex> g(h->eig_mutex);
  const int nl = int(h->host.size());
  BMG_CHECK(l >= 0 && l < nl, "level %d out of range", l);
  if (h->level_eig.size() < size_t(nl)) h->level_eig.resize(nl);
  if (h->level_eig[l]) {
    *out = h->level_eig[l].get();
    return BMG_OK;
  }
  const HostLevel& H = h->host[l];
  const int n = int(H.n);
  BMG_CHECK(H.n <= kLevelEigMax, "level %d has %lld vertices; the dense eigensolve takes at most %d", l,
            (long long)H.n, kLevelEigMax);
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> A(size_t(n) * n, 0.0), M(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < H.W; ++k) {
      const int j = H.cols[size_t(i) * H.W + k];
      A[size_t(i) * n + j] += H.a[size_t(i) * H.W + k];
      M[size_t(i) * n + j] += H.mm[size_t(i) * H.W + k];
    }
  auto e = std::make_unique<LevelEig>();
  e->level = l;
  e->n = n;
  const size_t nn = size_t(n) * n;
  if (n <= kHostEigMax) {
    std::vector<double> X;
    BMG_TRY(dense_sygv(n, A, M, e->lam, X));
    std::vector<double> rows(nn);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) rows[size_t(j) * n + i] = X[size_t(i) * n + j];
    BMG_TRY(upload(&e->d_phi64, rows.data(), nn, s, e->bytes));
    BMG_HIP(hipStreamSynchronize(s));  // rows is a local
  } else {
    A.shrink_to_fit();
    BMG_TRY(device_sygv_keep(n, A, M, e->lam, &e->d_phi64, s));
    e->bytes += int64_t(nn * sizeof(double));
  }
  BMG_TRY(upload(&e->d_lam, e->lam.data(), size_t(n), s, e->bytes));
  if (hipMalloc(reinterpret_cast<void**>(&e->d_phi32), nn * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    dev_free(e->d_phi64);
    dev_free(e->d_lam);
    set_error("hipMalloc of %zu bytes failed", nn * sizeof(float));
    return BMG_ENOMEM;
  }
  e->bytes += int64_t(nn * sizeof(float));
  BMG_TRY(launch_convert<float>(e->d_phi64, e->d_phi32, int64_t(nn), s));
  BMG_HIP(hipStreamSynchronize(s));  // lam is uploaded from the object itself; keep it simple
  e->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  h->level_eig[l] = std::move(e);
  *out = h->level_eig[l].get();
  return BMG_OK;
}

void free_level_eigs(bmg_hierarchy* h) {
  std::lock_guard<std::mutex> g(h->eig_mutex);
  for (auto& e : h->level_eig) {
    if (!e) continue;
    for (void* p : {(void*)e->d_lam, (void*)e->d_phi64, (void*)e->d_phi32})
      if (p) dev_free(p);
    e.reset();
  }
  h->level_eig.clear();
}

void free_device(bmg_hierarchy* h) {
  free_level_eigs(h);
  free_est_levels(h);
  for (auto& D : h->dev) {
    void* ptrs[] = {D.cols, D.a64, D.m64, D.a32, D.m32, D.dinv, D.parents, D.rtab, D.rself, D.colour_rows,
                     D.chunk_order, D.colour2_rows, D.perm, D.iperm};
    for (void* p : ptrs)
      if (p) dev_free(p);
    D = DevLevel();
  }
  void* ptrs[] = {h->d_phi0_64, h->d_phi0t_64, h->d_phi0_32, h->d_phi0t_32};
  for (void* p : ptrs)
    if (p) dev_free(p);
  h->d_phi0_64 = h->d_phi0t_64 = nullptr;
  h->d_phi0_32 = h->d_phi0t_32 = nullptr;
}

}  // namespace bmg
