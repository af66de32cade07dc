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

// Levels with at least this many rows get a row order (smaller levels stay in
// the caches in any order); BMG_ROW_ORDER_MIN_ROWS overrides it.
int64_t row_order_min_rows() {
  if (const char* e = std::getenv("BMG_ROW_ORDER_MIN_ROWS")) return std::atoll(e);
  return 131072;
}

}  // namespace

int upload_hierarchy(bmg_hierarchy* h, hipStream_t s) {
  const int nl = int(h->host.size());
  h->dev.resize(nl);
  std::vector<std::vector<float>> keep32;  // host staging must live until the stream syncs
  const int64_t min_ordered = row_order_min_rows();
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
    BMG_TRY(upload(&D.cols, H.cols.data(), nw, s, D.bytes));
    BMG_TRY(upload(&D.a64, H.a.data(), nw, s, D.bytes));
    BMG_TRY(upload(&D.m64, H.mm.data(), nw, s, D.bytes));
    keep32.emplace_back(H.a.begin(), H.a.end());
    BMG_TRY(upload(&D.a32, keep32.back().data(), nw, s, D.bytes));
    keep32.emplace_back(H.mm.begin(), H.mm.end());
    BMG_TRY(upload(&D.m32, keep32.back().data(), nw, s, D.bytes));
    std::vector<double> dinv(H.n);
    for (int64_t i = 0; i < H.n; ++i) dinv[i] = 1.0 / H.lumped[i];
    BMG_TRY(upload(&D.dinv, dinv.data(), size_t(H.n), s, D.bytes));
    BMG_TRY(upload(&D.parents, H.parents.data(), H.parents.size(), s, D.bytes));
    BMG_TRY(upload(&D.rtab, H.rtab.data(), H.rtab.size(), s, D.bytes));
    BMG_TRY(upload(&D.colour_rows, H.colour_rows.data(), H.colour_rows.size(), s, D.bytes));
    BMG_TRY(upload(&D.colour2_rows, H.colour2_rows.data(), H.colour2_rows.size(), s, D.bytes));
    D.n_colours2 = H.n_colours2;
    D.colour2_ptr = H.colour2_ptr;
    std::vector<int32_t> ord;
    if (H.n >= min_ordered) {
      ord = morton_order(H.xyz);
      BMG_TRY(upload(&D.row_order, ord.data(), ord.size(), s, D.bytes));
    }
    std::vector<int32_t> cord;
    if (H.n >= kChunkOrderMinRows) {
      cord = chunk_morton_order(H);
      BMG_TRY(upload(&D.chunk_order, cord.data(), cord.size(), s, D.bytes));
    }
    BMG_HIP(hipStreamSynchronize(s));  // dinv, ord and cord are locals
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
    (void)hipFree(e->d_phi64);
    (void)hipFree(e->d_lam);
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
      if (p) (void)hipFree(p);
    e.reset();
  }
  h->level_eig.clear();
}

void free_device(bmg_hierarchy* h) {
  free_level_eigs(h);
  free_est_levels(h);
  for (auto& D : h->dev) {
    void* ptrs[] = {D.cols, D.a64, D.m64, D.a32, D.m32, D.dinv, D.parents, D.rtab, D.colour_rows, D.row_order, D.chunk_order, D.colour2_rows};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    D = DevLevel();
  }
  void* ptrs[] = {h->d_phi0_64, h->d_phi0t_64, h->d_phi0_32, h->d_phi0t_32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->d_phi0_64 = h->d_phi0t_64 = nullptr;
  h->d_phi0_32 = h->d_phi0t_32 = nullptr;
}

}  // namespace bmg
