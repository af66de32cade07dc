// A posteriori error estimator of eq. est-res (Sec. 5): host side.  The
// triangle data of a level (vertex indices, edge neighbours, coordinates) is
// uploaded on first use and kept with the hierarchy.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>
#include <vector>

#include "bmg_internal.h"

namespace bmg {

namespace {

int est_level(bmg_hierarchy* h, int l, hipStream_t s, const EstLevel** out) {
  std::lock_guard<std::mutex> g(h->est_mutex);
  const int nl = int(h->host.size());
  if (h->est.size() < size_t(nl)) h->est.resize(nl);
  if (h->est[l]) {
    *out = h->est[l].get();
    return BMG_OK;
  }
  const HostLevel& H = h->host[l];
  const int64_t F = H.n_tri;
  // neighbour across edge i (opposite vertex i) of every triangle
  std::vector<int32_t> nbr(size_t(3 * F), -1);
  {
    std::vector<std::pair<std::pair<int32_t, int32_t>, int64_t>> E;  // (edge, 4 t + i)
    E.reserve(size_t(3 * F));
    for (int64_t t = 0; t < F; ++t)
      for (int i = 0; i < 3; ++i) {
        const int32_t a = H.tri[size_t(3 * t + (i + 1) % 3)], b = H.tri[size_t(3 * t + (i + 2) % 3)];
        E.push_back({{std::min(a, b), std::max(a, b)}, 4 * t + i});
      }
    std::sort(E.begin(), E.end());
    for (size_t q = 0; q + 1 < E.size(); ++q)
      if (E[q].first == E[q + 1].first) {
        const int64_t p = E[q].second, r = E[q + 1].second;
        nbr[size_t(3 * (p >> 2) + (p & 3))] = int32_t(r);
        nbr[size_t(3 * (r >> 2) + (r & 3))] = int32_t(p);
        ++q;
      }
    for (int32_t v : nbr) BMG_CHECK(v >= 0, "level %d has an edge without a second triangle", l);
  }
  auto e = std::make_unique<EstLevel>();
  e->level = l;
  e->F = F;
  auto up = [&](void** dst, const void* src, size_t bytes) -> int {
    if (hipMalloc(dst, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of %zu bytes failed", bytes);
      return BMG_ENOMEM;
    }
    e->bytes += int64_t(bytes);
    BMG_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
    return BMG_OK;
  };
  int st = up(reinterpret_cast<void**>(&e->tri), H.tri.data(), sizeof(int32_t) * H.tri.size());
  if (st == BMG_OK) st = up(reinterpret_cast<void**>(&e->nbr), nbr.data(), sizeof(int32_t) * nbr.size());
  if (st == BMG_OK) st = up(reinterpret_cast<void**>(&e->xyz), H.xyz.data(), sizeof(double) * H.xyz.size());
  if (st == BMG_OK && hipStreamSynchronize(s) != hipSuccess) st = BMG_EDEVICE;  // nbr is a local
  if (st != BMG_OK) {
    for (void* p : {static_cast<void*>(e->tri), static_cast<void*>(e->nbr), static_cast<void*>(e->xyz)})
      if (p) dev_free(p);
    return st;
  }
  *out = e.get();
  h->est[l] = std::move(e);
  return BMG_OK;
}

}  // namespace

void free_est_levels(bmg_hierarchy* h) {
  std::lock_guard<std::mutex> g(h->est_mutex);
  for (auto& e : h->est) {
    if (!e) continue;
    for (void* p : {static_cast<void*>(e->tri), static_cast<void*>(e->nbr), static_cast<void*>(e->xyz)})
      if (p) dev_free(p);
    e.reset();
  }
  h->est.clear();
}

int estimate(bmg_hierarchy* h, int level, int k, const double* evals, const double* evecs, int64_t ld,
             double* eta, double* parts, double* eta2_T, hipStream_t s) {
  TraceRange trace("bmg_estimate");
  const int nl = int(h->dev.size());
  BMG_CHECK(level >= 0 && level < nl, "level %d out of range", level);
  BMG_CHECK(k >= 1 && k <= 4096, "k = %d must be in [1, 4096]", k);
  BMG_CHECK(evals && evecs && eta, "evals, evecs and eta must be non-NULL");
  BMG_CHECK(ld >= h->host[level].n, "ld = %lld < N = %lld", (long long)ld, (long long)h->host[level].n);
  for (int j = 0; j < k; ++j) BMG_CHECK(std::isfinite(evals[j]), "evals[%d] is not finite", j);
  BMG_HIP(hipSetDevice(h->device));
  const EstLevel* E = nullptr;
  BMG_TRY(est_level(h, level, s, &E));
  const int nblk = est_blocks(E->F);
  double *part = nullptr, *lam = nullptr, *out = nullptr;
  std::vector<void*> bufs;
  auto alloc = [&](double** p, size_t count) -> int {
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of %zu bytes failed", count * sizeof(double));
      return BMG_ENOMEM;
    }
    bufs.push_back(*p);
    return BMG_OK;
  };
  auto run = [&]() -> int {
    BMG_TRY(alloc(&part, size_t(nblk) * k * 3));
    BMG_TRY(alloc(&lam, size_t(k)));
    BMG_TRY(alloc(&out, size_t(3 * k)));
    BMG_HIP(hipMemcpyAsync(lam, evals, sizeof(double) * k, hipMemcpyHostToDevice, s));
    BMG_TRY(launch_estimate(*E, k, evecs, ld, lam, h->kind == BMG_SPHERE ? 1 : 0, eta2_T, part, out, s));
    std::vector<double> o(size_t(3 * k));
    BMG_HIP(hipMemcpyAsync(o.data(), out, sizeof(double) * o.size(), hipMemcpyDeviceToHost, s));
    BMG_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) eta[j] = std::sqrt(o[size_t(j)] + o[size_t(k + j)] + o[size_t(2 * k + j)]);
    if (parts) std::copy(o.begin(), o.end(), parts);
    return BMG_OK;
  };
  const int st = run();
  (void)hipStreamSynchronize(s);
  for (void* p : bufs) dev_free(p);
  return st;
}

}  // namespace bmg
