// Host-side set-up code of the library (mesh construction, P1 assembly to
// ELL, colouring, restriction tables, Morton orders, the dense Jacobi
// eigensolver) run under AddressSanitizer and UndefinedBehaviorSanitizer,
// with invariants checked on the way.  Built and run by
// tests/test_host_sanitizers.py with clang++ (host code only, no device code).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "bmg_internal.h"

namespace bmg {
// The library's error buffer lives in the C-ABI source; these checks keep
// their own.
static std::string g_err;
void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
const char* get_error() { return g_err.c_str(); }
}  // namespace bmg

using namespace bmg;

static int g_fail = 0;
#define EXPECT(c, ...)                        \
  do {                                        \
    if (!(c)) {                               \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);      \
      std::fprintf(stderr, "\n");             \
      ++g_fail;                               \
    }                                         \
  } while (0)

static bool is_permutation(const std::vector<int32_t>& p, int64_t n) {
  if (int64_t(p.size()) != n) return false;
  std::vector<char> seen(size_t(n), 0);
  for (int32_t v : p) {
    if (v < 0 || v >= n || seen[size_t(v)]) return false;
    seen[size_t(v)] = 1;
  }
  return true;
}

static void check_level(const char* name, int l, const HostLevel& H, const HostLevel* C) {
  const int64_t n = H.n;
  EXPECT(int64_t(H.cols.size()) == n * H.W && H.a.size() == H.cols.size() && H.mm.size() == H.cols.size(),
         "%s level %d: ELL sizes", name, l);
  double worst_rowsum = 0.0, amax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    EXPECT(H.cols[size_t(i * H.W)] == i, "%s level %d: row %lld diagonal not first", name, l, (long long)i);
    double rs = 0.0, ms = 0.0;
    for (int k = 0; k < H.W; ++k) {
      const int32_t j = H.cols[size_t(i * H.W + k)];
      EXPECT(j >= 0 && j < n, "%s level %d: column out of range", name, l);
      rs += H.a[size_t(i * H.W + k)];
      ms += H.mm[size_t(i * H.W + k)];
      amax = std::max(amax, std::fabs(H.a[size_t(i * H.W + k)]));
      // a proper colouring: no neighbour shares the row's colour
      if (j != i && H.a[size_t(i * H.W + k)] != 0.0)
        EXPECT(H.colour[size_t(i)] != H.colour[size_t(j)], "%s level %d: edge inside a colour", name, l);
    }
    worst_rowsum = std::max(worst_rowsum, std::fabs(rs));
    EXPECT(std::fabs(ms - H.lumped[size_t(i)]) <= 1e-12 * std::fabs(ms), "%s level %d: lumped mass", name, l);
  }
  EXPECT(worst_rowsum <= 1e-12 * amax, "%s level %d: A row sums %g", name, l, worst_rowsum);
  EXPECT(int64_t(H.colour_ptr.size()) == H.n_colours + 1 && H.colour_ptr.back() == n, "%s level %d: colour_ptr",
         name, l);
  EXPECT(is_permutation(H.colour_rows, n), "%s level %d: colour rows not a permutation", name, l);
  if (C) {
    EXPECT(H.n_prev == C->n && int64_t(H.rtab.size()) == C->n * H.RW, "%s level %d: rtab size", name, l);
    for (int32_t v : H.rtab) EXPECT(v == -1 || (v >= C->n && v < n), "%s level %d: rtab entry %d", name, l, v);
    for (size_t e = 0; e < H.parents.size(); ++e)
      EXPECT(H.parents[e] >= 0 && H.parents[e] < C->n, "%s level %d: parent out of range", name, l);
  }
  EXPECT(is_permutation(morton_order(H.xyz), n), "%s level %d: Morton order", name, l);
  EXPECT(is_permutation(chunk_morton_order(H), (n + 15) / 16), "%s level %d: chunk order", name, l);
}

static void check_eig(const char* name, const HostLevel& H) {
  const int n = int(H.n);
  std::vector<double> A(size_t(n) * n, 0.0), M(size_t(n) * n, 0.0), lam, X;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < H.W; ++k) {
      const int j = H.cols[size_t(i) * H.W + k];
      A[size_t(i) * n + j] += H.a[size_t(i) * H.W + k];
      M[size_t(i) * n + j] += H.mm[size_t(i) * H.W + k];
    }
  EXPECT(dense_sygv(n, A, M, lam, X) == BMG_OK, "%s: dense_sygv failed: %s", name, get_error());
  if (int(lam.size()) != n) return;
  double orth = 0.0, res = 0.0, anorm = 0.0;
  for (double v : A) anorm = std::max(anorm, std::fabs(v));
  for (int p = 0; p < n; ++p) {
    EXPECT(p == 0 || lam[size_t(p)] >= lam[size_t(p - 1)], "%s: eigenvalues not ascending", name);
    for (int q = 0; q < n; ++q) {
      double g = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) g += X[size_t(i) * n + p] * M[size_t(i) * n + j] * X[size_t(j) * n + q];
      orth = std::max(orth, std::fabs(g - (p == q ? 1.0 : 0.0)));
    }
    for (int i = 0; i < n; ++i) {
      double r = 0.0;
      for (int j = 0; j < n; ++j) r += (A[size_t(i) * n + j] - lam[size_t(p)] * M[size_t(i) * n + j]) * X[size_t(j) * n + p];
      res = std::max(res, std::fabs(r));
    }
  }
  EXPECT(orth < 1e-10, "%s: X^T M X - I = %g", name, orth);
  EXPECT(res < 1e-10 * std::max(1.0, anorm), "%s: residual %g", name, res);
  std::printf("%s: n %d, lambda %.6g .. %.6g, orth %.1e, residual %.1e\n", name, n, lam.front(), lam.back(),
              orth, res);
}

static void run(const char* name, const bmg_surface_desc& d, int n_refine, int eig_level) {
  std::vector<HostLevel> lv;
  const int st = build_host_levels(&d, n_refine, lv);
  EXPECT(st == BMG_OK, "%s: build_host_levels: %s", name, get_error());
  if (st != BMG_OK) return;
  for (size_t l = 0; l < lv.size(); ++l) {
    const int a = assemble_level(lv[l], l ? &lv[l - 1] : nullptr);
    EXPECT(a == BMG_OK, "%s level %zu: assemble_level: %s", name, l, get_error());
    if (a == BMG_OK) check_level(name, int(l), lv[l], l ? &lv[l - 1] : nullptr);
  }
  std::printf("%s: %zu levels, finest %lld vertices, width %d, %d colours\n", name, lv.size(),
              (long long)lv.back().n, lv.back().W, lv.back().n_colours);
  if (eig_level >= 0) check_eig(name, lv[size_t(eig_level)]);
}

static void project_unit(double p[3], void*) {
  const double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  for (int k = 0; k < 3; ++k) p[k] /= r;
}

int main() {
  bmg_surface_desc d{};
  d.kind = BMG_SPHERE;
  d.axes[0] = d.axes[1] = d.axes[2] = 1.0;
  run("sphere", d, 5, 2);
  d.kind = BMG_ELLIPSOID;
  d.axes[0] = 1.0, d.axes[1] = 1.5, d.axes[2] = 2.0;
  run("ellipsoid", d, 4, 1);
  bmg_surface_desc t{};
  t.kind = BMG_TORUS;
  t.R = 1.0, t.r = 0.4, t.nu = 64, t.nv = 32;
  run("torus", t, 1, -1);
  t.nu = 8, t.nv = 6;
  run("torus 8x6", t, 2, 0);
  // octagonal bipyramid: two vertices of valence 8 (ELL width 9)
  std::vector<double> xyz = {0, 0, 1, 0, 0, -1};
  for (int i = 0; i < 8; ++i) {
    xyz.push_back(std::cos(2 * M_PI * i / 8));
    xyz.push_back(std::sin(2 * M_PI * i / 8));
    xyz.push_back(0.0);
  }
  std::vector<int32_t> tri;
  for (int i = 0; i < 8; ++i) {
    const int a = 2 + i, b = 2 + (i + 1) % 8;
    tri.insert(tri.end(), {0, a, b, 1, b, a});
  }
  bmg_surface_desc c{};
  c.kind = BMG_CUSTOM;
  c.n_vert = 10, c.n_tri = 16, c.xyz = xyz.data(), c.tri = tri.data(), c.project = project_unit;
  run("bipyramid", c, 3, 0);
  // rejected inputs: an open surface, a vertex index out of range, a level count
  std::vector<HostLevel> lv;
  c.n_tri = 15;
  EXPECT(build_host_levels(&c, 1, lv) == BMG_EINVAL, "open surface accepted");
  c.n_tri = 16;
  tri[5] = 10;
  EXPECT(build_host_levels(&c, 1, lv) == BMG_EINVAL, "vertex index 10 of 10 accepted");
  tri[5] = 2 + 1;
  EXPECT(build_host_levels(&d, -1, lv) == BMG_EINVAL, "n_refine = -1 accepted");
  EXPECT(build_host_levels(&d, 11, lv) == BMG_EINVAL, "n_refine = 11 accepted");
  t.r = 1.5;
  EXPECT(build_host_levels(&t, 1, lv) == BMG_EINVAL, "torus with r > R accepted");
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
