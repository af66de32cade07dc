// Surface meshes and uniform refinement with projected midpoints.
//
// Paper Sec. 3 (opening paragraphs, Fig. 2): the fine mesh is the uniform
// refinement of the coarse one; the midpoints of the coarse edges become new
// vertices and are moved onto the surface (closest-point lift, eq. lift), so
// every vertex lies on Gamma (Sec. 2.1).  Numbering used by this library:
// coarse edges (a<b) in lexicographic order, midpoint of edge e = vertex
// N_coarse + e; triangle (a,b,c) -> (a,ab,ca), (ab,b,bc), (ca,bc,c), (ab,bc,ca).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>

#include "bmg_internal.h"

namespace bmg {
namespace {

using Vec3 = std::array<double, 3>;

void orient_outward_origin(const std::vector<double>& xyz, std::vector<int32_t>& tri) {
  for (size_t t = 0; t < tri.size() / 3; ++t) {
    int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    double u[3], v[3], n[3], cen[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = xyz[3 * b + k] - xyz[3 * a + k];
      v[k] = xyz[3 * c + k] - xyz[3 * a + k];
      cen[k] = xyz[3 * a + k] + xyz[3 * b + k] + xyz[3 * c + k];
    }
    n[0] = u[1] * v[2] - u[2] * v[1];
    n[1] = u[2] * v[0] - u[0] * v[2];
    n[2] = u[0] * v[1] - u[1] * v[0];
    if (n[0] * cen[0] + n[1] * cen[1] + n[2] * cen[2] < 0) std::swap(tri[3 * t + 1], tri[3 * t + 2]);
  }
}

// Regular icosahedron inscribed in the unit sphere; faces are the vertex
// triples pairwise at unnormalised distance 2, oriented outward, rotated so
// the smallest index is first, sorted lexicographically.
void icosahedron(std::vector<double>& xyz, std::vector<int32_t>& tri) {
  const double p = (1.0 + std::sqrt(5.0)) / 2.0;
  const double v[12][3] = {{-1, p, 0}, {1, p, 0}, {-1, -p, 0}, {1, -p, 0}, {0, -1, p}, {0, 1, p},
                           {0, -1, -p}, {0, 1, -p}, {p, 0, -1}, {p, 0, 1}, {-p, 0, -1}, {-p, 0, 1}};
  auto dist = [&](int i, int j) {
    double s = 0;
    for (int k = 0; k < 3; ++k) s += (v[i][k] - v[j][k]) * (v[i][k] - v[j][k]);
    return std::sqrt(s);
  };
  tri.clear();
  for (int a = 0; a < 12; ++a)
    for (int b = a + 1; b < 12; ++b)
      for (int c = b + 1; c < 12; ++c)
        if (std::fabs(dist(a, b) - 2) < 1e-9 && std::fabs(dist(b, c) - 2) < 1e-9 &&
            std::fabs(dist(a, c) - 2) < 1e-9) {
          tri.push_back(a);
          tri.push_back(b);
          tri.push_back(c);
        }
  std::vector<double> raw(36);
  for (int i = 0; i < 12; ++i)
    for (int k = 0; k < 3; ++k) raw[3 * i + k] = v[i][k];
  orient_outward_origin(raw, tri);
  const size_t nt = tri.size() / 3;
  std::vector<std::array<int32_t, 3>> t3(nt);
  for (size_t t = 0; t < nt; ++t) {
    int32_t x[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    int k = int(std::min_element(x, x + 3) - x);
    t3[t] = {x[k], x[(k + 1) % 3], x[(k + 2) % 3]};
  }
  std::sort(t3.begin(), t3.end());
  for (size_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) tri[3 * t + k] = t3[t][k];
  xyz.resize(36);
  for (int i = 0; i < 12; ++i) {
    double r = std::sqrt(raw[3 * i] * raw[3 * i] + raw[3 * i + 1] * raw[3 * i + 1] +
                         raw[3 * i + 2] * raw[3 * i + 2]);
    for (int k = 0; k < 3; ++k) xyz[3 * i + k] = raw[3 * i + k] / r;
  }
}

void torus_grid(double R, double r, int nu, int nv, std::vector<double>& xyz,
                std::vector<int32_t>& tri) {
  xyz.assign(size_t(3) * nu * nv, 0.0);
  for (int i = 0; i < nu; ++i) {
    double u = 2.0 * M_PI * i / nu;
    for (int j = 0; j < nv; ++j) {
      double w = 2.0 * M_PI * j / nv;
      size_t id = size_t(nv) * i + j;
      xyz[3 * id] = (R + r * std::cos(w)) * std::cos(u);
      xyz[3 * id + 1] = (R + r * std::cos(w)) * std::sin(u);
      xyz[3 * id + 2] = r * std::sin(w);
    }
  }
  tri.clear();
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nv; ++j) {
      int p00 = nv * i + j, p10 = nv * ((i + 1) % nu) + j;
      int p11 = nv * ((i + 1) % nu) + (j + 1) % nv, p01 = nv * i + (j + 1) % nv;
      int32_t t1[3] = {p00, p10, p11}, t2[3] = {p00, p11, p01};
      for (int32_t* t : {t1, t2}) {
        // outward: normal away from the tube's centre circle
        double a[3], b[3], n[3], cen[3];
        for (int k = 0; k < 3; ++k) {
          a[k] = xyz[3 * t[1] + k] - xyz[3 * t[0] + k];
          b[k] = xyz[3 * t[2] + k] - xyz[3 * t[0] + k];
          cen[k] = (xyz[3 * t[0] + k] + xyz[3 * t[1] + k] + xyz[3 * t[2] + k]) / 3.0;
        }
        n[0] = a[1] * b[2] - a[2] * b[1];
        n[1] = a[2] * b[0] - a[0] * b[2];
        n[2] = a[0] * b[1] - a[1] * b[0];
        double rho = std::hypot(cen[0], cen[1]);
        double d[3] = {cen[0] - R * cen[0] / rho, cen[1] - R * cen[1] / rho, cen[2]};
        if (n[0] * d[0] + n[1] * d[1] + n[2] * d[2] < 0) std::swap(t[1], t[2]);
        tri.insert(tri.end(), t, t + 3);
      }
    }
}

// Closed, consistently oriented 2-manifold: every directed edge appears once
// and its reverse appears once.
int check_manifold(int64_t n, const std::vector<int32_t>& tri) {
  std::vector<std::pair<int64_t, int64_t>> de;
  de.reserve(tri.size());
  for (size_t t = 0; t < tri.size() / 3; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      BMG_CHECK(a >= 0 && a < n && b >= 0 && b < n && a != b, "triangle %zu has an invalid vertex", t);
      de.push_back({a, b});
    }
  std::sort(de.begin(), de.end());
  for (size_t i = 1; i < de.size(); ++i)
    BMG_CHECK(de[i] != de[i - 1], "directed edge (%lld,%lld) used twice: not an oriented manifold",
              (long long)de[i].first, (long long)de[i].second);
  for (auto& e : de)
    BMG_CHECK(std::binary_search(de.begin(), de.end(), std::make_pair(e.second, e.first)),
              "edge (%lld,%lld) has no opposite triangle: surface not closed", (long long)e.first,
              (long long)e.second);
  std::vector<char> used(n, 0);
  for (int32_t v : tri) used[v] = 1;
  for (int64_t i = 0; i < n; ++i) BMG_CHECK(used[i], "vertex %lld is in no triangle", (long long)i);
  return BMG_OK;
}

// Uniform refinement; `project` moves a midpoint onto Gamma in place.
void refine(const HostLevel& c, HostLevel& f, const std::function<void(double*)>& project) {
  const int64_t n = c.n;
  const size_t nt = c.tri.size() / 3;
  std::vector<std::pair<int32_t, int32_t>> E;
  E.reserve(3 * nt);
  for (size_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t a = c.tri[3 * t + k], b = c.tri[3 * t + (k + 1) % 3];
      E.push_back({std::min(a, b), std::max(a, b)});
    }
  std::sort(E.begin(), E.end());
  E.erase(std::unique(E.begin(), E.end()), E.end());
  auto mid = [&](int32_t a, int32_t b) -> int32_t {
    std::pair<int32_t, int32_t> key{std::min(a, b), std::max(a, b)};
    return int32_t(n + (std::lower_bound(E.begin(), E.end(), key) - E.begin()));
  };
  f.n_prev = n;
  f.n = n + int64_t(E.size());
  f.xyz.resize(3 * f.n);
  std::memcpy(f.xyz.data(), c.xyz.data(), sizeof(double) * 3 * n);
  f.parents.resize(2 * E.size());
  for (size_t e = 0; e < E.size(); ++e) {
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = 0.5 * (c.xyz[3 * E[e].first + k] + c.xyz[3 * E[e].second + k]);
    project(p);
    for (int k = 0; k < 3; ++k) f.xyz[3 * (n + e) + k] = p[k];
    f.parents[2 * e] = E[e].first;
    f.parents[2 * e + 1] = E[e].second;
  }
  f.n_tri = 4 * int64_t(nt);
  f.tri.resize(3 * f.n_tri);
  for (size_t t = 0; t < nt; ++t) {
    int32_t a = c.tri[3 * t], b = c.tri[3 * t + 1], cc = c.tri[3 * t + 2];
    int32_t ab = mid(a, b), bc = mid(b, cc), ca = mid(cc, a);
    int32_t ch[12] = {a, ab, ca, ab, b, bc, ca, bc, cc, ab, bc, ca};
    std::memcpy(&f.tri[12 * t], ch, sizeof(ch));
  }
}

}  // namespace

int build_host_levels(const bmg_surface_desc* d, int n_refine, std::vector<HostLevel>& out) {
  BMG_CHECK(d != nullptr, "surface descriptor is NULL");
  BMG_CHECK(n_refine >= 0 && n_refine <= 10, "n_refine must be in [0, 10]");
  out.clear();
  out.resize(n_refine + 1);
  HostLevel& l0 = out[0];
  std::function<void(double*)> project;
  const int kind = d->kind;
  if (kind == BMG_SPHERE || kind == BMG_ELLIPSOID) {
    if (kind == BMG_ELLIPSOID)
      BMG_CHECK(d->axes[0] > 0 && d->axes[1] > 0 && d->axes[2] > 0 && std::isfinite(d->axes[0]) &&
                    std::isfinite(d->axes[1]) && std::isfinite(d->axes[2]),
                "ellipsoid semi-axes must be positive and finite");
    icosahedron(l0.xyz, l0.tri);
    project = [](double* p) {
      double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      p[0] /= r;
      p[1] /= r;
      p[2] /= r;
    };
  } else if (kind == BMG_TORUS) {
    const double R = d->R, r = d->r;
    BMG_CHECK(R > r && r > 0 && std::isfinite(R), "torus radii must satisfy R > r > 0");
    BMG_CHECK(d->nu >= 3 && d->nv >= 3 && int64_t(d->nu) * d->nv <= 4096, "torus grid nu, nv >= 3, nu*nv <= 4096");
    torus_grid(R, r, d->nu, d->nv, l0.xyz, l0.tri);
    project = [R, r](double* p) {
      double rho = std::hypot(p[0], p[1]);
      double c[3] = {R * p[0] / rho, R * p[1] / rho, 0.0};
      double v[3] = {p[0] - c[0], p[1] - c[1], p[2]};
      double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      for (int k = 0; k < 3; ++k) p[k] = c[k] + r * v[k] / s;
    };
  } else if (kind == BMG_CUSTOM) {
    BMG_CHECK(d->xyz && d->tri && d->n_vert >= 4 && d->n_tri >= 4 && d->n_vert <= 4096,
              "custom mesh needs 4 <= n_vert <= 4096, n_tri >= 4 and non-NULL arrays");
    l0.xyz.assign(d->xyz, d->xyz + 3 * size_t(d->n_vert));
    l0.tri.assign(d->tri, d->tri + 3 * size_t(d->n_tri));
    for (double x : l0.xyz) BMG_CHECK(std::isfinite(x), "custom mesh has a non-finite coordinate");
    void (*cb)(double*, void*) = d->project;
    void* ctx = d->ctx;
    project = [cb, ctx](double* p) {
      if (cb) cb(p, ctx);
    };
  } else {
    BMG_CHECK(false, "unknown surface kind %d", kind);
  }
  l0.n = int64_t(l0.xyz.size() / 3);
  l0.n_tri = int64_t(l0.tri.size() / 3);
  l0.n_prev = 0;
  BMG_TRY(check_manifold(l0.n, l0.tri));
  for (int l = 1; l <= n_refine; ++l) refine(out[l - 1], out[l], project);
  if (kind == BMG_ELLIPSOID)
    for (auto& lv : out)
      for (int64_t i = 0; i < lv.n; ++i)
        for (int k = 0; k < 3; ++k) lv.xyz[3 * i + k] *= d->axes[k];
  if (kind == BMG_CUSTOM)
    for (auto& lv : out)
      for (double x : lv.xyz) BMG_CHECK(std::isfinite(x), "projection produced a non-finite point");
  return BMG_OK;
}

}  // namespace bmg
