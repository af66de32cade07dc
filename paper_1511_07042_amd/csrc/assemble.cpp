// P1 surface-FEM matrices of one level, stored in ELL form, plus the vertex
// colourings used by the multicolour Gauss-Seidel and Kaczmarz smoothers and
// the gather table of the restriction.
//
// Paper Sec. 2.1 (eq. bl-dis) and Sec. 2.2 (eq. sp-fe, pb-eig-fea): a_h and
// b_h integrate over flat triangles.  For a triangle with vertices x0, x1, x2
// and edge vectors e_i opposite vertex i (e_0 = x2 - x1, e_1 = x0 - x2,
// e_2 = x1 - x0), the P1 gradients are the rotated edges over 2|T|, which gives
//   A_ij += e_i.e_j / (4|T|) (i != j),  M_ij += |T|/12 (i != j),  M_ii += |T|/6,
// and A_ii = -sum_{j != i} A_ij (zero row sums, as e_0 + e_1 + e_2 = 0).
// Restriction = transpose of the prolongation of eq. proj-1 (Sec. 3): coarse
// vertex i gathers its own value and half of each new vertex created on an
// edge incident to i.
#include <algorithm>
#include <cmath>

#include "bmg_internal.h"

namespace bmg {

int assemble_level(HostLevel& lv, const HostLevel* coarser) {
  const int64_t n = lv.n;
  const int64_t nt = lv.n_tri;
  // adjacency (sorted neighbour lists)
  std::vector<std::vector<int32_t>> nb(n);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t a = lv.tri[3 * t + k], b = lv.tri[3 * t + (k + 1) % 3];
      nb[a].push_back(b);
      nb[b].push_back(a);
    }
  int32_t W = 1;
  for (int64_t i = 0; i < n; ++i) {
    auto& v = nb[i];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    W = std::max<int32_t>(W, int32_t(v.size()) + 1);
  }
  BMG_CHECK(W <= 31, "vertex valence %d exceeds 30", W - 1);
  lv.W = W;
  lv.cols.assign(size_t(n) * W, 0);
  lv.a.assign(size_t(n) * W, 0.0);
  lv.mm.assign(size_t(n) * W, 0.0);
  lv.nnz = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t* c = &lv.cols[size_t(i) * W];
    c[0] = int32_t(i);
    for (size_t k = 0; k < nb[i].size(); ++k) c[k + 1] = nb[i][k];
    for (int k = int(nb[i].size()) + 1; k < W; ++k) c[k] = int32_t(i);
    lv.nnz += int64_t(nb[i].size()) + 1;
  }
  auto slot = [&](int32_t i, int32_t j) -> size_t {
    const int32_t* c = &lv.cols[size_t(i) * W];
    for (int k = 1; k < W; ++k)
      if (c[k] == j) return size_t(i) * W + k;
    return size_t(-1);
  };
  lv.area = 0.0;
  lv.hmax = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t v[3] = {lv.tri[3 * t], lv.tri[3 * t + 1], lv.tri[3 * t + 2]};
    double x[3][3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) x[i][k] = lv.xyz[3 * size_t(v[i]) + k];
    double e[3][3];
    for (int k = 0; k < 3; ++k) {
      e[0][k] = x[2][k] - x[1][k];
      e[1][k] = x[0][k] - x[2][k];
      e[2][k] = x[1][k] - x[0][k];
    }
    double u[3], w[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = x[1][k] - x[0][k];
      w[k] = x[2][k] - x[0][k];
    }
    for (int i = 0; i < 3; ++i)
      lv.hmax = std::max(lv.hmax, std::sqrt(e[i][0] * e[i][0] + e[i][1] * e[i][1] + e[i][2] * e[i][2]));
    double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    BMG_CHECK(area > 0 && std::isfinite(area), "degenerate triangle %lld", (long long)t);
    lv.area += area;
    for (int i = 0; i < 3; ++i) {
      lv.mm[size_t(v[i]) * W] += area / 6.0;
      for (int j = 0; j < 3; ++j) {
        if (i == j) continue;
        const size_t s = slot(v[i], v[j]);
        const double dot = e[i][0] * e[j][0] + e[i][1] * e[j][1] + e[i][2] * e[j][2];
        lv.a[s] += dot / (4.0 * area);
        lv.mm[s] += area / 12.0;
      }
    }
  }
  lv.lumped.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double off = 0.0, ms = 0.0;
    for (int k = 1; k < W; ++k) off += lv.a[size_t(i) * W + k];
    lv.a[size_t(i) * W] = -off;
    for (int k = 0; k < W; ++k) ms += lv.mm[size_t(i) * W + k];
    lv.lumped[i] = ms;
  }
  // greedy colouring in increasing vertex index
  lv.colour.assign(n, -1);
  int32_t nc = 0;
  std::vector<int32_t> mark(W + 2, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t j : nb[i])
      if (j < i && lv.colour[j] < W + 2) mark[lv.colour[j]] = int32_t(i);
    int32_t c = 0;
    while (mark[c] == int32_t(i)) ++c;
    lv.colour[i] = c;
    nc = std::max(nc, c + 1);
  }
  lv.n_colours = nc;
  lv.colour_ptr.assign(nc + 1, 0);
  for (int64_t i = 0; i < n; ++i) lv.colour_ptr[lv.colour[i] + 1]++;
  for (int c = 0; c < nc; ++c) lv.colour_ptr[c + 1] += lv.colour_ptr[c];
  lv.colour_rows.assign(n, 0);
  {
    std::vector<int32_t> pos(lv.colour_ptr.begin(), lv.colour_ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) lv.colour_rows[pos[lv.colour[i]]++] = int32_t(i);
  }
  // distance-2 colouring for the Kaczmarz smoother: greedy in increasing
  // vertex index, each vertex taking the smallest colour not used by a
  // lower-numbered vertex within two edges (so the rows of a colour share no
  // column of S)
  lv.colour2.assign(n, -1);
  int32_t nc2 = 0;
  {
    std::vector<int64_t> seen;
    std::vector<int32_t> mark2;
    for (int64_t i = 0; i < n; ++i) {
      for (int32_t j : nb[i]) {
        if (j < i) {
          const int32_t cj = lv.colour2[j];
          if (cj >= int32_t(mark2.size())) mark2.resize(cj + 1, -1);
          mark2[cj] = int32_t(i);
        }
        for (int32_t k : nb[j])
          if (k < i) {
            const int32_t ck = lv.colour2[k];
            if (ck >= int32_t(mark2.size())) mark2.resize(ck + 1, -1);
            mark2[ck] = int32_t(i);
          }
      }
      int32_t c = 0;
      while (c < int32_t(mark2.size()) && mark2[c] == int32_t(i)) ++c;
      lv.colour2[i] = c;
      nc2 = std::max(nc2, c + 1);
    }
  }
  lv.n_colours2 = nc2;
  lv.colour2_ptr.assign(nc2 + 1, 0);
  for (int64_t i = 0; i < n; ++i) lv.colour2_ptr[lv.colour2[i] + 1]++;
  for (int c = 0; c < nc2; ++c) lv.colour2_ptr[c + 1] += lv.colour2_ptr[c];
  lv.colour2_rows.assign(n, 0);
  {
    std::vector<int32_t> pos(lv.colour2_ptr.begin(), lv.colour2_ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) lv.colour2_rows[pos[lv.colour2[i]]++] = int32_t(i);
  }
  // restriction gather table: new vertices adjacent to each coarse vertex
  lv.RW = 0;
  lv.rtab.clear();
  if (coarser) {
    const int64_t nc_v = coarser->n;
    std::vector<int32_t> cnt(nc_v, 0);
    const int64_t nnew = n - nc_v;
    for (int64_t e = 0; e < nnew; ++e) {
      cnt[lv.parents[2 * e]]++;
      cnt[lv.parents[2 * e + 1]]++;
    }
    int32_t RW = 1;
    for (int32_t c : cnt) RW = std::max(RW, c);
    lv.RW = RW;
    lv.rtab.assign(size_t(nc_v) * RW, -1);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t e = 0; e < nnew; ++e)
      for (int s = 0; s < 2; ++s) {
        int32_t p = lv.parents[2 * e + s];
        lv.rtab[size_t(p) * RW + cnt[p]++] = int32_t(nc_v + e);
      }
  }
  return BMG_OK;
}

}  // namespace bmg
