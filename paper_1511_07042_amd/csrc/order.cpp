// Row visiting orders of the large levels (host side, set-up only).
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "bmg_internal.h"

namespace bmg {

// Rows ordered along a Morton (Z-order) curve through the vertex positions:
// each coordinate is quantised to 21 bits over the level's bounding box and
// the bits are interleaved; ties keep the index order.  Rows visited in this
// order gather neighbour rows that were gathered a moment before, so a pass
// over a level much larger than the caches fetches each row about once
// instead of several times (the index order puts the coarse vertices first,
// so every row's neighbours are also used half a pass away).
std::vector<int32_t> morton_order(const std::vector<double>& xyz) {
  const int64_t n = int64_t(xyz.size() / 3);
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) lo[d] = hi[d] = n > 0 ? xyz[d] : 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * i + d]);
      hi[d] = std::max(hi[d], xyz[3 * i + d]);
    }
  constexpr int kBits = 21;
  const double top = double((1u << kBits) - 1);
  std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) {
    uint64_t code = 0;
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
      const double w = hi[d] > lo[d] ? (xyz[3 * i + d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
      q[d] = uint32_t(std::min(top, std::max(0.0, std::floor(w * top))));
    }
    for (int b = kBits - 1; b >= 0; --b)
      for (int d = 0; d < 3; ++d) code = (code << 1) | ((q[d] >> b) & 1u);
    key[size_t(i)] = {code, int32_t(i)};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> ord(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) ord[size_t(i)] = key[size_t(i)].second;
  return ord;
}

// The same order over 16-row chunks (the fused Gram kernel's unit), each
// placed at the centroid of its vertices.
std::vector<int32_t> chunk_morton_order(const HostLevel& H) {
  constexpr int64_t kChunk = 16;
  const int64_t nch = (H.n + kChunk - 1) / kChunk;
  std::vector<double> cxyz(static_cast<size_t>(3 * nch), 0.0);
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t r0 = c * kChunk, r1 = std::min(H.n, r0 + kChunk);
    for (int64_t r = r0; r < r1; ++r)
      for (int d = 0; d < 3; ++d) cxyz[size_t(3 * c + d)] += H.xyz[size_t(3 * r + d)];
    for (int d = 0; d < 3; ++d) cxyz[size_t(3 * c + d)] /= double(r1 - r0);
  }
  return morton_order(cxyz);
}

}  // namespace bmg
