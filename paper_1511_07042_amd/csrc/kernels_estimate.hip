// A posteriori error estimator eta_T of eq. est-res (Sec. 5), one thread per
// triangle, all requested eigenpairs in a loop.  Per triangle T with
// vertices x_0..x_2 (outward unit normal n, area |T|, longest edge h_T):
//   residual  h_T^2 lambda^2 |T| / 12 (sum u_i^2 + (sum u_i)^2)
//   jumps     1/2 sum_e |e|^2 (grad u_T . mu_T,e + grad u_T' . mu_T',e)^2
//   geometry  (unit sphere only) |T|/3 sum over edge midpoints q of
//             |(c - 1) g + ((t . g) / c) t|^2,  nu = q / |q|, c = nu . n,
//             t = nu - c n, g = grad u_T
// with mu_T,e the unit conormal of edge e in the plane of T pointing away
// from T and T' the neighbour across e.  The conormal derivatives are
// precomputed per triangle as weights on the vertex values, so the pair loop
// only gathers values.  Per-block sums per pair and term are added in a fixed
// order afterwards.
#include "bmg_internal.h"

namespace bmg {

namespace {

constexpr int kEstBlock = 256;
constexpr int kEstMaxBlocks = 2048;

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 ldv(const double* p) { return V3{p[0], p[1], p[2]}; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 add(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 scl(V3 a, double s) { return V3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Geometry of triangle t: vertices, outward normal, area, gradients of the
// three barycentric functions.
struct TriGeom {
  V3 X[3], n, grad[3];
  double area;
};
__device__ TriGeom tri_geom(const int32_t* tri, const double* xyz, int64_t t) {
  TriGeom G;
  for (int i = 0; i < 3; ++i) G.X[i] = ldv(xyz + 3 * int64_t(tri[3 * t + i]));
  const V3 cr = cross(sub(G.X[1], G.X[0]), sub(G.X[2], G.X[0]));
  const double a2 = sqrt(dot(cr, cr));
  G.area = 0.5 * a2;
  G.n = scl(cr, 1.0 / a2);
  const V3 cen = scl(add(add(G.X[0], G.X[1]), G.X[2]), 1.0 / 3.0);
  if (dot(G.n, cen) < 0) G.n = scl(G.n, -1.0);
  for (int i = 0; i < 3; ++i) {
    const V3 e = sub(G.X[(i + 2) % 3], G.X[(i + 1) % 3]);
    V3 g = scl(cross(G.n, e), 1.0 / a2);
    if (dot(g, sub(G.X[i], G.X[(i + 1) % 3])) < 0) g = scl(g, -1.0);  // towards vertex i
    G.grad[i] = g;
  }
  return G;
}

// unit conormal of edge i (opposite vertex i), in the plane, away from T
__device__ V3 conormal(const TriGeom& G, int i) {
  const V3 a = G.X[(i + 1) % 3], b = G.X[(i + 2) % 3], c = G.X[i];
  const V3 e = sub(b, a);
  const V3 tau = scl(e, 1.0 / sqrt(dot(e, e)));
  V3 v = sub(scl(add(a, b), 0.5), c);
  v = sub(v, scl(tau, dot(v, tau)));
  return scl(v, 1.0 / sqrt(dot(v, v)));
}

__global__ void __launch_bounds__(kEstBlock) k_estimate(int64_t F, int k, const int32_t* __restrict__ tri,
                                                       const int32_t* __restrict__ nbr,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ U, int64_t ld,
                                                       const double* __restrict__ lam, int sphere,
                                                       double* __restrict__ eta2_T,
                                                       double* __restrict__ part) {
  __shared__ double red[kEstBlock / 64][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a block's triangles: a contiguous range, grid-stride over ranges
  for (int64_t base = int64_t(blockIdx.x) * kEstBlock; base < F; base += int64_t(gridDim.x) * kEstBlock) {
    const int64_t t = base + threadIdx.x;
    const bool live = t < F;
    int vi[3] = {0, 0, 0}, vn[3] = {0, 0, 0};
    double wown[3][3], wnb[3], el2[3];
    double h2a12 = 0, area = 0;
    V3 grad[3];
    double qa[3], qb[3];
    V3 qt[3];
    for (int i = 0; i < 3; ++i) {
      qa[i] = qb[i] = 0;
      qt[i] = V3{0, 0, 0};
      wnb[i] = el2[i] = 0;
      grad[i] = V3{0, 0, 0};
      for (int j = 0; j < 3; ++j) wown[i][j] = 0;
    }
    if (live) {
      const TriGeom G = tri_geom(tri, xyz, t);
      area = G.area;
      double hmax2 = 0;
      for (int i = 0; i < 3; ++i) {
        vi[i] = tri[3 * t + i];
        grad[i] = G.grad[i];
        const V3 e = sub(G.X[(i + 2) % 3], G.X[(i + 1) % 3]);
        el2[i] = dot(e, e);
        hmax2 = fmax(hmax2, el2[i]);
      }
      h2a12 = hmax2 * G.area / 12.0;
      for (int e = 0; e < 3; ++e) {
        const V3 mu = conormal(G, e);
        for (int i = 0; i < 3; ++i) wown[e][i] = dot(G.grad[i], mu);
        // the neighbour across edge e: its conormal derivative weights on its
        // own vertex opposite the shared edge (the shared vertices' weights
        // are folded into the own weights below)
        const int32_t pk = nbr[3 * t + e];
        const int64_t tn = pk >> 2;
        const int en = pk & 3;
        const TriGeom H = tri_geom(tri, xyz, tn);
        const V3 mun = conormal(H, en);
        vn[e] = tri[3 * tn + en];
        wnb[e] = dot(H.grad[en], mun);
        for (int i = 0; i < 3; ++i) {
          const int vj = tri[3 * tn + i];
          if (i == en) continue;
          const double w = dot(H.grad[i], mun);
          for (int m = 0; m < 3; ++m)
            if (vi[m] == vj) wown[e][m] += w;
        }
      }
      if (sphere) {
        for (int q = 0; q < 3; ++q) {
          const V3 x = scl(add(G.X[(q + 1) % 3], G.X[(q + 2) % 3]), 0.5);
          const V3 nu = scl(x, 1.0 / sqrt(dot(x, x)));
          const double c = dot(nu, G.n);
          const V3 tt = sub(nu, scl(G.n, c));
          qa[q] = (c - 1.0) * (c - 1.0);
          qb[q] = 2.0 * (c - 1.0) / c + dot(tt, tt) / (c * c);
          qt[q] = tt;
        }
      }
    }
    double tot = 0;
    for (int j = 0; j < k; ++j) {
      double r = 0, jp = 0, gm = 0;
      if (live) {
        const double* u = U + int64_t(j) * ld;
        const double u0 = u[vi[0]], u1 = u[vi[1]], u2 = u[vi[2]];
        const double l = lam[j];
        const double s = u0 + u1 + u2;
        r = h2a12 * l * l * (u0 * u0 + u1 * u1 + u2 * u2 + s * s);
        for (int e = 0; e < 3; ++e) {
          const double jump = wown[e][0] * u0 + wown[e][1] * u1 + wown[e][2] * u2 + wnb[e] * u[vn[e]];
          jp += 0.5 * el2[e] * jump * jump;
        }
        if (sphere) {
          const V3 g = add(add(scl(grad[0], u0), scl(grad[1], u1)), scl(grad[2], u2));
          const double g2 = dot(g, g);
          for (int q = 0; q < 3; ++q) {
            const double tg = dot(qt[q], g);
            gm += qa[q] * g2 + qb[q] * tg * tg;
          }
          gm *= area / 3.0;
        }
      }
      tot += r + jp + gm;
      // block sums of the three terms, wavefront first, in a fixed order
      double v[3] = {r, jp, gm};
      for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
      if (lane == 0)
        for (int c = 0; c < 3; ++c) red[wave][c] = v[c];
      __syncthreads();
      if (threadIdx.x < 3) {
        double acc = 0;
        for (int w = 0; w < kEstBlock / 64; ++w) acc += red[w][threadIdx.x];
        double* p = part + (int64_t(blockIdx.x) * k + j) * 3 + threadIdx.x;
        *p = (base == int64_t(blockIdx.x) * kEstBlock ? 0.0 : *p) + acc;
      }
      __syncthreads();
    }
    if (live && eta2_T) eta2_T[t] = tot;
  }
}

// out[c][j] = sum_b part[b][j][c], blocks in order
__global__ void __launch_bounds__(256) k_estimate_reduce(int nblk, int k, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  for (int e = threadIdx.x; e < 3 * k; e += blockDim.x) {
    const int j = e / 3, c = e % 3;
    double acc = 0;
    for (int b = 0; b < nblk; ++b) acc += part[(int64_t(b) * k + j) * 3 + c];
    out[c * k + j] = acc;
  }
}

}  // namespace

int est_blocks(int64_t F) {
  return int(std::max<int64_t>(1, std::min<int64_t>((F + kEstBlock - 1) / kEstBlock, kEstMaxBlocks)));
}

int launch_estimate(const EstLevel& E, int k, const double* U, int64_t ld, const double* lam, int sphere,
                    double* eta2_T, double* part, double* out, hipStream_t s) {
  const int nblk = est_blocks(E.F);
  k_estimate<<<nblk, kEstBlock, 0, s>>>(E.F, k, E.tri, E.nbr, E.xyz, U, ld, lam, sphere, eta2_T, part);
  k_estimate_reduce<<<1, 256, 0, s>>>(nblk, k, part, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("estimator launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

}  // namespace bmg
