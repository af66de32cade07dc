// Row-parallel kernels of the BMG cycle on interleaved vector blocks [n][m].
//
// Thread mapping (all row kernels): a block covers `rpb` whole rows, each row
// split into cpr = m / VW chunks of 16 bytes (VW = 2 doubles or 4 floats), so a
// wavefront reads whole 16-byte chunks of consecutive rows: the gathered
// neighbour rows x[j][*] are contiguous segments and the outputs are fully
// coalesced.  Matrix rows are ELL with the diagonal in slot 0 and padding
// slots that point at the row itself with value 0.  Blocks loop over row
// groups (grid-stride) so grids stay a few thousand blocks at most.
#include <cmath>

#include "bmg_internal.h"

namespace bmg {
namespace {

template <typename T>
struct alignas(16) Vec {
  static constexpr int N = 16 / sizeof(T);
  T v[N];
};

template <typename T>
__device__ __forceinline__ Vec<T> ld(const T* p) {
  return *reinterpret_cast<const Vec<T>*>(p);
}
template <typename T>
__device__ __forceinline__ void st(T* p, const Vec<T>& x) {
  *reinterpret_cast<Vec<T>*>(p) = x;
}

struct Geom {
  int cpr, rpb, block, grid;
};

template <typename T>
Geom row_geom(int64_t n, int m, int max_grid = 8192) {
  Geom g;
  g.cpr = m / Vec<T>::N;
  g.rpb = g.cpr >= 256 ? 1 : 256 / g.cpr;
  g.block = g.rpb * g.cpr;
  int64_t groups = (n + g.rpb - 1) / g.rpb;
  g.grid = int(groups < max_grid ? (groups > 0 ? groups : 1) : max_grid);
  return g;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

// Neighbour gather of one ELL row: acc = sum_k S[base+k] x[cols[base+k]][off..]
// and xr = x[row][off..] (slot 0 is the diagonal).  With WT > 0 the width is a
// compile-time constant: every column index and value is loaded first, then
// every x segment, so a thread has all 2 WT loads of the row in flight at once.
template <typename T, int WT>
__device__ __forceinline__ void row_gather(const int* __restrict__ cols, const T* __restrict__ S,
                                           int64_t base, int W, const T* __restrict__ x, int m,
                                           int off, Vec<T>& acc, Vec<T>& xr) {
  constexpr int VW = Vec<T>::N;
  for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
  if (WT > 0) {
    int j[WT > 0 ? WT : 1];
    T sv[WT > 0 ? WT : 1];
    Vec<T> xv[WT > 0 ? WT : 1];
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      j[k] = cols[base + k];
      sv[k] = S[base + k];
    }
#pragma unroll
    for (int k = 0; k < WT; ++k) xv[k] = ld(x + int64_t(j[k]) * m + off);
#pragma unroll
    for (int k = 0; k < WT; ++k)
      for (int c = 0; c < VW; ++c) acc.v[c] += sv[k] * xv[k].v[c];
    xr = xv[0];
  } else {
    for (int k = 0; k < W; ++k) {
      const int jj = cols[base + k];
      const T s = S[base + k];
      const Vec<T> v = ld(x + int64_t(jj) * m + off);
      if (k == 0) xr = v;
      for (int c = 0; c < VW; ++c) acc.v[c] += s * v.v[c];
    }
  }
}

// ---------------------------------------------------------- shifted ops --
enum { K_SHIFTED = 0, K_RESIDUAL = 1, K_JACOBI = 2, K_JACOBI0 = 3, K_JACOBI_ADD = 4 };

// MODE K_SHIFTED: y = S x; K_RESIDUAL: y = f - S x;
// K_JACOBI: y = x + omega (f - S x) / d; K_JACOBI0: y = omega f / d  (x = 0),
// with S = A - sigma M (precomputed once per solve) and d = S_ii.
// WT: ELL width when it is the built-in 7, else 0 (runtime W).
template <typename T, int MODE, int WT>
__global__ void __launch_bounds__(256) k_rowop(int64_t n, int W, int m, int cpr, int rpb,
                                               const int* __restrict__ cols,
                                               const T* __restrict__ S, T omega,
                                               const T* __restrict__ x,
                                               const T* __restrict__ f, T* __restrict__ y,
                                               double* __restrict__ u) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < n; i += int64_t(gridDim.x) * rpb) {
    const int64_t r = i;
    const int64_t base = r * W;
    Vec<T> acc, xr;
    const T d = S[base];
    if (MODE == K_JACOBI0) {
      const Vec<T> fv = ld(f + r * m + ch * VW);
      for (int c = 0; c < VW; ++c) acc.v[c] = omega * fv.v[c] / d;
    } else {
      Vec<T> fv;
      constexpr bool kF = MODE == K_RESIDUAL || MODE == K_JACOBI || MODE == K_JACOBI_ADD;
      if (kF) fv = ld(f + r * m + ch * VW);
      row_gather<T, WT>(cols, S, base, W, x, m, ch * VW, acc, xr);
      if (kF)
        for (int c = 0; c < VW; ++c) acc.v[c] = fv.v[c] - acc.v[c];
      if (MODE == K_JACOBI || MODE == K_JACOBI_ADD)
        for (int c = 0; c < VW; ++c) acc.v[c] = xr.v[c] + omega * acc.v[c] / d;
    }
    if (MODE == K_JACOBI_ADD) {
      // the sweep's result is the correction: added to the FP64 iterate
      double* ur = u + r * m + ch * VW;
      for (int c = 0; c < VW; ++c) ur[c] += double(acc.v[c]);
    } else {
      st(y + r * m + ch * VW, acc);
    }
  }
}

// Gauss-Seidel update of the rows of one colour, in place:
// x_r <- x_r + (f_r - (S x)_r) / S_rr.  Rows of one colour are never adjacent,
// so the rows of a pass are independent.
template <typename T, int WT>
__global__ void __launch_bounds__(256) k_gs(int64_t cnt, const int* __restrict__ rows, int W, int m,
                                            int cpr, int rpb, const int* __restrict__ cols,
                                            const T* __restrict__ S, T* x, const T* __restrict__ f) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < cnt; i += int64_t(gridDim.x) * rpb) {
    const int64_t r = rows[i];
    const int64_t base = r * W;
    Vec<T> acc, xr;
    const T d = S[base];
    const Vec<T> fv = ld(f + r * m + ch * VW);
    row_gather<T, WT>(cols, S, base, W, x, m, ch * VW, acc, xr);
    for (int c = 0; c < VW; ++c) xr.v[c] += (fv.v[c] - acc.v[c]) / d;
    st(x + r * m + ch * VW, xr);
  }
}

// Kaczmarz projection of the rows of one colour of a distance-2 colouring, in
// place (Sec. 5.3): with t = (f_r - (S x)_r) / sum_k S_rk^2,
// x_j <- x_j + t S_rj for every column j of row r (r included).  Rows of one
// colour share no column, so the rows of a pass read and write disjoint
// entries of x; each thread owns VW columns of the block.  ELL padding
// entries (value 0, column r) add nothing.
template <typename T, int WT>
__global__ void __launch_bounds__(256) k_kaczmarz(int64_t cnt, const int* __restrict__ rows, int W,
                                                  int m, int cpr, int rpb,
                                                  const int* __restrict__ cols,
                                                  const T* __restrict__ S, T* x,
                                                  const T* __restrict__ f) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < cnt; i += int64_t(gridDim.x) * rpb) {
    const int64_t r = rows[i];
    const int64_t base = r * W;
    Vec<T> acc, xr;
    const Vec<T> fv = ld(f + r * m + ch * VW);
    row_gather<T, WT>(cols, S, base, W, x, m, ch * VW, acc, xr);
    T q = T(0);
    const int w = WT > 0 ? WT : W;
    for (int k = 0; k < w; ++k) {
      const T sv = S[base + k];
      q += sv * sv;
    }
    Vec<T> t;
    for (int c = 0; c < VW; ++c) t.v[c] = (fv.v[c] - acc.v[c]) / q;
    for (int k = 0; k < w; ++k) {
      const T sv = S[base + k];
      T* xj = x + int64_t(cols[base + k]) * m + ch * VW;
      Vec<T> v = ld(xj);
      for (int c = 0; c < VW; ++c) v.v[c] += t.v[c] * sv;
      st(xj, v);
    }
  }
}

// The same projections with a shift per column (FP64): column c relaxes
// (A - shifts[c] M) x_c = f_c, the operator formed on the fly from A and M.
// A thread owns two columns of one row (m even).
template <int WT>
__global__ void __launch_bounds__(256) k_kaczmarz_shifts(int64_t cnt, const int* __restrict__ rows,
                                                         int W, int m, const int* __restrict__ cols,
                                                         const double* __restrict__ a,
                                                         const double* __restrict__ mm,
                                                         const double* __restrict__ shifts, double* x,
                                                         const double* __restrict__ f) {
  const int cpr = m >> 1;
  const int rpb = 256 / cpr;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  const double s0 = shifts[2 * ch], s1 = shifts[2 * ch + 1];
  const int w = WT > 0 ? WT : W;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < cnt; i += int64_t(gridDim.x) * rpb) {
    const int64_t r = rows[i];
    const int64_t base = r * W;
    double acc0 = 0, acc1 = 0, q0 = 0, q1 = 0;
    for (int k = 0; k < w; ++k) {
      const double av = a[base + k], mv = mm[base + k];
      const double v0 = av - s0 * mv, v1 = av - s1 * mv;
      const double2 xv = *reinterpret_cast<const double2*>(x + int64_t(cols[base + k]) * m + 2 * ch);
      acc0 += v0 * xv.x;
      acc1 += v1 * xv.y;
      q0 += v0 * v0;
      q1 += v1 * v1;
    }
    const double2 fv = *reinterpret_cast<const double2*>(f + r * m + 2 * ch);
    const double t0 = (fv.x - acc0) / q0, t1 = (fv.y - acc1) / q1;
    for (int k = 0; k < w; ++k) {
      const double av = a[base + k], mv = mm[base + k];
      double2* xj = reinterpret_cast<double2*>(x + int64_t(cols[base + k]) * m + 2 * ch);
      double2 v = *xj;
      v.x += t0 * (av - s0 * mv);
      v.y += t1 * (av - s1 * mv);
      *xj = v;
    }
  }
}

// ---------------------------------------------------- fused cycle kernels --
// Each computes, row by row, what a sequence of the kernels above computes,
// with the same operations in the same order (so the results are identical
// bit for bit), without writing the intermediate block to memory.

// Two weighted-Jacobi sweeps from a zero iterate:
//   y1 = omega f / d;  y = y1 + omega (f - S y1) / d,
// with y1 at the neighbours formed on the fly from f and their diagonals.
template <typename T, int WT>
__global__ void __launch_bounds__(256) k_jacobi2z(int64_t n, int W, int m, int cpr, int rpb,
                                                  const int* __restrict__ cols,
                                                  const T* __restrict__ S, T omega,
                                                  const T* __restrict__ f, T* __restrict__ y) {
  constexpr int VW = Vec<T>::N;
  constexpr int KM = WT > 0 ? WT : 1;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  const int off = ch * VW;
  for (int64_t r = int64_t(blockIdx.x) * rpb + rloc; r < n; r += int64_t(gridDim.x) * rpb) {
    const int64_t base = r * W;
    const T d = S[base];
    const Vec<T> fr = ld(f + r * m + off);
    Vec<T> acc, xr;
    for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
    if (WT > 0) {
      int j[KM];
      T sv[KM], dj[KM];
      Vec<T> fv[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        j[k] = cols[base + k];
        sv[k] = S[base + k];
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        dj[k] = S[int64_t(j[k]) * W];
        fv[k] = ld(f + int64_t(j[k]) * m + off);
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        Vec<T> y1;
        for (int c = 0; c < VW; ++c) y1.v[c] = omega * fv[k].v[c] / dj[k];
        if (k == 0) xr = y1;
        for (int c = 0; c < VW; ++c) acc.v[c] += sv[k] * y1.v[c];
      }
    } else {
      for (int k = 0; k < W; ++k) {
        const int jj = cols[base + k];
        const T sk = S[base + k];
        const T dk = S[int64_t(jj) * W];
        const Vec<T> fk = ld(f + int64_t(jj) * m + off);
        Vec<T> y1;
        for (int c = 0; c < VW; ++c) y1.v[c] = omega * fk.v[c] / dk;
        if (k == 0) xr = y1;
        for (int c = 0; c < VW; ++c) acc.v[c] += sk * y1.v[c];
      }
    }
    for (int c = 0; c < VW; ++c) acc.v[c] = fr.v[c] - acc.v[c];
    for (int c = 0; c < VW; ++c) acc.v[c] = xr.v[c] + omega * acc.v[c] / d;
    st(y + r * m + off, acc);
  }
}

// Residual and restriction: fc[i] = r[i] + 1/2 sum_{children c of i} r[c],
// r = f - S e on the fine rows (P^T of eq. proj-1 applied to the residual).
template <typename T, int WT>
__device__ __forceinline__ Vec<T> residual_row(const int* __restrict__ cols,
                                               const T* __restrict__ S, int64_t r, int W,
                                               const T* __restrict__ e, const T* __restrict__ f,
                                               int m, int off) {
  constexpr int VW = Vec<T>::N;
  const Vec<T> fv = ld(f + r * m + off);
  Vec<T> acc, xr;
  row_gather<T, WT>(cols, S, r * W, W, e, m, off, acc, xr);
  for (int c = 0; c < VW; ++c) acc.v[c] = fv.v[c] - acc.v[c];
  return acc;
}

template <typename T, int WT>
__global__ void __launch_bounds__(256) k_resrestrict(int64_t nc, int W, int RW, int m, int cpr,
                                                     int rpb, const int* __restrict__ cols,
                                                     const T* __restrict__ S,
                                                     const int* __restrict__ rtab,
                                                     const int* __restrict__ rself,
                                                     const T* __restrict__ e,
                                                     const T* __restrict__ f,
                                                     T* __restrict__ fc) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  const int off = ch * VW;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < nc; i += int64_t(gridDim.x) * rpb) {
    const int64_t self = rself != nullptr ? int64_t(rself[i]) : i;
    Vec<T> acc = residual_row<T, WT>(cols, S, self, W, e, f, m, off);
    Vec<T> h;
    for (int c = 0; c < VW; ++c) h.v[c] = T(0);
    for (int k = 0; k < RW; ++k) {
      const int j = rtab[i * RW + k];
      if (j < 0) break;
      const Vec<T> rv = residual_row<T, WT>(cols, S, j, W, e, f, m, off);
      for (int c = 0; c < VW; ++c) h.v[c] += rv.v[c];
    }
    for (int c = 0; c < VW; ++c) acc.v[c] += T(0.5) * h.v[c];
    st(fc + i * m + off, acc);
  }
}

// Prolongation and one Jacobi sweep: with e' = e + P ec (P of eq. proj-1),
// y = e' + omega (f - S e') / d; e' at the neighbours is formed on the fly.
template <typename T>
__device__ __forceinline__ Vec<T> prolonged(const T* __restrict__ e, const T* __restrict__ ec,
                                            const int* __restrict__ parents, int64_t nc, int64_t j,
                                            int m, int off) {
  constexpr int VW = Vec<T>::N;
  Vec<T> v;
  if (j < nc) {
    v = ld(ec + j * m + off);
  } else {
    const int64_t q = j - nc;
    const Vec<T> xa = ld(ec + int64_t(parents[2 * q]) * m + off);
    const Vec<T> xb = ld(ec + int64_t(parents[2 * q + 1]) * m + off);
    for (int c = 0; c < VW; ++c) v.v[c] = T(0.5) * (xa.v[c] + xb.v[c]);
  }
  Vec<T> yv = ld(e + j * m + off);
  for (int c = 0; c < VW; ++c) yv.v[c] += v.v[c];
  return yv;
}

template <typename T, int WT>
__global__ void __launch_bounds__(256) k_prolong_jacobi(int64_t n, int64_t nc, int W, int m,
                                                        int cpr, int rpb,
                                                        const int* __restrict__ cols,
                                                        const T* __restrict__ S,
                                                        const int* __restrict__ parents, T omega,
                                                        const T* __restrict__ e,
                                                        const T* __restrict__ ec,
                                                        const T* __restrict__ f,
                                                        T* __restrict__ y) {
  constexpr int VW = Vec<T>::N;
  constexpr int KM = WT > 0 ? WT : 1;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  const int off = ch * VW;
  for (int64_t r = int64_t(blockIdx.x) * rpb + rloc; r < n; r += int64_t(gridDim.x) * rpb) {
    const int64_t base = r * W;
    const T d = S[base];
    const Vec<T> fr = ld(f + r * m + off);
    Vec<T> acc, xr;
    for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
    if (WT > 0) {
      int j[KM];
      T sv[KM];
      Vec<T> xv[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        j[k] = cols[base + k];
        sv[k] = S[base + k];
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) xv[k] = prolonged<T>(e, ec, parents, nc, j[k], m, off);
#pragma unroll
      for (int k = 0; k < KM; ++k)
        for (int c = 0; c < VW; ++c) acc.v[c] += sv[k] * xv[k].v[c];
      xr = xv[0];
    } else {
      for (int k = 0; k < W; ++k) {
        const int jj = cols[base + k];
        const T sk = S[base + k];
        const Vec<T> v = prolonged<T>(e, ec, parents, nc, jj, m, off);
        if (k == 0) xr = v;
        for (int c = 0; c < VW; ++c) acc.v[c] += sk * v.v[c];
      }
    }
    for (int c = 0; c < VW; ++c) acc.v[c] = fr.v[c] - acc.v[c];
    for (int c = 0; c < VW; ++c) acc.v[c] = xr.v[c] + omega * acc.v[c] / d;
    st(y + r * m + off, acc);
  }
}

// S = A - sigma M, elementwise over the ELL values, in precision T.
template <typename T>
__global__ void k_shift(int64_t cnt, const T* __restrict__ a, const T* __restrict__ mm, T sigma,
                        T* __restrict__ S) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    S[i] = a[i] - sigma * mm[i];
}

// FP64 gather of one ELL row against both matrices: (A x)[row][off, off+1] and
// (M x)[row][off, off+1]; same load order as row_gather.
template <int WT>
__device__ __forceinline__ void row_gather_am(const int* __restrict__ cols,
                                              const double* __restrict__ a,
                                              const double* __restrict__ mm, int64_t base, int W,
                                              const double* __restrict__ x, int m, int off,
                                              double& a0, double& a1, double& m0, double& m1) {
  a0 = a1 = m0 = m1 = 0.0;
  if (WT > 0) {
    int j[WT > 0 ? WT : 1];
    double av[WT > 0 ? WT : 1], mv[WT > 0 ? WT : 1];
    Vec<double> xv[WT > 0 ? WT : 1];
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      j[k] = cols[base + k];
      av[k] = a[base + k];
      mv[k] = mm[base + k];
    }
#pragma unroll
    for (int k = 0; k < WT; ++k) xv[k] = ld(x + int64_t(j[k]) * m + off);
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      a0 += av[k] * xv[k].v[0];
      a1 += av[k] * xv[k].v[1];
      m0 += mv[k] * xv[k].v[0];
      m1 += mv[k] * xv[k].v[1];
    }
  } else {
    for (int k = 0; k < W; ++k) {
      const int jj = cols[base + k];
      const double av = a[base + k], mv = mm[base + k];
      const Vec<double> xv = ld(x + int64_t(jj) * m + off);
      a0 += av * xv.v[0];
      a1 += av * xv.v[1];
      m0 += mv * xv.v[0];
      m1 += mv * xv.v[1];
    }
  }
}

// ------------------------------------------------------- FP64 SpMM (A, M) --
template <int WT>
__global__ void __launch_bounds__(256) k_spmm_am(int64_t n, int W, int m, int cpr, int rpb,
                                                 const int* __restrict__ cols,
                                                 const double* __restrict__ a,
                                                 const double* __restrict__ mm,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ ya, double* __restrict__ ym) {
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  if (rloc >= rpb) return;
  for (int64_t r = int64_t(blockIdx.x) * rpb + rloc; r < n; r += int64_t(gridDim.x) * rpb) {
    double a0, a1, m0, m1;
    row_gather_am<WT>(cols, a, mm, r * W, W, x, m, ch * 2, a0, a1, m0, m1);
    Vec<double> oa, om;
    oa.v[0] = a0;
    oa.v[1] = a1;
    om.v[0] = m0;
    om.v[1] = m1;
    st(ya + r * m + ch * 2, oa);
    st(ym + r * m + ch * 2, om);
  }
}

// Eigen-residual R = A X - (M X) diag(theta), FP64 arithmetic, stored as
// sgn * R in T; per-block partial sums of R^2 / lumped per column.
template <typename T, int WT>
__global__ void __launch_bounds__(256) k_eigres(int64_t n, int W, int m, int cpr, int rpb,
                                                const int* __restrict__ cols,
                                                const double* __restrict__ a,
                                                const double* __restrict__ mm,
                                                const double* __restrict__ dinv,
                                                const double* __restrict__ x,
                                                const double* __restrict__ theta, double sgn,
                                                T* __restrict__ y, double* __restrict__ part) {
  extern __shared__ double sred[];  // [rpb][m]
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  const bool active = rloc < rpb;
  double s0 = 0, s1 = 0;
  if (active) {
    const double t0 = theta[2 * ch], t1 = theta[2 * ch + 1];
    for (int64_t r = int64_t(blockIdx.x) * rpb + rloc; r < n; r += int64_t(gridDim.x) * rpb) {
      double a0, a1, m0, m1;
      row_gather_am<WT>(cols, a, mm, r * W, W, x, m, ch * 2, a0, a1, m0, m1);
      const double r0 = a0 - m0 * t0, r1 = a1 - m1 * t1;
      const double di = dinv[r];
      s0 += r0 * r0 * di;
      s1 += r1 * r1 * di;
      T* yp = y + r * m + ch * 2;
      yp[0] = T(sgn * r0);
      yp[1] = T(sgn * r1);
    }
  }
  if (part) {
    if (active) {
      sred[rloc * m + 2 * ch] = s0;
      sred[rloc * m + 2 * ch + 1] = s1;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
      double s = 0;
      for (int q = 0; q < rpb; ++q) s += sred[q * m + c];
      part[int64_t(c) * gridDim.x + blockIdx.x] = s;  // column-major: [m][blocks]
    }
  }
}

// out[c] = sum_b part[c][b] (partials stored column-major), one 256-thread
// block per column: each thread sums a fixed strided subset, then a fixed
// reduction tree (deterministic).
// With mirror set (a host-mapped buffer laid out like [theta m][rho2 m][8
// status words], src = the device copy of that layout with out = src + m) the
// kernel also writes theta, the sums and the status words there, so the host
// reads a cycle's results without a separate copy.
__global__ void __launch_bounds__(256) k_colsum(const double* __restrict__ part, int nblk, int m,
                                                double* __restrict__ out, const double* src,
                                                double* mirror) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  const double* pc = part + int64_t(c) * nblk;
  double s = 0;
  // eight loads in flight, added in the order b = tid, tid + 256, ...
  constexpr int kU = 8;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 256 * kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = b0 + 256 * u < nblk ? pc[b0 + 256 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (b0 + 256 * u < nblk) s += v[u];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    out[c] = t;
    if (mirror != nullptr) {
      mirror[c] = src[c];
      mirror[m + c] = t;
    }
  }
  if (mirror != nullptr && c == 0 && threadIdx.x < 8) mirror[2 * m + threadIdx.x] = src[2 * m + threadIdx.x];
}

// --------------------------------------------------------------- transfers --
// y[i] = x[i] + 1/2 sum_{children c of i} x[c]   (P^T, eq. proj-1 transposed)
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(int64_t nc, int RW, int m, int cpr, int rpb,
                                                  const int* __restrict__ rtab,
                                                  const int* __restrict__ rself,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < nc; i += int64_t(gridDim.x) * rpb) {
    const int64_t self = rself != nullptr ? int64_t(rself[i]) : i;
    Vec<T> acc = ld(x + self * m + ch * VW);
    Vec<T> h;
    for (int c = 0; c < VW; ++c) h.v[c] = T(0);
    for (int k = 0; k < RW; ++k) {
      const int j = rtab[i * RW + k];
      if (j < 0) break;
      const Vec<T> xv = ld(x + int64_t(j) * m + ch * VW);
      for (int c = 0; c < VW; ++c) h.v[c] += xv.v[c];
    }
    for (int c = 0; c < VW; ++c) acc.v[c] += T(0.5) * h.v[c];
    st(y + i * m + ch * VW, acc);
  }
}

// y[i] += x[i] (i < nc);  y[nc + e] += (x[a_e] + x[b_e]) / 2   (P, eq. proj-1).
// With nc = 0 (general tables) every row takes its two parents, equal for a
// vertex of the coarse level.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(int64_t n, int64_t nc, int m, int cpr, int rpb,
                                                     const int* __restrict__ parents,
                                                     const T* __restrict__ x, T* __restrict__ y) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < n; i += int64_t(gridDim.x) * rpb) {
    Vec<T> v;
    if (i < nc) {
      v = ld(x + i * m + ch * VW);
    } else {
      const int64_t e = i - nc;
      const Vec<T> xa = ld(x + int64_t(parents[2 * e]) * m + ch * VW);
      const Vec<T> xb = ld(x + int64_t(parents[2 * e + 1]) * m + ch * VW);
      for (int c = 0; c < VW; ++c) v.v[c] = T(0.5) * (xa.v[c] + xb.v[c]);
    }
    Vec<T> yv = ld(y + i * m + ch * VW);
    for (int c = 0; c < VW; ++c) yv.v[c] += v.v[c];
    st(y + i * m + ch * VW, yv);
  }
}

// ------------------------------------------------------------ small dense --
// y[i][:] = sum_k mat[i][k] g[k] x[k][:]   (g nullable), mat row-major [nr][nk]
template <typename T>
__global__ void __launch_bounds__(256) k_dense_mm(int nr, int nk, int m, int cpr, int rpb,
                                                  const T* __restrict__ mat,
                                                  const T* __restrict__ g,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  constexpr int VW = Vec<T>::N;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < nr; i += int64_t(gridDim.x) * rpb) {
    Vec<T> acc;
    for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
    for (int k = 0; k < nk; ++k) {
      const T w = mat[i * nk + k] * (g ? g[k] : T(1));
      const Vec<T> xv = ld(x + int64_t(k) * m + ch * VW);
      for (int c = 0; c < VW; ++c) acc.v[c] += w * xv.v[c];
    }
    st(y + i * m + ch * VW, acc);
  }
}

// ----------------------------------------------------------- elementwise --
template <typename T>
__global__ void k_fill(T* y, int64_t cnt, T v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    y[i] = v;
}

template <typename T>
__global__ void k_add_to(double* u, const T* __restrict__ e, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    u[i] += double(e[i]);
}

template <typename T>
__global__ void k_convert(const double* __restrict__ x, T* __restrict__ y, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    y[i] = T(x[i]);
}

// SplitMix64 output for state x (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Element (i, j), counter c = i m + j: u1, u2 in (0, 1] from counters 2c and
// 2c + 1; z = sqrt(-2 ln u1) cos(2 pi u2)  (Box-Muller).
__global__ void k_gaussian(double* y, int64_t cnt, int m, uint64_t seed, const int* __restrict__ perm) {
  const double two53 = 1.0 / 9007199254740992.0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cnt;
       c += int64_t(gridDim.x) * blockDim.x) {
    // the counter is the element's place in vertex order (storage row r holds
    // vertex perm[r])
    const int64_t r = c / m;
    const uint64_t cc = perm != nullptr ? uint64_t(int64_t(perm[r]) * m + (c - r * m)) : uint64_t(c);
    const double u1 = (double(splitmix64(seed ^ (2 * cc)) >> 11) + 1.0) * two53;
    const double u2 = (double(splitmix64(seed ^ (2 * cc + 1)) >> 11) + 1.0) * two53;
    y[c] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  }
}

// ---------------------------------------------------------------- output --
// Per block and selected column j: (max |U[i][sel_j]|, lowest vertex i
// attaining it); vertex i is storage row iperm[i] (iperm null: row i).
__global__ void k_argmax(int64_t n, const double* __restrict__ U, int m,
                         const int* __restrict__ sel, int k, const int* __restrict__ iperm, double* pv,
                         int* pi) {
  __shared__ double sv[256];
  __shared__ int si[256];
  for (int j = 0; j < k; ++j) {
    const int col = sel[j];
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
      const int64_t r = iperm != nullptr ? int64_t(iperm[i]) : i;
      const double v = fabs(U[r * m + col]);
      if (v > best) {
        best = v;
        bi = int(i);
      }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        const double v2 = sv[threadIdx.x + off];
        const int i2 = si[threadIdx.x + off];
        if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
          sv[threadIdx.x] = v2;
          si[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      pv[int64_t(blockIdx.x) * k + j] = sv[0];
      pi[int64_t(blockIdx.x) * k + j] = si[0];
    }
    __syncthreads();
  }
}

__global__ void k_sign_final(const double* __restrict__ U, int m, const int* __restrict__ sel, int k,
                             const int* __restrict__ iperm, const double* __restrict__ pv,
                             const int* __restrict__ pi, int nblk, double* sign_out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int b = 0; b < nblk; ++b) {
    const double v = pv[int64_t(b) * k + j];
    const int i = pi[int64_t(b) * k + j];
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  }
  const int64_t r = iperm != nullptr ? int64_t(iperm[bi]) : int64_t(bi);
  sign_out[j] = (U[r * m + sel[j]] < 0) ? -1.0 : 1.0;
}

// out[j][i] = sign_j U[iperm[i]][sel_j]: column-major, vertex order.
__global__ void k_write_evecs(int64_t n, const double* __restrict__ U, int m,
                              const int* __restrict__ sel, const double* __restrict__ sign, int k,
                              const int* __restrict__ iperm, double* out, int64_t ld) {
  const int64_t total = n * k;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(t / n);
    const int64_t i = t - int64_t(j) * n;
    const int64_t r = iperm != nullptr ? int64_t(iperm[i]) : i;
    out[int64_t(j) * ld + i] = sign[j] * U[r * m + sel[j]];
  }
}

// Row permutation of an [n][m] block: y[r] = x[map[r]] (vector loads of 16 bytes).
template <typename T>
__global__ void k_permute_rows(int64_t n, int m, const int* __restrict__ map, const T* __restrict__ x,
                               T* __restrict__ y) {
  const int64_t total = n * m;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = t / m;
    y[t] = x[int64_t(map[r]) * m + (t - r * m)];
  }
}

int grid1d(int64_t cnt) {
  int64_t g = (cnt + 255) / 256;
  return int(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

template <typename T>
const T* aval(const DevLevel& L);
template <>
const double* aval<double>(const DevLevel& L) { return L.a64; }
template <>
const float* aval<float>(const DevLevel& L) { return L.a32; }
template <typename T>
const T* mval(const DevLevel& L);
template <>
const double* mval<double>(const DevLevel& L) { return L.m64; }
template <>
const float* mval<float>(const DevLevel& L) { return L.m32; }

}  // namespace

template <typename T>
int launch_shift(const DevLevel& L, double sigma, T* S, hipStream_t s) {
  const int64_t cnt = L.n * L.W;
  k_shift<T><<<grid1d(cnt), 256, 0, s>>>(cnt, aval<T>(L), mval<T>(L), T(sigma), S);
  return check_launch();
}

// Launch `kern<..., 7>` for the built-in ELL width 7, `kern<..., 0>` otherwise.
#define BMG_BY_WIDTH(W, KT7, KT0, grid, block, shm, s, ...)   \
  do {                                                        \
    if ((W) == 7)                                             \
      BMG_LAUNCH(KT7, grid, block, shm, s, __VA_ARGS__);      \
    else                                                      \
      BMG_LAUNCH(KT0, grid, block, shm, s, __VA_ARGS__);      \
  } while (0)

template <typename T>
int launch_shifted(const DevLevel& L, const T* S, int mode, const T* x, const T* f, T* y, int m,
                   hipStream_t s) {
  Geom g = row_geom<T>(L.n, m);
  if (mode == ROW_SHIFTED)
    BMG_BY_WIDTH(L.W, (k_rowop<T, K_SHIFTED, 7>), (k_rowop<T, K_SHIFTED, 0>), g.grid, g.block, 0, s,
                 L.n, L.W, m, g.cpr, g.rpb, L.cols, S, T(0), x, f, y, nullptr);
  else
    BMG_BY_WIDTH(L.W, (k_rowop<T, K_RESIDUAL, 7>), (k_rowop<T, K_RESIDUAL, 0>), g.grid, g.block, 0, s,
                 L.n, L.W, m, g.cpr, g.rpb, L.cols, S, T(0), x, f, y, nullptr);
  return check_launch();
}

template <typename T>
int launch_jacobi(const DevLevel& L, const T* S, double omega, const T* x, const T* f, T* y,
                  bool x_is_zero, int m, hipStream_t s, double* u_add) {
  Geom g = row_geom<T>(L.n, m);
  if (x_is_zero)
    BMG_LAUNCH((k_rowop<T, K_JACOBI0, 0>), g.grid, g.block, 0, s, L.n, L.W, m, g.cpr, g.rpb, L.cols,
               S, T(omega), x, f, y, nullptr);
  else if (u_add != nullptr)
    BMG_BY_WIDTH(L.W, (k_rowop<T, K_JACOBI_ADD, 7>), (k_rowop<T, K_JACOBI_ADD, 0>), g.grid, g.block, 0,
                 s, L.n, L.W, m, g.cpr, g.rpb, L.cols, S, T(omega), x, f, y, u_add);
  else
    BMG_BY_WIDTH(L.W, (k_rowop<T, K_JACOBI, 7>), (k_rowop<T, K_JACOBI, 0>), g.grid, g.block, 0, s,
                 L.n, L.W, m, g.cpr, g.rpb, L.cols, S, T(omega), x, f, y, nullptr);
  return check_launch();
}

template <typename T>
int launch_gs_colour(const DevLevel& L, const T* S, int colour, T* x, const T* f, int m,
                     hipStream_t s) {
  const int64_t b = L.colour_ptr[colour], e = L.colour_ptr[colour + 1];
  if (e <= b) return BMG_OK;
  Geom g = row_geom<T>(e - b, m);
  BMG_BY_WIDTH(L.W, (k_gs<T, 7>), (k_gs<T, 0>), g.grid, g.block, 0, s, e - b, L.colour_rows + b,
               L.W, m, g.cpr, g.rpb, L.cols, S, x, f);
  return check_launch();
}

template <typename T>
int launch_kaczmarz_colour(const DevLevel& L, const T* S, int colour, T* x, const T* f, int m,
                           hipStream_t s) {
  if (colour < 0 || colour >= L.n_colours2) {
    set_error("Kaczmarz colour %d out of range [0, %d)", colour, L.n_colours2);
    return BMG_EINVAL;
  }
  const int64_t b = L.colour2_ptr[colour], e = L.colour2_ptr[colour + 1];
  if (e <= b) return BMG_OK;
  Geom g = row_geom<T>(e - b, m);
  BMG_BY_WIDTH(L.W, (k_kaczmarz<T, 7>), (k_kaczmarz<T, 0>), g.grid, g.block, 0, s, e - b,
               L.colour2_rows + b, L.W, m, g.cpr, g.rpb, L.cols, S, x, f);
  return check_launch();
}

int launch_kaczmarz_shifts_colour(const DevLevel& L, int colour, const double* shifts, double* x,
                                  const double* f, int m, hipStream_t s) {
  if (colour < 0 || colour >= L.n_colours2 || m < 2 || m % 2 != 0 || m > 512) {
    set_error("Kaczmarz (per-column shifts): colour %d of %d, m = %d (even, at most 512)", colour,
              L.n_colours2, m);
    return BMG_EINVAL;
  }
  const int64_t b = L.colour2_ptr[colour], e = L.colour2_ptr[colour + 1];
  if (e <= b) return BMG_OK;
  const int rpb = 256 / (m / 2);
  const int grid = int(std::min<int64_t>((e - b + rpb - 1) / rpb, 8192));
  BMG_BY_WIDTH(L.W, k_kaczmarz_shifts<7>, k_kaczmarz_shifts<0>, grid, 256, 0, s, e - b,
               L.colour2_rows + b, L.W, m, L.cols, L.a64, L.m64, shifts, x, f);
  return check_launch();
}

template <typename T>
int launch_jacobi2z(const DevLevel& L, const T* S, double omega, const T* f, T* y, int m,
                    hipStream_t s) {
  Geom g = row_geom<T>(L.n, m);
  BMG_BY_WIDTH(L.W, (k_jacobi2z<T, 7>), (k_jacobi2z<T, 0>), g.grid, g.block, 0, s, L.n, L.W, m,
               g.cpr, g.rpb, L.cols, S, T(omega), f, y);
  return check_launch();
}

template <typename T>
int launch_resrestrict(const DevLevel& fine, const T* S, const T* e, const T* f, T* fc, int m,
                       hipStream_t s) {
  Geom g = row_geom<T>(fine.n_prev, m);
  BMG_BY_WIDTH(fine.W, (k_resrestrict<T, 7>), (k_resrestrict<T, 0>), g.grid, g.block, 0, s,
               fine.n_prev, fine.W, fine.RW, m, g.cpr, g.rpb, fine.cols, S, fine.rtab, fine.rself, e, f, fc);
  return check_launch();
}

template <typename T>
int launch_prolong_jacobi(const DevLevel& fine, const T* S, double omega, const T* e, const T* ec,
                          const T* f, T* y, int m, hipStream_t s) {
  Geom g = row_geom<T>(fine.n, m);
  BMG_BY_WIDTH(fine.W, (k_prolong_jacobi<T, 7>), (k_prolong_jacobi<T, 0>), g.grid, g.block, 0, s,
               fine.n, fine.par_nc, fine.W, m, g.cpr, g.rpb, fine.cols, S, fine.parents, T(omega),
               e, ec, f, y);
  return check_launch();
}

int launch_spmm_am(const DevLevel& L, const double* x, double* ya, double* ym, int m,
                   hipStream_t s) {
  Geom g = row_geom<double>(L.n, m);
  BMG_BY_WIDTH(L.W, (k_spmm_am<7>), (k_spmm_am<0>), g.grid, g.block, 0, s, L.n, L.W, m, g.cpr,
               g.rpb, L.cols, L.a64, L.m64, x, ya, ym);
  return check_launch();
}

int eigres_blocks(const DevLevel& L, int m) { return row_geom<double>(L.n, m, 4096).grid; }

template <typename T>
int launch_eigres(const DevLevel& L, const double* x, const double* theta, double sgn, T* y,
                  double* rho2_part, int nblk, int m, hipStream_t s) {
  Geom g = row_geom<double>(L.n, m, 4096);
  if (nblk != g.grid) {
    set_error("eigres grid mismatch");
    return BMG_EINVAL;
  }
  const size_t shm = size_t(g.rpb) * m * sizeof(double);
  BMG_BY_WIDTH(L.W, (k_eigres<T, 7>), (k_eigres<T, 0>), g.grid, g.block, shm, s, L.n, L.W, m, g.cpr,
               g.rpb, L.cols, L.a64, L.m64, L.dinv, x, theta, sgn, y, rho2_part);
  return check_launch();
}

int launch_colsum(const double* part, int nblk, int m, double* out, hipStream_t s, const double* src,
                  double* mirror) {
  k_colsum<<<m, 256, 0, s>>>(part, nblk, m, out, src, mirror);
  return check_launch();
}

template <typename T>
int launch_restrict(const DevLevel& fine, const T* x, T* y, int m, hipStream_t s) {
  Geom g = row_geom<T>(fine.n_prev, m);
  BMG_LAUNCH((k_restrict<T>), g.grid, g.block, 0, s, fine.n_prev, fine.RW, m, g.cpr, g.rpb, fine.rtab, fine.rself,
             x, y);
  return check_launch();
}

template <typename T>
int launch_prolong_add(const DevLevel& fine, const T* x, T* y, int m, hipStream_t s) {
  Geom g = row_geom<T>(fine.n, m);
  BMG_LAUNCH((k_prolong_add<T>), g.grid, g.block, 0, s, fine.n, fine.par_nc, m, g.cpr, g.rpb, fine.parents, x, y);
  return check_launch();
}

template <typename T>
int launch_dense_apply(int n, const T* mat, const T* g, const T* x, T* y, int m, hipStream_t s) {
  Geom gm = row_geom<T>(n, m);
  k_dense_mm<T><<<gm.grid, gm.block, 0, s>>>(n, n, m, gm.cpr, gm.rpb, mat, g, x, y);
  return check_launch();
}

template <typename T>
int launch_fill(T* y, int64_t count, T value, hipStream_t s) {
  k_fill<T><<<grid1d(count), 256, 0, s>>>(y, count, value);
  return check_launch();
}

template <typename T>
int launch_add_to(double* u, const T* e, int64_t count, hipStream_t s) {
  k_add_to<T><<<grid1d(count), 256, 0, s>>>(u, e, count);
  return check_launch();
}

template <typename T>
int launch_convert(const double* x, T* y, int64_t count, hipStream_t s) {
  k_convert<T><<<grid1d(count), 256, 0, s>>>(x, y, count);
  return check_launch();
}

int launch_gaussian(double* y, int64_t n, int m, uint64_t seed, hipStream_t s, const int* perm) {
  k_gaussian<<<grid1d(n * m), 256, 0, s>>>(y, n * m, m, seed, perm);
  return check_launch();
}

int launch_signs(int64_t n, const double* U, int m, const int* sel, int k, const int* iperm, double* sign_out,
                 double* part_val, int* part_idx, int nblk, hipStream_t s) {
  k_argmax<<<nblk, 256, 0, s>>>(n, U, m, sel, k, iperm, part_val, part_idx);
  k_sign_final<<<(k + 63) / 64, 64, 0, s>>>(U, m, sel, k, iperm, part_val, part_idx, nblk, sign_out);
  return check_launch();
}

int launch_write_evecs(int64_t n, const double* U, int m, const int* sel, const double* sign,
                       int k, const int* iperm, double* out, int64_t ld, hipStream_t s) {
  k_write_evecs<<<grid1d(n * k), 256, 0, s>>>(n, U, m, sel, sign, k, iperm, out, ld);
  return check_launch();
}

template <typename T>
int launch_permute_rows(int64_t n, int m, const int* map, const T* x, T* y, hipStream_t s) {
  k_permute_rows<T><<<grid1d(n * m), 256, 0, s>>>(n, m, map, x, y);
  return check_launch();
}
template int launch_permute_rows<double>(int64_t, int, const int*, const double*, double*, hipStream_t);
template int launch_permute_rows<float>(int64_t, int, const int*, const float*, float*, hipStream_t);

#define BMG_INST(T)                                                                              \
  template int launch_shift<T>(const DevLevel&, double, T*, hipStream_t);                        \
  template int launch_shifted<T>(const DevLevel&, const T*, int, const T*, const T*, T*, int,   \
                                 hipStream_t);                                                   \
  template int launch_jacobi<T>(const DevLevel&, const T*, double, const T*, const T*, T*, bool, \
                                int, hipStream_t, double*);                                               \
  template int launch_gs_colour<T>(const DevLevel&, const T*, int, T*, const T*, int, hipStream_t); \
  template int launch_kaczmarz_colour<T>(const DevLevel&, const T*, int, T*, const T*, int,      \
                                         hipStream_t);                                           \
  template int launch_eigres<T>(const DevLevel&, const double*, const double*, double, T*,       \
                                double*, int, int, hipStream_t);                                 \
  template int launch_restrict<T>(const DevLevel&, const T*, T*, int, hipStream_t);              \
  template int launch_prolong_add<T>(const DevLevel&, const T*, T*, int, hipStream_t);           \
  template int launch_dense_apply<T>(int, const T*, const T*, const T*, T*, int, hipStream_t);   \
  template int launch_fill<T>(T*, int64_t, T, hipStream_t);                                      \
  template int launch_add_to<T>(double*, const T*, int64_t, hipStream_t);                        \
  template int launch_convert<T>(const double*, T*, int64_t, hipStream_t);                       \
  template int launch_jacobi2z<T>(const DevLevel&, const T*, double, const T*, T*, int,          \
                                  hipStream_t);                                                   \
  template int launch_resrestrict<T>(const DevLevel&, const T*, const T*, const T*, T*, int,     \
                                     hipStream_t);                                                \
  template int launch_prolong_jacobi<T>(const DevLevel&, const T*, double, const T*, const T*,   \
                                        const T*, T*, int, hipStream_t);
BMG_INST(double)
BMG_INST(float)
#undef BMG_INST

}  // namespace bmg
