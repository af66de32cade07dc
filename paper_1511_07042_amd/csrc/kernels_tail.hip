// The coarse end of the correction V-cycle, resident in LDS.
//
// On the smallest levels a smoothing pass, residual or transfer has only a few
// hundred rows: a kernel launch costs more than the work.  This kernel runs
// the whole V-cycle for levels lo..hi (lo = l_c) inside 1024-thread
// workgroups with every array of those levels in LDS.  The cycle acts on each
// column of the block independently, so the columns are shared out: workgroup
// g takes columns [g m, (g + 1) m) of the m_full-column blocks (m a multiple of
// the 16-byte vector width), which lets a level whose full-width work arrays
// would not fit LDS run here.  Each workgroup holds the shifted operator
// S_l = A_l - sigma M_l (values and 16-bit column indices), the colour lists,
// the parent and restriction tables, the level-0 spectral inverse, and the
// work blocks e, f, t.  The operations and their order are those of the
// multi-block kernels (multicolour Gauss-Seidel or weighted Jacobi, residual,
// restriction P^T, coarse solve, prolongation P; paper Sec. 3, Remark 3.2),
// with workgroup barriers in place of kernel boundaries.  The host packs the
// static part once per solve into one contiguous image; a call copies the
// image and f[hi] into LDS and writes e[hi] back.
#include <mutex>

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

template <typename T>
struct LdsLevel {
  int n, n_prev, W, RW, n_colours;
  const T* S;               // [n][W], S = A - sigma M, slot 0 is the diagonal
  const uint16_t* cols;     // [n][W]
  const uint16_t* crow;     // [n] rows grouped by colour
  const uint16_t* parents;  // [n - n_prev][2]
  const int16_t* rtab;      // [n_prev][RW]
  T *e, *f, *t;
  const int* cptr;          // [n_colours + 1]
};

template <typename T>
__device__ __forceinline__ LdsLevel<T> level(const TailArgs& A, char* lds, int l) {
  const TailLevel& d = A.lv[l];
  LdsLevel<T> L;
  L.n = d.n;
  L.n_prev = d.n_prev;
  L.W = d.W;
  L.RW = d.RW;
  L.n_colours = d.n_colours;
  L.S = reinterpret_cast<const T*>(lds + d.off_S);
  L.cols = reinterpret_cast<const uint16_t*>(lds + d.off_cols);
  L.crow = reinterpret_cast<const uint16_t*>(lds + d.off_crow);
  L.parents = reinterpret_cast<const uint16_t*>(lds + d.off_par);
  L.rtab = reinterpret_cast<const int16_t*>(lds + d.off_rtab);
  L.e = reinterpret_cast<T*>(lds + d.off_e);
  L.f = reinterpret_cast<T*>(lds + d.off_f);
  L.t = reinterpret_cast<T*>(lds + d.off_t);
  L.cptr = d.colour_ptr;
  return L;
}

// (S x)_r for one 16-byte chunk; d = S_rr and xr = x_r on return.
template <typename T>
__device__ __forceinline__ Vec<T> row_apply(const LdsLevel<T>& L, int r, int ch, int m,
                                            const T* x, T& d, Vec<T>& xr) {
  constexpr int VW = Vec<T>::N;
  Vec<T> acc;
  for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
  const int base = r * L.W;
  d = L.S[base];
  for (int k = 0; k < L.W; ++k) {
    const int j = L.cols[base + k];
    const T s = L.S[base + k];
    const Vec<T> xv = ld(x + j * m + ch * VW);
    if (k == 0) xr = xv;
    for (int c = 0; c < VW; ++c) acc.v[c] += s * xv.v[c];
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void swap_et(LdsLevel<T>& L) {
  T* tmp = L.e;
  L.e = L.t;
  L.t = tmp;
}

// One smoothing sweep (GS: colours in the given direction, in place on e;
// Jacobi: e -> t, then the two swap roles).  `zero`: e starts at 0.
template <typename T>
__device__ void sweep(LdsLevel<T>& L, int m, int smoother, T omega, bool forward, bool zero) {
  constexpr int VW = Vec<T>::N;
  const int cpr = m / VW, tid = threadIdx.x, nt = blockDim.x;
  if (smoother == BMG_SMOOTH_JACOBI) {
    for (int idx = tid; idx < L.n * cpr; idx += nt) {
      const int r = idx / cpr, ch = idx - r * cpr;
      const Vec<T> fv = ld(L.f + r * m + ch * VW);
      Vec<T> out;
      if (zero) {
        const T d = L.S[r * L.W];
        for (int c = 0; c < VW; ++c) out.v[c] = omega * fv.v[c] / d;
      } else {
        T d;
        Vec<T> xr;
        const Vec<T> sx = row_apply(L, r, ch, m, L.e, d, xr);
        for (int c = 0; c < VW; ++c) out.v[c] = xr.v[c] + omega * (fv.v[c] - sx.v[c]) / d;
      }
      st(L.t + r * m + ch * VW, out);
    }
    __syncthreads();
    swap_et(L);
    return;
  }
  if (zero) {
    for (int idx = tid; idx < L.n * m; idx += nt) L.e[idx] = T(0);
    __syncthreads();
  }
  for (int k = 0; k < L.n_colours; ++k) {
    const int col = forward ? k : L.n_colours - 1 - k;
    const int b = L.cptr[col], e = L.cptr[col + 1];
    for (int idx = tid; idx < (e - b) * cpr; idx += nt) {
      const int i = idx / cpr, ch = idx - i * cpr;
      const int r = L.crow[b + i];
      T d;
      Vec<T> xr;
      const Vec<T> sx = row_apply(L, r, ch, m, L.e, d, xr);
      const Vec<T> fv = ld(L.f + r * m + ch * VW);
      for (int c = 0; c < VW; ++c) xr.v[c] += (fv.v[c] - sx.v[c]) / d;
      st(L.e + r * m + ch * VW, xr);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_tail(const TailArgs* __restrict__ args) {
  constexpr int VW = Vec<T>::N;
  extern __shared__ char lds[];
  __shared__ TailArgs A;
  const int tid = threadIdx.x, nt = blockDim.x;
  {
    const int nw = int(sizeof(TailArgs) / sizeof(int));
    const int* src = reinterpret_cast<const int*>(args);
    int* dst = reinterpret_cast<int*>(&A);
    for (int i = tid; i < nw; i += nt) dst[i] = src[i];
  }
  __syncthreads();
  const int m = A.m, cpr = m / VW;
  const T omega = T(A.omega);
  // static image and the right-hand side of the top level into LDS
  {
    const int4* src = reinterpret_cast<const int4*>(A.image);
    int4* dst = reinterpret_cast<int4*>(lds);
    for (int i = tid; i < A.image_bytes / 16; i += nt) dst[i] = src[i];
    const LdsLevel<T> H = level<T>(A, lds, A.hi);
    // this workgroup's columns of f (rows of m_full columns) into rows of m
    const int4* fs = reinterpret_cast<const int4*>(A.f_top);
    int4* fd = reinterpret_cast<int4*>(H.f);
    const int c16 = m * int(sizeof(T)) / 16, f16 = A.m_full * int(sizeof(T)) / 16;
    const int nf = H.n * c16;
    for (int i = tid; i < nf; i += nt) {
      const int r = i / c16, c = i - r * c16;
      fd[i] = fs[r * f16 + blockIdx.x * c16 + c];
    }
  }
  __syncthreads();
  // Jacobi buffer roles per level (bit l set: e and t exchanged), uniform
  uint32_t swapped = 0;
  auto lev = [&](int l) {
    LdsLevel<T> L = level<T>(A, lds, l);
    if ((swapped >> l) & 1u) swap_et(L);
    return L;
  };
  auto keep = [&](int l, const LdsLevel<T>& L) {
    if (L.e != level<T>(A, lds, l).e) swapped |= (1u << l);
    else swapped &= ~(1u << l);
  };
  // down: pre-smoothing, residual, restriction
  for (int l = A.hi; l > A.lo; --l) {
    LdsLevel<T> L = lev(l);
    for (int k = 0; k < A.nu1; ++k) sweep(L, m, A.smoother, omega, true, k == 0);
    if (A.nu1 == 0) {
      for (int idx = tid; idx < L.n * m; idx += nt) L.e[idx] = T(0);
      __syncthreads();
    }
    for (int idx = tid; idx < L.n * cpr; idx += nt) {
      const int r = idx / cpr, ch = idx - r * cpr;
      T d;
      Vec<T> xr;
      const Vec<T> sx = row_apply(L, r, ch, m, L.e, d, xr);
      const Vec<T> fv = ld(L.f + r * m + ch * VW);
      Vec<T> o;
      for (int c = 0; c < VW; ++c) o.v[c] = fv.v[c] - sx.v[c];
      st(L.t + r * m + ch * VW, o);
    }
    __syncthreads();
    const LdsLevel<T> C = level<T>(A, lds, l - 1);
    for (int idx = tid; idx < L.n_prev * cpr; idx += nt) {
      const int i = idx / cpr, ch = idx - i * cpr;
      Vec<T> acc = ld(L.t + i * m + ch * VW), h;
      for (int c = 0; c < VW; ++c) h.v[c] = T(0);
      for (int k = 0; k < L.RW; ++k) {
        const int j = L.rtab[i * L.RW + k];
        if (j < 0) break;
        const Vec<T> xv = ld(L.t + j * m + ch * VW);
        for (int c = 0; c < VW; ++c) h.v[c] += xv.v[c];
      }
      for (int c = 0; c < VW; ++c) acc.v[c] += T(0.5) * h.v[c];
      st(C.f + i * m + ch * VW, acc);
    }
    __syncthreads();
    keep(l, L);
  }
  // coarsest level of the cycle
  {
    LdsLevel<T> L = lev(A.lo);
    if (A.lo == 0 && A.off_phi >= 0) {
      // truncated spectral inverse: e = Phi (g o (Phi^T f))
      const int n0 = L.n;
      const T* phi = reinterpret_cast<const T*>(lds + A.off_phi);
      const T* phit = reinterpret_cast<const T*>(lds + A.off_phit);
      const T* g = reinterpret_cast<const T*>(lds + A.off_g);
      for (int idx = tid; idx < n0 * cpr; idx += nt) {
        const int i = idx / cpr, ch = idx - i * cpr;
        Vec<T> acc;
        for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
        for (int k = 0; k < n0; ++k) {
          const T w = phit[i * n0 + k];
          const Vec<T> fv = ld(L.f + k * m + ch * VW);
          for (int c = 0; c < VW; ++c) acc.v[c] += w * fv.v[c];
        }
        st(L.t + i * m + ch * VW, acc);
      }
      __syncthreads();
      for (int idx = tid; idx < n0 * cpr; idx += nt) {
        const int i = idx / cpr, ch = idx - i * cpr;
        Vec<T> acc;
        for (int c = 0; c < VW; ++c) acc.v[c] = T(0);
        for (int k = 0; k < n0; ++k) {
          const T w = phi[i * n0 + k] * g[k];
          const Vec<T> tv = ld(L.t + k * m + ch * VW);
          for (int c = 0; c < VW; ++c) acc.v[c] += w * tv.v[c];
        }
        st(L.e + i * m + ch * VW, acc);
      }
      __syncthreads();
    } else {
      for (int k = 0; k < 8; ++k) sweep(L, m, A.smoother, omega, k % 2 == 0, k == 0);
    }
    keep(A.lo, L);
  }
  // up: prolongation and post-smoothing
  for (int l = A.lo + 1; l <= A.hi; ++l) {
    LdsLevel<T> L = lev(l);
    const T* ec = lev(l - 1).e;
    for (int idx = tid; idx < L.n * cpr; idx += nt) {
      const int i = idx / cpr, ch = idx - i * cpr;
      Vec<T> v;
      if (i < L.n_prev) {
        v = ld(ec + i * m + ch * VW);
      } else {
        const int q = i - L.n_prev;
        const Vec<T> xa = ld(ec + int(L.parents[2 * q]) * m + ch * VW);
        const Vec<T> xb = ld(ec + int(L.parents[2 * q + 1]) * m + ch * VW);
        for (int c = 0; c < VW; ++c) v.v[c] = T(0.5) * (xa.v[c] + xb.v[c]);
      }
      Vec<T> y = ld(L.e + i * m + ch * VW);
      for (int c = 0; c < VW; ++c) y.v[c] += v.v[c];
      st(L.e + i * m + ch * VW, y);
    }
    __syncthreads();
    for (int k = 0; k < A.nu2; ++k) sweep(L, m, A.smoother, omega, false, false);
    keep(l, L);
  }
  // result of the top level back to global memory
  {
    const LdsLevel<T> H = lev(A.hi);
    const int4* src = reinterpret_cast<const int4*>(H.e);
    int4* dst = reinterpret_cast<int4*>(A.e_top);
    const int c16 = m * int(sizeof(T)) / 16, f16 = A.m_full * int(sizeof(T)) / 16;
    const int ne = H.n * c16;
    for (int i = tid; i < ne; i += nt) {
      const int r = i / c16, c = i - r * c16;
      dst[r * f16 + blockIdx.x * c16 + c] = src[i];
    }
  }
}

}  // namespace

template <typename T>
int launch_tail(const TailArgs* dev_args, int lds_bytes, int groups, hipStream_t s) {
  static std::once_flag once;  // solves on several threads may arrive together
  std::call_once(once, [] {
    (void)hipFuncSetAttribute((const void*)k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kTailLdsBudget);
    (void)hipFuncSetAttribute((const void*)k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kTailLdsBudget);
  });
  k_tail<T><<<groups, 1024, lds_bytes, s>>>(dev_args);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("tail kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

template int launch_tail<float>(const TailArgs*, int, int, hipStream_t);
template int launch_tail<double>(const TailArgs*, int, int, hipStream_t);

}  // namespace bmg
