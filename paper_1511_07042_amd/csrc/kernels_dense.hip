// One-workgroup FP64 dense kernels of the Rayleigh-Ritz step.
//
// The enriched pencil (eq. pb-c-aux-mat, Alg. 2 step 4 / Alg. 3 step 5) is
// small (nz = n_c + m <= 96) and lives in LDS.  Its M-block is made orthonormal
// by SVQB (Stathopoulos & Wu, SIAM J. Sci. Comput. 2002: scale to unit
// diagonal, eigendecompose, drop directions whose eigenvalue is below 1e-12 of
// the largest), which is the "orthogonalize with respect to b_h" step of
// Alg. 2 step 3; the reduced standard problem is shifted by sigma and solved
// again by Jacobi; the m eigenpairs nearest sigma are kept (Alg. 2 step 2,
// Remark 4.1).
//
// Jacobi method (Golub & Van Loan, Matrix Computations, Sec. 8.5): two-sided
// rotations in parallel (round-robin) order.  In one round the n/2 disjoint
// pairs (p, q) get their rotations at once; every 2x2 block [p1 q1] x [p2 q2]
// of the matrix is then rotated on both sides by one thread, and each row of
// the eigenvector matrix by one thread.  Sweeps repeat until the off-diagonal
// Frobenius norm is below 1e-15 of the total.
#include <cmath>

#include "bmg_internal.h"

namespace bmg {
namespace {

constexpr int kMaxN = 96;
constexpr int kThreads = 512;

struct JacobiShared {
  double c[kMaxN / 2], s[kMaxN / 2], t[kMaxN / 2];
  int p[kMaxN / 2], q[kMaxN / 2];
  double red[2 * (kThreads / 64)];
  double bcast[2];
};

__device__ void block_sum2(double a, double b, JacobiShared& sh, double& ra, double& rb) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sh.red[2 * w] = a;
    sh.red[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int i = 0; i < int(blockDim.x >> 6); ++i) {
      sa += sh.red[2 * i];
      sb += sh.red[2 * i + 1];
    }
    sh.bcast[0] = sa;
    sh.bcast[1] = sb;
  }
  __syncthreads();
  ra = sh.bcast[0];
  rb = sh.bcast[1];
  __syncthreads();
}

// Diagonalise the symmetric n x n matrix X (row-major, LDS) in place:
// on return X is diagonal (eigenvalues on the diagonal, unsorted) and
// X_in = V diag V^T with V (LDS) orthogonal.  Returns sweeps used (-1 if the
// sweep limit was hit).
__device__ int block_jacobi(double* X, double* V, int n, JacobiShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ne = n + (n & 1);
  const int half = ne / 2;
  for (int e = tid; e < n * n; e += nt) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const double v = X[e] * X[e];
      tot += v;
      if (e / n != e % n) off += v;
    }
    double so, stot;
    block_sum2(off, tot, sh, so, stot);
    if (so <= 1e-30 * stot) return sweep;
    for (int rd = 0; rd < ne - 1; ++rd) {
      if (tid < half) {
        int p = (tid + rd) % (ne - 1);
        int q = tid == 0 ? ne - 1 : (ne - 1 - tid + rd) % (ne - 1);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
          const double apq = X[p * n + q];
          const double app = X[p * n + p], aqq = X[q * n + q];
          if (apq != 0.0 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            if (fabs(tau) > 1e150) {
              t = 0.5 / tau;
            } else {
              t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            }
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        sh.c[tid] = c;
        sh.s[tid] = s;
        sh.t[tid] = t;
        sh.p[tid] = p;
        sh.q[tid] = q;
      }
      __syncthreads();
      // two-sided update of the blocks (t1 <= t2), each written with its transpose
      const int nblk = half * (half + 1) / 2;
      for (int idx = tid; idx < nblk; idx += nt) {
        // unrank idx -> (t1, t2) with t1 <= t2, row-wise over the upper triangle
        int t1 = 0, rem = idx;
        while (rem >= half - t1) {
          rem -= half - t1;
          ++t1;
        }
        const int t2 = t1 + rem;
        const int p1 = sh.p[t1], q1 = sh.q[t1], p2 = sh.p[t2], q2 = sh.q[t2];
        const double c1 = sh.c[t1], s1 = sh.s[t1], c2 = sh.c[t2], s2 = sh.s[t2];
        if (t1 == t2) {
          if (q1 < n && s1 != 0.0) {
            const double apq = X[p1 * n + q1];
            X[p1 * n + p1] -= sh.t[t1] * apq;
            X[q1 * n + q1] += sh.t[t1] * apq;
            X[p1 * n + q1] = 0.0;
            X[q1 * n + p1] = 0.0;
          }
          continue;
        }
        const bool hq1 = q1 < n, hq2 = q2 < n;
        const double bpp = X[p1 * n + p2];
        const double bpq = hq2 ? X[p1 * n + q2] : 0.0;
        const double bqp = hq1 ? X[q1 * n + p2] : 0.0;
        const double bqq = (hq1 && hq2) ? X[q1 * n + q2] : 0.0;
        // left: J1^T B
        const double lpp = c1 * bpp - s1 * bqp, lpq = c1 * bpq - s1 * bqq;
        const double lqp = s1 * bpp + c1 * bqp, lqq = s1 * bpq + c1 * bqq;
        // right: (J1^T B) J2
        const double npp = c2 * lpp - s2 * lpq, npq = s2 * lpp + c2 * lpq;
        const double nqp = c2 * lqp - s2 * lqq, nqq = s2 * lqp + c2 * lqq;
        X[p1 * n + p2] = npp;
        X[p2 * n + p1] = npp;
        if (hq2) {
          X[p1 * n + q2] = npq;
          X[q2 * n + p1] = npq;
        }
        if (hq1) {
          X[q1 * n + p2] = nqp;
          X[p2 * n + q1] = nqp;
        }
        if (hq1 && hq2) {
          X[q1 * n + q2] = nqq;
          X[q2 * n + q1] = nqq;
        }
      }
      for (int idx = tid; idx < n * half; idx += nt) {
        const int k = idx / half, t = idx - (idx / half) * half;
        const int p = sh.p[t], q = sh.q[t];
        if (q >= n || sh.s[t] == 0.0) continue;
        const double c = sh.c[t], s = sh.s[t];
        const double vp = V[k * n + p], vq = V[k * n + q];
        V[k * n + p] = c * vp - s * vq;
        V[k * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  return -1;
}

struct RitzShared {
  JacobiShared j;
  double sv[kMaxN];
  double d[kMaxN];
  int kk[kMaxN];
  int sel[kMaxN];
  int r;
};

// LDS: [RitzShared][X: nz*nz][V: nz*nz]
__global__ void __launch_bounds__(kThreads) k_ritz(int n_c, int m, double sigma,
                                                   const double* __restrict__ G,
                                                   const double* __restrict__ GW, double* Y,
                                                   double* theta, double* scratch, int* status) {
  extern __shared__ double lds[];
  RitzShared& sh = *reinterpret_cast<RitzShared*>(lds);
  const int nz = n_c + m;
  double* X = lds + (sizeof(RitzShared) + 7) / 8;
  double* V = X + nz * nz;
  double* GA = scratch;             // [nz][nz]
  double* GM = GA + nz * nz;        // [nz][nz]
  double* T = GM + nz * nz;         // [nz][nz]
  double* Y1 = T + nz * nz;         // [nz][nz]
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m2 = 2 * m, nc2 = 2 * n_c;
  // assemble the enriched pencil (Galerkin blocks, symmetrised)
  for (int e = tid; e < nz * nz; e += nt) {
    const int i = e / nz, j = e - (e / nz) * nz;
    double va, vm;
    if (i < n_c && j < n_c) {
      va = 0.5 * (GW[i * nc2 + j] + GW[j * nc2 + i]);
      vm = 0.5 * (GW[i * nc2 + n_c + j] + GW[j * nc2 + n_c + i]);
    } else if (i < n_c) {
      va = G[i * m2 + (j - n_c)];
      vm = G[i * m2 + m + (j - n_c)];
    } else if (j < n_c) {
      va = G[j * m2 + (i - n_c)];
      vm = G[j * m2 + m + (i - n_c)];
    } else {
      va = 0.5 * (G[i * m2 + (j - n_c)] + G[j * m2 + (i - n_c)]);
      vm = 0.5 * (G[i * m2 + m + (j - n_c)] + G[j * m2 + m + (i - n_c)]);
    }
    GA[e] = va;
    GM[e] = vm;
    X[e] = vm;
  }
  __syncthreads();
  for (int i = tid; i < nz; i += nt) {
    const double dg = X[i * nz + i];
    sh.sv[i] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < nz * nz; e += nt) {
    const int i = e / nz, j = e - (e / nz) * nz;
    X[e] *= sh.sv[i] * sh.sv[j];
  }
  __syncthreads();
  const int sw1 = block_jacobi(X, V, nz, sh.j);
  if (tid == 0) {
    double dmax = 0.0;
    for (int j = 0; j < nz; ++j) dmax = fmax(dmax, X[j * nz + j]);
    int r = 0;
    for (int j = 0; j < nz; ++j) {
      const double dj = X[j * nz + j];
      if (dj > 1e-12 * dmax) {
        sh.kk[r] = j;
        sh.d[r] = dj;
        ++r;
      }
    }
    sh.r = r;
  }
  __syncthreads();
  const int r = sh.r;
  for (int e = tid; e < nz * r; e += nt) {
    const int i = e / r, q = e - (e / r) * r;
    T[e] = sh.sv[i] * V[i * nz + sh.kk[q]] / sqrt(sh.d[q]);
  }
  __syncthreads();
  for (int e = tid; e < nz * r; e += nt) {
    const int i = e / r, q = e - (e / r) * r;
    double acc = 0.0;
    for (int k = 0; k < nz; ++k) acc += (GA[i * nz + k] - sigma * GM[i * nz + k]) * T[k * r + q];
    Y1[e] = acc;
  }
  __syncthreads();
  // C = T^T Y1 (r x r) into X
  for (int e = tid; e < r * r; e += nt) {
    const int p = e / r, q = e - (e / r) * r;
    double acc = 0.0;
    for (int i = 0; i < nz; ++i) acc += T[i * r + p] * Y1[i * r + q];
    X[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int p = e / r, q = e - (e / r) * r;
    if (p < q) {
      const double avg = 0.5 * (X[p * r + q] + X[q * r + p]);
      X[p * r + q] = avg;
      X[q * r + p] = avg;
    }
  }
  __syncthreads();
  const int sw2 = block_jacobi(X, V, r, sh.j);
  // select the m eigenvalues nearest 0 (ties: by value, then index), ascending
  const int mm = m < r ? m : r;
  for (int j = tid; j < r; j += nt) {
    const double mj = X[j * r + j], aj = fabs(mj);
    int rank = 0;
    for (int i = 0; i < r; ++i) {
      const double mi = X[i * r + i], ai = fabs(mi);
      if (ai < aj || (ai == aj && (mi < mj || (mi == mj && i < j)))) ++rank;
    }
    sh.kk[j] = rank;  // reuse: rank by distance
  }
  __syncthreads();
  for (int j = tid; j < r; j += nt) {
    if (sh.kk[j] >= mm) continue;
    const double mj = X[j * r + j];
    int pos = 0;
    for (int i = 0; i < r; ++i) {
      if (sh.kk[i] >= mm) continue;
      const double mi = X[i * r + i];
      if (mi < mj || (mi == mj && i < j)) ++pos;
    }
    sh.sel[pos] = j;
  }
  __syncthreads();
  for (int e = tid; e < nz * m; e += nt) {
    const int i = e / m, c = e - (e / m) * m;
    double acc = 0.0;
    if (c < mm) {
      const int col = sh.sel[c];
      for (int q = 0; q < r; ++q) acc += T[i * r + q] * V[q * r + col];
    }
    Y[e] = acc;
  }
  for (int c = tid; c < m; c += nt) theta[c] = c < mm ? X[sh.sel[c] * r + sh.sel[c]] + sigma : 0.0;
  if (tid == 0) *status = (r < m) ? 1 : ((sw1 < 0 || sw2 < 0) ? 2 : 0);
}

// Symmetric eigendecomposition of one n x n matrix (n <= 96), ascending.
__global__ void __launch_bounds__(kThreads) k_syev(int n, const double* __restrict__ A, double* w,
                                                   double* Vout, int* status) {
  extern __shared__ double lds[];
  RitzShared& sh = *reinterpret_cast<RitzShared*>(lds);
  double* X = lds + (sizeof(RitzShared) + 7) / 8;
  double* V = X + n * n;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, j = e - (e / n) * n;
    X[e] = 0.5 * (A[i * n + j] + A[j * n + i]);
  }
  __syncthreads();
  const int sw = block_jacobi(X, V, n, sh.j);
  for (int j = tid; j < n; j += nt) {
    const double mj = X[j * n + j];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double mi = X[i * n + i];
      if (mi < mj || (mi == mj && i < j)) ++pos;
    }
    sh.sel[pos] = j;
  }
  __syncthreads();
  for (int c = tid; c < n; c += nt) w[c] = X[sh.sel[c] * n + sh.sel[c]];
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, c = e - (e / n) * n;
    Vout[e] = V[i * n + sh.sel[c]];
  }
  if (tid == 0) *status = sw < 0 ? 2 : 0;
}

size_t lds_bytes(int n) { return ((sizeof(RitzShared) + 7) / 8) * 8 + 2 * size_t(n) * n * sizeof(double); }

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

void set_lds_attr() {
  static bool done = false;
  if (done) return;
  (void)hipFuncSetAttribute((const void*)k_ritz, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_syev, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  done = true;
}

}  // namespace

int ritz_scratch_doubles(int nz) { return 4 * nz * nz; }

int launch_ritz(const RitzArgs& a, hipStream_t s) {
  if (a.nz > kMaxN || a.nz != a.n_c + a.m) {
    set_error("ritz: nz = %d exceeds %d", a.nz, kMaxN);
    return BMG_EINVAL;
  }
  set_lds_attr();
  k_ritz<<<1, kThreads, lds_bytes(a.nz), s>>>(a.n_c, a.m, a.sigma, a.G, a.GW, a.Y, a.theta,
                                              a.scratch, a.status);
  return check_launch();
}

int launch_syev(int n, const double* A, double* w, double* V, int* status, hipStream_t s) {
  if (n < 1 || n > kMaxN) {
    set_error("syev: n = %d outside [1, %d]", n, kMaxN);
    return BMG_EINVAL;
  }
  set_lds_attr();
  k_syev<<<1, kThreads, lds_bytes(n), s>>>(n, A, w, V, status);
  return check_launch();
}

}  // namespace bmg
