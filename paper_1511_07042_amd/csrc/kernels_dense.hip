// One-workgroup FP64 dense kernels of the Rayleigh-Ritz step.
//
// The enriched pencil (eq. pb-c-aux-mat, Alg. 2 step 4 / Alg. 3 step 5) is
// small (nz = n_c + m <= 96) and lives in LDS.  Its basis is ordered
// [U', W_c] and made M-orthonormal (the "orthogonalize with respect to b_h"
// step of Alg. 2 step 3) by a Cholesky factorisation of the unit-diagonal
// scaled M-Gram matrix; because U' is close to the previous, already
// M-orthonormal and A-diagonal Ritz block, the reduced matrix
// C = L^-1 S (G_A - sigma G_M) S L^-T is then close to diagonal in its leading
// m x m block and Jacobi needs few sweeps.  When a Cholesky pivot falls below
// 1e-10 (the basis is numerically rank deficient) the kernel switches to SVQB
// (Stathopoulos & Wu, SIAM J. Sci. Comput. 2002: eigendecompose the scaled
// Gram matrix, drop directions below 1e-12 of the largest eigenvalue).  The m
// eigenpairs nearest sigma are kept (Alg. 2 step 2, Remark 4.1).
//
// Jacobi method (Golub & Van Loan, Matrix Computations, Sec. 8.5): two-sided
// rotations in parallel (round-robin) order.  In one round the n/2 disjoint
// pairs (p, q) get their rotations at once; every 2x2 block [p1 q1] x [p2 q2]
// of the matrix is rotated on both sides by one thread and each row of the
// eigenvector matrix by one thread.  Only significant rotations are applied,
// |a_pq| > 1e-15 max(sqrt|a_pp a_qq|, ||A||_F / n), so rounding noise is not
// churned; sweeps stop after a sweep without one.
#include <cmath>

#include "bmg_internal.h"

namespace bmg {
namespace {

constexpr int kMaxN = 96;
constexpr int kThreads = 1024;

struct JacobiShared {
  double c[kMaxN / 2], s[kMaxN / 2], t[kMaxN / 2];
  int p[kMaxN / 2], q[kMaxN / 2];
  unsigned char pq[kMaxN - 1][kMaxN];  // round-robin pairs: round r, slot t -> (p, q) at [r][2t], [r][2t+1]
  int rflag;
  double red[2 * (kThreads / 64)];
  double bcast[2];
  int sig[2];
  int flag;
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
// X_in = V diag V^T with V (LDS) orthogonal.  Returns the sweeps used, or -1
// if the sweep limit was hit.
__device__ int block_jacobi(double* X, double* V, int n, JacobiShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ne = n + (n & 1);
  const int half = ne / 2;
  double f2 = 0.0;
  for (int e = tid; e < n * n; e += nt) {
    V[e] = (e / n == e % n) ? 1.0 : 0.0;
    f2 += X[e] * X[e];
  }
  if (tid == 0) {
    sh.sig[0] = 0;
    sh.sig[1] = 0;
  }
  double fro2, dummy;
  block_sum2(f2, 0.0, sh, fro2, dummy);
  const double floor_abs = sqrt(fro2) / n;
  int lh = 0;  // 2^lh >= half: 2-D thread indices without integer division
  while ((1 << lh) < half) ++lh;
  const int hp = 1 << lh;
  // round-robin (circle method) pair table, built once per call
  for (int e = tid; e < (ne - 1) * half; e += nt) {
    const int rd = e / half, t = e - (e / half) * half;
    int p = (t + rd) % (ne - 1);
    int q = t == 0 ? ne - 1 : (ne - 1 - t + rd) % (ne - 1);
    sh.pq[rd][2 * t] = (unsigned char)(p < q ? p : q);
    sh.pq[rd][2 * t + 1] = (unsigned char)(p < q ? q : p);
  }
  if (tid == 0) sh.rflag = 0;
  __syncthreads();
  int gr = 0;  // global round counter
  for (int sweep = 0; sweep < 30; ++sweep) {
    const int cur = sweep & 1;
    for (int rd = 0; rd < ne - 1; ++rd, ++gr) {
      if (tid < half) {
        const int p = sh.pq[rd][2 * tid], q = sh.pq[rd][2 * tid + 1];
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
          const double apq = X[p * n + q];
          const double app = X[p * n + p], aqq = X[q * n + q];
          if (fabs(apq) > 1e-15 * fmax(sqrt(fabs(app * aqq)), floor_abs)) {
            sh.sig[cur] = 1;
            sh.rflag = gr + 1;
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
      if (rd == 0 && tid == 0) sh.sig[cur ^ 1] = 0;  // everyone has read it by now
      // no significant rotation in this round: nothing changes, and the next
      // round's parameters may be written without a second barrier
      if (sh.rflag != gr + 1) continue;
      // Thread (g, t): fixed pair slot t = tid mod hp, groups g = tid / hp.  All
      // operands of a thread's items are loaded before any is written back.
      const int t = tid & (hp - 1);
      const int g0 = tid >> lh, G = nt >> lh;
      if (t < half) {
        const int p2 = sh.p[t], q2 = sh.q[t];
        const double c2 = sh.c[t], s2 = sh.s[t];
        const bool hq2 = q2 < n;
        // 2x2 blocks (t1 <= t2 = t), each written with its transpose; with
        // 1024 threads a thread has one block (n <= 64) or at most three
        const double tt2 = sh.t[t];
        for (int t1 = g0; t1 <= t; t1 += G) {
          const int a1 = sh.p[t1], b1 = sh.q[t1];
          const double c1 = sh.c[t1], s1 = sh.s[t1];
          const bool hq1 = b1 < n;
          const double bpp = X[a1 * n + p2];
          const double bpq = hq2 ? X[a1 * n + q2] : 0.0;
          const double bqp = hq1 ? X[b1 * n + p2] : 0.0;
          const double bqq = (hq1 && hq2) ? X[b1 * n + q2] : 0.0;
          if (t1 == t) {
            if (hq2 && s2 != 0.0) {
              X[p2 * n + p2] = bpp - tt2 * bpq;
              X[q2 * n + q2] = bqq + tt2 * bpq;
              X[p2 * n + q2] = 0.0;
              X[q2 * n + p2] = 0.0;
            }
            continue;
          }
          if (s1 == 0.0 && s2 == 0.0) continue;
          const double lpp = c1 * bpp - s1 * bqp, lpq = c1 * bpq - s1 * bqq;
          const double lqp = s1 * bpp + c1 * bqp, lqq = s1 * bpq + c1 * bqq;
          const double npp = c2 * lpp - s2 * lpq, npq = s2 * lpp + c2 * lpq;
          const double nqp = c2 * lqp - s2 * lqq, nqq = s2 * lqp + c2 * lqq;
          X[a1 * n + p2] = npp;
          X[p2 * n + a1] = npp;
          if (hq2) {
            X[a1 * n + q2] = npq;
            X[q2 * n + a1] = npq;
          }
          if (hq1) {
            X[b1 * n + p2] = nqp;
            X[p2 * n + b1] = nqp;
          }
          if (hq1 && hq2) {
            X[b1 * n + q2] = nqq;
            X[q2 * n + b1] = nqq;
          }
        }
        // eigenvector rows k = g0, g0 + G, ... rotated in columns (p2, q2)
        if (hq2 && s2 != 0.0) {
          for (int k = g0; k < n; k += G) {
            const double vp = V[k * n + p2], vq = V[k * n + q2];
            V[k * n + p2] = c2 * vp - s2 * vq;
            V[k * n + q2] = s2 * vp + c2 * vq;
          }
        }
      }
      __syncthreads();
    }
    if (sh.sig[cur] == 0) return sweep + 1;
  }
  return -1;
}

struct RitzShared {
  JacobiShared j;
  double sv[kMaxN];
  double d[kMaxN];
  int kk[kMaxN];
  int sel[kMaxN];
  int dropmap[kMaxN];  // permuted column -> position among the kept ones, or -1
  int r;
};

static_assert(((sizeof(RitzShared) + 7) / 8) * 8 + 2 * kMaxN * kMaxN * sizeof(double) <= 160 * 1024,
              "the Ritz kernel's LDS must fit one CU (160 KiB)");

// Ranks of the diagonal of X (r x r): select the mm values nearest 0 (ties by
// value, then index) and order them ascending into sh.sel[0..mm).
__device__ void select_nearest_zero(const double* X, int r, int mm, RitzShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < r; j += nt) {
    const double mj = X[j * r + j], aj = fabs(mj);
    int rank = 0;
    for (int i = 0; i < r; ++i) {
      const double mi = X[i * r + i], ai = fabs(mi);
      if (ai < aj || (ai == aj && (mi < mj || (mi == mj && i < j)))) ++rank;
    }
    sh.kk[j] = rank;
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
}

// LDS: [RitzShared][X: nz*nz][V: nz*nz].  Global scratch: GA, GM (permuted
// order [U', W_c]), L, Li (or T, Y1 on the SVQB path), W1.
__global__ void __launch_bounds__(kThreads) k_ritz(int n_c, int m, double sigma,
                                                   const double* __restrict__ G,
                                                   const double* __restrict__ GW, double* Y,
                                                   double* theta, double* scratch, int* status) {
  extern __shared__ double lds[];
  RitzShared& sh = *reinterpret_cast<RitzShared*>(lds);
  const int nz = n_c + m;
  const int n = nz;
  double* X = lds + (sizeof(RitzShared) + 7) / 8;
  double* V = X + nz * nz;
  double* GA = scratch;        // [nz][nz]
  double* GM = GA + nz * nz;   // [nz][nz]
  double* L = GM + nz * nz;    // [nz][nz] Cholesky factor / SVQB basis T
  double* Li = L + nz * nz;    // [nz][nz] inverse of L / SVQB Y1
  double* W1 = Li + nz * nz;   // [nz][nz]
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m2 = 2 * m, nc2 = 2 * n_c;
  long long ts[6];
  ts[0] = wall_clock64();
  // permuted position a -> original Z column: a < m -> U' column a, else W column a - m
  auto orig = [&](int a) { return a < m ? n_c + a : a - m; };
  // assemble the enriched pencil (Galerkin blocks, symmetrised) in order [U', W_c]
  for (int e = tid; e < nz * nz; e += nt) {
    const int a = e / nz, b = e - (e / nz) * nz;
    const int i = orig(a), j = orig(b);
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
    L[e] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < nz; i += nt) {
    const double dg = X[i * nz + i];
    sh.sv[i] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
  }
  if (tid == 0) sh.j.flag = 1;
  __syncthreads();
  for (int e = tid; e < nz * nz; e += nt) {
    const int i = e / nz, j = e - (e / nz) * nz;
    X[e] *= sh.sv[i] * sh.sv[j];
  }
  __syncthreads();
  ts[1] = wall_clock64();
  // ---- Cholesky of the scaled Gram matrix (right-looking, one barrier per
  // column).  A column whose pivot (the squared sine of its angle to the
  // span of the kept columns before it) is below 1e-10 is dropped: it adds
  // nothing to the enriched space.  With sigma = 0 this happens to the
  // constant vector of W_c once U' holds the converged constant mode.
  if (tid == 0) sh.r = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = X[j * n + j];
    if (piv > 1e-10) {  // uniform: every thread reads the same pivot
      const double rp = sqrt(piv);
      const int w = n - j;
      for (int e = tid; e < w * w; e += nt) {
        const int i = j + e / w, k = j + e - (e / w) * w;
        if (k == j)
          L[i * n + j] = X[i * n + j] / rp;
        else if (k <= i)
          X[i * n + k] -= X[i * n + j] * X[k * n + j] / piv;
      }
      if (tid == 0) sh.kk[sh.r++] = j;
    }
    __syncthreads();
  }
  ts[2] = wall_clock64();
  int r = sh.r;
  double* T = L;  // SVQB path: basis coefficients Y = T Q
  const bool chol = r >= m;
  for (int a = tid; a < n; a += nt) sh.dropmap[a] = -1;
  __syncthreads();
  for (int q = tid; q < r; q += nt) sh.dropmap[sh.kk[q]] = q;
  if (chol) {
    // compact factor Lc = L[kept, kept] in X (LDS; X is free after the
    // factorisation) and its inverse Li in V (LDS), row by row: row i of Li
    // needs rows < i, its columns are independent.
    for (int e = tid; e < r * r; e += nt) {
      const int a = e / r, b = e - (e / r) * r;
      X[e] = (b <= a) ? L[sh.kk[a] * n + sh.kk[b]] : 0.0;
      V[e] = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < r; ++i) {
      const double lii = X[i * r + i];
      for (int c = tid; c <= i; c += nt) {
        double acc = (i == c) ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) acc -= X[i * r + k] * V[k * r + c];
        V[i * r + c] = acc / lii;
      }
      __syncthreads();
    }
    for (int e = tid; e < r * r; e += nt) Li[e] = V[e];  // kept for the final Y
    // W1 = Li B, B = S (G_A - sigma G_M) S restricted to the kept columns
    for (int e = tid; e < r * r; e += nt) {
      const int i = e / r, j = e - (e / r) * r;
      const int cj = sh.kk[j];
      double acc = 0.0;
      for (int k = 0; k <= i; ++k) {
        const int ck = sh.kk[k];
        acc += V[i * r + k] * sh.sv[ck] * (GA[ck * n + cj] - sigma * GM[ck * n + cj]);
      }
      L[e] = acc * sh.sv[cj];  // L is free now: reuse as W1
    }
    __syncthreads();
    // C = W1 Li^T
    for (int e = tid; e < r * r; e += nt) {
      const int i = e / r, j = e - (e / r) * r;
      double acc = 0.0;
      for (int k = 0; k <= j; ++k) acc += L[i * r + k] * V[j * r + k];
      X[e] = acc;
    }
    __syncthreads();
  } else {
    // ---- SVQB: eigendecompose the scaled Gram matrix, drop tiny directions
    for (int e = tid; e < nz * nz; e += nt) {
      const int i = e / nz, j = e - (e / nz) * nz;
      X[e] = GM[e] * sh.sv[i] * sh.sv[j];
    }
    __syncthreads();
    (void)block_jacobi(X, V, nz, sh.j);
    if (tid == 0) {
      double dmax = 0.0;
      for (int j = 0; j < nz; ++j) dmax = fmax(dmax, X[j * nz + j]);
      int rr = 0;
      for (int j = 0; j < nz; ++j) {
        const double dj = X[j * nz + j];
        if (dj > 1e-12 * dmax) {
          sh.kk[rr] = j;
          sh.d[rr] = dj;
          ++rr;
        }
      }
      sh.r = rr;
    }
    __syncthreads();
    r = sh.r;
    for (int e = tid; e < nz * r; e += nt) {
      const int i = e / r, q = e - (e / r) * r;
      T[e] = sh.sv[i] * V[i * nz + sh.kk[q]] / sqrt(sh.d[q]);
    }
    __syncthreads();
    for (int e = tid; e < nz * r; e += nt) {
      const int i = e / r, q = e - (e / r) * r;
      double acc = 0.0;
      for (int k = 0; k < nz; ++k) acc += (GA[i * nz + k] - sigma * GM[i * nz + k]) * T[k * r + q];
      W1[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += nt) {
      const int p = e / r, q = e - (e / r) * r;
      double acc = 0.0;
      for (int i = 0; i < nz; ++i) acc += T[i * r + p] * W1[i * r + q];
      X[e] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < r * r; e += nt) {
    const int p = e / r, q = e - (e / r) * r;
    if (p < q) {
      const double avg = 0.5 * (X[p * r + q] + X[q * r + p]);
      X[p * r + q] = avg;
      X[q * r + p] = avg;
    }
  }
  __syncthreads();
  ts[3] = wall_clock64();
  const int sw = block_jacobi(X, V, r, sh.j);
  ts[4] = wall_clock64();
  const int mm = m < r ? m : r;
  select_nearest_zero(X, r, mm, sh);
  // Y (rows in the caller's order [W_c, U']) = basis coefficients of the selection
  for (int e = tid; e < nz * m; e += nt) {
    const int a = e / m, c = e - (e / m) * m;  // a: permuted row
    double acc = 0.0;
    if (c < mm) {
      const int col = sh.sel[c];
      if (chol) {
        const int q = sh.dropmap[a];
        if (q >= 0) {
          for (int b = q; b < r; ++b) acc += Li[b * r + q] * V[b * r + col];
          acc *= sh.sv[a];
        }
      } else {
        for (int q = 0; q < r; ++q) acc += T[a * r + q] * V[q * r + col];
      }
    }
    Y[orig(a) * m + c] = acc;
  }
  for (int c = tid; c < m; c += nt) theta[c] = c < mm ? X[sh.sel[c] * r + sh.sel[c]] + sigma : 0.0;
  ts[5] = wall_clock64();
  if (tid == 0) {
    status[0] = (r < m) ? 1 : (sw < 0 ? 2 : 0);
    status[1] = sw;
    status[2] = chol ? 0 : 1;
    status[3] = n - (chol ? r : n);
    for (int i = 0; i < 5; ++i) status[4 + i] = int(ts[i + 1] - ts[i]);  // 100 MHz ticks
  }
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

int ritz_scratch_doubles(int nz) { return 5 * nz * nz; }

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
