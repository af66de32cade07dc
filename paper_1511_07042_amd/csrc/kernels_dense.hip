// One-workgroup FP64 dense kernels of the Rayleigh-Ritz step.
//
// The enriched pencil (eq. pb-c-aux-mat, Alg. 2 step 4 / Alg. 3 step 5) is
// small (nz = n_c + m <= 96) and is worked on in LDS.  Its basis is ordered
// [U', W_c] and made M-orthonormal (the "orthogonalize with respect to b_h"
// step of Alg. 2 step 3) by a Cholesky factorisation of the unit-diagonal
// scaled M-Gram matrix; because U' is close to the previous, already
// M-orthonormal and A-diagonal Ritz block, the reduced matrix
// C = L^-1 S (G_A - sigma G_M) S L^-T is then close to diagonal in its leading
// m x m block and Jacobi needs few sweeps.  When fewer than m Cholesky pivots
// exceed 1e-10 (the basis is numerically rank deficient) the kernel switches
// to SVQB (Stathopoulos & Wu, SIAM J. Sci. Comput. 2002: eigendecompose the
// scaled Gram matrix, drop directions below 1e-12 of the largest eigenvalue).
// The m eigenpairs nearest sigma are kept (Alg. 2 step 2, Remark 4.1).
//
// The work is latency-bound: the kernel runs eight waves (two per SIMD),
// stores symmetric matrices packed (lower triangle by rows) so two of them and
// the full eigenvector matrix fit one CU's LDS for nz <= 96, and every loop that
// runs once per column or per Jacobi round touches LDS only.
//
// Jacobi method (Golub & Van Loan, Matrix Computations, Sec. 8.5): two-sided
// rotations in parallel (round-robin) order.  In a round the n/2 disjoint
// pairs (p, q) are rotated at once.  Each wave computes the round's rotations
// (lane i: pair i) into its own LDS slot, so no barrier is needed to share
// them; a round in which no rotation is significant is skipped by every wave
// (the vote is identical in all of them).  Otherwise the 2x2 blocks
// [p1 q1] x [p2 q2] of the packed matrix and the rotated rows of the
// eigenvector matrix are updated in place between two barriers.  Only
// significant rotations are applied, a_pq^2 > rtol2 max(|a_pp a_qq|,
// (||A||_F / n)^2) (rtol2 = 1e-22 in the Ritz step), so rounding noise is not
// churned; sweeps stop after a sweep without one.  Across cycles the Ritz step
// starts Jacobi from the previous cycle's basis of the coarse block (see
// k_ritz), which leaves mostly the small couplings the correction introduced.
#include <cmath>
#include <mutex>

#include "bmg_internal.h"

namespace bmg {
namespace {

constexpr int kMaxN = 96;
constexpr int kMaxHalf = kMaxN / 2;
constexpr int kWarmMax = 24;  // largest coarse block the Ritz step warm-starts
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

// packed lower-triangular index, i >= j
__device__ __forceinline__ int tri(int i, int j) { return ((i * (i + 1)) >> 1) + j; }
// packed symmetric index, any order
__device__ __forceinline__ int sym(int i, int j) { return i >= j ? tri(i, j) : tri(j, i); }

struct alignas(16) RotRec {
  double c, s, t;
  int p, q;
};

struct JacobiShared {
  // each wave's copy of the round's rotations (written and read by that wave
  // only): (c, s), t, and the pair (p, q)
  double2 cs[kWaves][kMaxHalf];
  double tt[kWaves][kMaxHalf];
  double red[2 * kWaves];
  double bcast[2];
  int sig[3];  // per sweep (mod 3): a significant rotation was applied
  int rounds;  // rounds with at least one significant rotation
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// Pair of slot t in round rd of the circle method on ne (even) indices, p < q.
__device__ __forceinline__ void rr_pair(int t, int rd, int ne, int& p, int& q) {
  const int m1 = ne - 1;
  int a = t + rd;
  if (a >= m1) a -= m1;
  int b = m1;
  if (t != 0) {
    b = m1 - t + rd;
    if (b >= m1) b -= m1;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Symmetric Schur rotation of the pair (p, q) of the packed matrix X
// (Golub & Van Loan, Alg. 8.5.1, with tau = d / b folded into
// t = sign(d) b / (|d| + hypot(d, b))), or the identity (s = 0) when a_pq is
// not significant.  The square roots and the division start from the
// hardware estimates (v_rsq_f64, v_rcp_f64) refined by Newton steps: t only
// has to be close to the annihilating tangent (a small error leaves a tiny
// a_pq for the next sweep), but c = (1 + t^2)^-1/2 is refined to full
// precision so that c^2 + s^2 = 1 to rounding and V stays orthogonal.
__device__ __forceinline__ double rsq_refined(double u, int steps) {
  double r = __builtin_amdgcn_rsq(u);
  for (int i = 0; i < steps; ++i) r = r * fma(-0.5 * u * r, r, 1.5);
  return r;
}

__device__ __forceinline__ RotRec rot_params(const double* X, int p, int q, int n, double floor2,
                                             double rtol2) {
  RotRec r{1.0, 0.0, 0.0, p, q};
  if (q >= n) return r;
  const double apq = X[tri(q, p)], app = X[tri(p, p)], aqq = X[tri(q, q)];
  if (apq * apq > rtol2 * fmax(fabs(app * aqq), floor2)) {
    const double d = aqq - app, b = 2.0 * apq;
    const double h2 = fma(d, d, b * b);
    double t;
    if (h2 > 1e-280 && h2 < 1e280) {
      const double h = h2 * rsq_refined(h2, 1);
      const double den = fabs(d) + h;
      double rc = __builtin_amdgcn_rcp(den);
      rc = rc * fma(-den, rc, 2.0);
      t = (d >= 0.0 ? b : -b) * rc;
    } else {
      t = (d >= 0.0 ? b : -b) / (fabs(d) + sqrt(d * d + b * b));
    }
    const double u = fma(t, t, 1.0);
    r.c = rsq_refined(u, 2);
    r.s = t * r.c;
    r.t = t;
  }
  return r;
}

// Diagonalise the packed symmetric n x n matrix X (LDS) in place.  On return
// X holds the diagonal form (eigenvalues on the diagonal, unsorted) and V (LDS)
// holds the eigenvectors as rows: V[j * ldv + i] = component i of eigenvector
// j, with ldv = n rounded up to even, so X_in = V^T diag V.  With Q0 set, X is
// taken to be T^T C T for T = diag(I_m0, Q0) (Q0: (n - m0)^2, row-major,
// orthogonal, in LDS) and V starts from T^T, so that on return V holds the
// eigenvectors of C instead.  A rotation is
// significant when a_pq^2 > rtol2 max(|a_pp a_qq|, (||X||_F / n)^2); sweeps
// stop after a sweep without one.  Returns the sweeps used, or -1 if the limit
// was hit.
//
// A round costs two barriers (rotations computed, then updates done), and
// nothing when none of its rotations is significant.  Every wave computes the
// round's rotations (lane i: pair i) into its own LDS slot and keeps the
// ballot of significant pairs in a scalar register; the pairs themselves are
// recomputed from the round number (circle method) wherever they are needed.
// A thread touches a 2x2 block of X only if one of its two rotations is
// significant, and a 16-byte item of two rows of V only if its rotation is.
// The blocks of a round partition X and the items partition the changed
// entries of V, so the updates are done in place.
__device__ __forceinline__ int block_jacobi(double* X, double* V, int n, JacobiShared& sh,
                                            double rtol2, const double* Q0 = nullptr, int m0 = 0) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int ne = n + (n & 1);
  const int ldv = ne;
  const int half = ne / 2;
  const int nb = half * (half + 1) / 2;  // blocks (t1 <= t2)
  constexpr int kNB = (kMaxHalf * (kMaxHalf + 1) / 2 + kThreads - 1) / kThreads;
  constexpr int kVI = (kMaxHalf * kMaxHalf + kThreads - 1) / kThreads;
  double f2 = 0.0;
  const int nw0 = n - m0;
  for (int e = tid; e < n * ldv; e += nt) {
    const int i = e / ldv, j = e - (e / ldv) * ldv;
    V[e] = (Q0 != nullptr && i >= m0 && j >= m0 && j < n) ? Q0[(j - m0) * nw0 + (i - m0)]
                                                           : ((i == j) ? 1.0 : 0.0);
    if (j < n) {
      const double x = X[sym(i, j)];
      f2 += x * x;
    }
  }
  if (tid == 0) {
    sh.sig[0] = 0;
    sh.sig[1] = 0;
    sh.sig[2] = 0;
    sh.rounds = 0;
  }
  double fro2, dummy;
  block_sum2(f2, 0.0, sh, fro2, dummy);
  const double floor2 = fro2 / (double(n) * n);  // (||X||_F / n)^2
  // this thread's blocks b = tid + i nt, decoded once: (t1, t2), t1 <= t2
  int bt1[kNB], bt2[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i) {
    const int b = tid + i * nt;
    int t2 = -1, t1 = 0;
    if (b < nb) {
      t2 = int((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
      if (tri(t2, 0) > b) --t2;
      if (tri(t2 + 1, 0) <= b) ++t2;
      t1 = b - tri(t2, 0);
    }
    bt1[i] = t1;
    bt2[i] = t2;
  }
  // eigenvector items: (pair slot vt, column pair vc) of the rows p and q of V.
  // When the blocks fit the first half of the threads (n <= 44), the items go
  // to the second half, so no thread carries both a block and an item.
  const int nvc = ne / 2;
  const bool split = nb <= nt / 2;
  const int vbase = split ? nt / 2 : 0, vstride = split ? nt / 2 : nt;
  int vt[kVI], vc[kVI];
#pragma unroll
  for (int i = 0; i < kVI; ++i) {
    const int it = (tid - vbase) + i * vstride;
    const bool ok = tid >= vbase && it < half * nvc;
    vt[i] = ok ? it / nvc : -1;
    vc[i] = ok ? it - (it / nvc) * nvc : 0;
  }
  double2* cs = sh.cs[wave];
  double* tt = sh.tt[wave];
  int rounds = 0;  // thread 0: rounds with a significant rotation
  int ret = -1;
  for (int sweep = 0; sweep < 30 && ret < 0; ++sweep) {
    // this flag was last read at the end of sweep - 2, before the barriers of
    // sweep - 1; the next sweep writes it only after a barrier of this sweep
    if (tid == 0) sh.sig[(sweep + 1) % 3] = 0;
    for (int rd = 0; rd < ne - 1; ++rd) {
      bool sg = false;
      if (lane < half) {
        int p, q;
        rr_pair(lane, rd, ne, p, q);
        const RotRec r = rot_params(X, p, q, n, floor2, rtol2);
        cs[lane] = double2{r.c, r.s};
        tt[lane] = r.t;
        sg = r.s != 0.0;
      }
      // identical in every wave: skip the round (no writes, no barrier)
      const uint64_t mask = __ballot(sg);
      if (mask == 0) continue;
      if (tid == 0) {
        sh.sig[sweep % 3] = 1;
        ++rounds;
      }
      // every wave has read X for its rotations before any thread updates X
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kNB; ++i) {
        if (bt2[i] < 0) continue;
        const int t1 = bt1[i], t2 = bt2[i];
        const bool g1 = (mask >> t1) & 1, g2 = (mask >> t2) & 1;
        if (!g1 && !g2) continue;
        int a1, b1, p2, q2;
        rr_pair(t2, rd, ne, p2, q2);
        const double2 C2 = cs[t2];
        if (t1 == t2) {
          const double app = X[tri(p2, p2)], apq = X[tri(q2, p2)], aqq = X[tri(q2, q2)];
          const double t = tt[t2];
          X[tri(p2, p2)] = app - t * apq;
          X[tri(q2, q2)] = aqq + t * apq;
          X[tri(q2, p2)] = 0.0;
          continue;
        }
        rr_pair(t1, rd, ne, a1, b1);
        const double2 C1 = cs[t1];
        const bool hq1 = b1 < n, hq2 = q2 < n;
        const double bpp = X[sym(a1, p2)];
        const double bpq = hq2 ? X[sym(a1, q2)] : 0.0;
        const double bqp = hq1 ? X[sym(b1, p2)] : 0.0;
        const double bqq = (hq1 && hq2) ? X[sym(b1, q2)] : 0.0;
        const double c1 = C1.x, s1 = C1.y, c2 = C2.x, s2 = C2.y;
        const double lpp = c1 * bpp - s1 * bqp, lpq = c1 * bpq - s1 * bqq;
        const double lqp = s1 * bpp + c1 * bqp, lqq = s1 * bpq + c1 * bqq;
        X[sym(a1, p2)] = c2 * lpp - s2 * lpq;
        if (hq2) X[sym(a1, q2)] = s2 * lpp + c2 * lpq;
        if (hq1) X[sym(b1, p2)] = c2 * lqp - s2 * lqq;
        if (hq1 && hq2) X[sym(b1, q2)] = s2 * lqp + c2 * lqq;
      }
#pragma unroll
      for (int i = 0; i < kVI; ++i) {
        if (vt[i] < 0 || !((mask >> vt[i]) & 1)) continue;
        int p, q;
        rr_pair(vt[i], rd, ne, p, q);
        const double2 C = cs[vt[i]];
        double2* vp = reinterpret_cast<double2*>(V + p * ldv) + vc[i];
        double2* vq = reinterpret_cast<double2*>(V + q * ldv) + vc[i];
        const double2 a = *vp, b = *vq;
        *vp = double2{C.x * a.x - C.y * b.x, C.x * a.y - C.y * b.y};
        *vq = double2{C.y * a.x + C.x * b.x, C.y * a.y + C.x * b.y};
      }
      __syncthreads();
    }
    if (sh.sig[sweep % 3] == 0) ret = sweep + 1;
  }
  if (tid == 0) sh.rounds = rounds;
  __syncthreads();
  return ret;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// C (M x N) = A (M x K) B (K x N) for small operands in LDS, on the FP64
// matrix cores: the 16 x 16 output tiles are shared out over the workgroup's
// wavefronts; a tile runs ceil(K / 4) v_mfma_f64_16x16x4f64 steps with the
// fragments fetched through fa(i, k) and fb(k, j) (0 outside the operands), and
// each output element is handed once to fo(i, j, value).  Lane layouts: A lane
// l holds row l % 16 and k = l / 16; B lane l holds k = l / 16 and column l % 16;
// result lane l holds column l % 16 of rows l / 16 + 4 v.  skip(ti, tj) drops
// tiles whose outputs are not needed.  The fragments of eight k steps are
// fetched before their MFMAs, so a tile waits on LDS once per 32 of K.
template <class FA, class FB, class FO, class SK>
__device__ __forceinline__ void lds_mfma_gemm(int M, int N, int K, FA fa, FB fb, FO fo, SK skip) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  for (int id = wave; id < tm * tn; id += nw) {
    const int ti = id / tn, tj = id - (id / tn) * tn;
    if (skip(ti, tj)) continue;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    const int i = 16 * ti + li, j = 16 * tj + li;
    constexpr int kS = 8;
    for (int k0 = 0; k0 < K; k0 += 4 * kS) {
      double a[kS], b[kS];
#pragma unroll
      for (int t = 0; t < kS; ++t) {
        const int k = k0 + 4 * t + lk;
        a[t] = (i < M && k < K) ? fa(i, k) : 0.0;
        b[t] = (k < K && j < N) ? fb(k, j) : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kS; ++t)
        if (k0 + 4 * t < K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * ti + lk + 4 * v;
      if (row < M && j < N) fo(row, j, acc[v]);
    }
  }
}

struct RitzShared {
  JacobiShared j;
  double sv[kMaxN];
  double d[kMaxN];
  int kk[kMaxN];
  int sel[kMaxN];
  int rank[kMaxN];     // selection scratch
  double p1[kMaxN];    // Cholesky: pivots of the blocks' rows j + 1..j + 3
  int dropmap[kMaxN];  // permuted column -> position among the kept ones, or -1
  int wany[kWaves];    // block_any: per-wave votes
  int r;
};

// true in every thread if pred holds in any thread of the workgroup (two
// barriers; a workgroup reduction of the device library would add static LDS,
// and the kernel needs all 160 KiB as dynamic LDS)
__device__ bool block_any(bool pred, RitzShared& sh) {
  const uint64_t b = __ballot(pred);
  if ((threadIdx.x & 63) == 0) sh.wany[threadIdx.x >> 6] = b != 0;
  __syncthreads();
  bool any = false;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) any = any || sh.wany[w] != 0;
  __syncthreads();
  return any;
}

// doubles before the matrices: even, so the eigenvector rows are 16-byte aligned
constexpr int shared_doubles() { return int((sizeof(RitzShared) + 15) / 16) * 2; }
// doubles of the eigenvector matrix: n rows of n rounded up to even
__host__ __device__ constexpr int vsize(int n) { return n * (n + (n & 1)); }

// LDS: [RitzShared][R0: n*n][Ra: n(n+1)/2][Rb: n(n+1)/2]
size_t lds_bytes(int n) { return (size_t(shared_doubles()) + size_t(vsize(n)) + size_t(n) * (n + 1)) * 8; }

static_assert((shared_doubles() + vsize(kMaxN) + kMaxN * (kMaxN + 1)) * 8 <= 160 * 1024,
              "the Ritz kernel's LDS must fit one CU (160 KiB)");

// Select the mm diagonal entries of the packed r x r matrix X nearest 0 (ties
// by value, then index) and order them ascending into sh.sel[0..mm).  The
// wavefronts share out the entries j; a wavefront counts the entries ahead of
// j with one ballot per 64 of them (lane l compares entry i0 + l).
__device__ void select_nearest_zero(const double* X, int r, int mm, RitzShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwv = nt >> 6;
  for (int j = tid; j < r; j += nt) sh.d[j] = X[tri(j, j)];
  __syncthreads();
  for (int j = wave; j < r; j += nwv) {
    const double mj = sh.d[j], aj = fabs(mj);
    int rank = 0;
    for (int i0 = 0; i0 < r; i0 += 64) {
      const int i = i0 + lane;
      bool ahead = false;
      if (i < r) {
        const double mi = sh.d[i], ai = fabs(mi);
        ahead = ai < aj || (ai == aj && (mi < mj || (mi == mj && i < j)));
      }
      rank += __popcll(__ballot(ahead));
    }
    if (lane == 0) sh.rank[j] = rank;
  }
  __syncthreads();
  for (int j = wave; j < r; j += nwv) {
    if (sh.rank[j] >= mm) continue;  // the same j in every lane of the wavefront
    const double mj = sh.d[j];
    int pos = 0;
    for (int i0 = 0; i0 < r; i0 += 64) {
      const int i = i0 + lane;
      bool ahead = false;
      if (i < r && sh.rank[i] < mm) {
        const double mi = sh.d[i];
        ahead = mi < mj || (mi == mj && i < j);
      }
      pos += __popcll(__ballot(ahead));
    }
    if (lane == 0) sh.sel[pos] = j;
  }
  __syncthreads();
}

// Global scratch: GA, GM (permuted order [U', W_c]; read back by SVQB only),
// an unused nz^2 slot, Lg (packed inverse Cholesky factor, or the SVQB basis
// T), W1 (SVQB only).  The scaled shifted matrix S (GA - sigma GM) S stays in
// LDS (packed, in R0) until the products.
__device__ __forceinline__ void ritz_body(double* lds, int n_c, int m, double sigma, double rtol2, int warm,
                                          const double* __restrict__ G, const double* __restrict__ GW,
                                          double* Y, double* theta, double* scratch, int* status,
                                          const double* __restrict__ rho2) {
  RitzShared& sh = *reinterpret_cast<RitzShared*>(lds);
  // Jacobi's significance threshold follows the block's accuracy: with the
  // previous Ritz values theta and residual norms rho2 (both [m], read before
  // theta is overwritten), eps = the geometric mean over the columns of
  // sqrt(rho2_j) / max(|theta_j|, 1) (a column already exact, such as the
  // constant mode inside the coarse space, does not pin it at rounding), and
  // rotations below tau = 1e-3 eps (at most 1e-4, at least sqrt(rtol2)) are
  // skipped.  A skipped rotation moves a Ritz vector by about tau times
  // ||C|| over the gap to the other values, three orders below the block's
  // typical error, so it does not slow the iteration; the certificate is
  // computed from true residuals either way.  rho2 null: rtol2 as given.
  if (rho2 != nullptr) {
    if (threadIdx.x < 64) {
      double e = 0.0;
      for (int j = threadIdx.x; j < m; j += 64)
        e += log(fmax(sqrt(fmax(rho2[j], 0.0)) / fmax(fabs(theta[j]), 1.0), 1e-30));
      for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
      if (threadIdx.x == 0) sh.j.bcast[0] = exp(e / m);
    }
    __syncthreads();
    const double tau = fmin(1e-4, 1e-3 * sh.j.bcast[0]);
    rtol2 = fmax(rtol2, tau * tau);
    __syncthreads();  // bcast is reused below
  }
  const int nz = n_c + m;
  const int n = nz;
  double* R0 = lds + shared_doubles();  // [nz][nz] (eigenvectors: rows of even length)
  double* Ra = R0 + vsize(nz);          // packed
  double* Rb = Ra + nz * (nz + 1) / 2;  // packed
  double* GA = scratch;
  double* GM = GA + nz * nz;
  double* Lg = GM + 2 * nz * nz;
  double* W1 = Lg + nz * nz;
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
    if (b <= a) {  // lower triangles (both blocks are symmetric) into LDS
      Ra[tri(a, b)] = vm;
      Rb[tri(a, b)] = va;
    }
  }
  __syncthreads();
  for (int i = tid; i < nz; i += nt) {
    const double dg = Ra[tri(i, i)];
    sh.sv[i] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
  }
  if (tid == 0) sh.r = 0;
  __syncthreads();
  for (int e = tid; e < nz * nz; e += nt) {
    const int i = e / nz, j = e - (e / nz) * nz;
    if (j > i) continue;
    const double sij = sh.sv[i] * sh.sv[j];
    const double vm = Ra[tri(i, j)], va = Rb[tri(i, j)];
    Ra[tri(i, j)] = vm * sij;
    Rb[tri(i, j)] = (i == j) ? 1.0 : 0.0;
    R0[tri(i, j)] = (va - sigma * vm) * sij;  // S (GA - sigma GM) S, packed
  }
  __syncthreads();
  ts[1] = wall_clock64();
  // ---- Cholesky of the scaled Gram matrix X (Ra), right-looking, one
  // barrier per column.  Step j subtracts f_i = X_ij / X_jj times the pivot
  // row from every row i > j: on the trailing part of X (columns j < c <= i)
  // and, in the same pass, on Z (Rb, columns c <= j), which starts as I and
  // so ends as the unit lower-triangular inverse of the LDL^T factor:
  // L^-1 = D^-1/2 Z.  A column whose pivot (the squared sine of its angle to
  // the span of the kept columns before it) is below 1e-10 is dropped: it
  // adds nothing to the enriched space.  With sigma = 0 this happens to the
  // constant vector of W_c once U' holds the converged constant mode.
  // Columns are eliminated four at a time (one barrier per block of four).
  // Every thread factors the block's 4 x 4 pivot part (LDL^T: pivots p_t,
  // multipliers l_kt) from the values before the block.  A trailing row i
  // forms its multipliers f_t by forward substitution from its four block
  // entries, and every entry it owns subtracts sum_t f_t y_t(c), where y_t(c),
  // pivot row t's value at column c after the block's earlier steps, comes
  // from the stored pivot rows by the same substitution
  // (y_t = x_t - sum_{r<t} l_tr y_r; on Z the pivot rows start as the
  // identity in the block's columns).  The pivot rows' own Z rows and pivots
  // are written after the last block (every thread of a pass reads the old
  // ones); the multipliers are kept in the Jacobi scratch, free until Jacobi.
  constexpr int kCW = 16, kCE = (kMaxN + kCW - 1) / kCW;
  constexpr int kB = 4;
  double* lblk = reinterpret_cast<double*>(sh.j.cs);  // [n][3]: l_{t,r} of pivot row j + t
  static_assert(sizeof(sh.j.cs) >= sizeof(double) * kMaxN * 3, "block multipliers fit the Jacobi scratch");
  int j = 0;
  for (; j + kB - 1 < n; j += kB) {
    // the pivot block (lower part, values before this block), factored
    double a[kB][kB];
#pragma unroll
    for (int t = 0; t < kB; ++t)
#pragma unroll
      for (int u = 0; u <= t; ++u) a[t][u] = Ra[tri(j + t, j + u)];
    double pv[kB], ip[kB], l[kB][kB];
    bool kept[kB];
#pragma unroll
    for (int t = 0; t < kB; ++t) {
      pv[t] = a[t][t];
      kept[t] = pv[t] > 1e-10;  // uniform: every thread reads the same values
      ip[t] = kept[t] ? 1.0 / pv[t] : 0.0;
#pragma unroll
      for (int k = t + 1; k < kB; ++k) {
        l[k][t] = a[k][t] * ip[t];
#pragma unroll
        for (int u = t + 1; u <= k; ++u) a[k][u] -= l[k][t] * a[u][t];
      }
    }
    if (tid == 0) {
#pragma unroll
      for (int t = 1; t < kB; ++t) {
        sh.p1[j + t] = pv[t];
#pragma unroll
        for (int r = 0; r < t; ++r) lblk[(j + t) * 3 + r] = l[t][r];
      }
#pragma unroll
      for (int t = 0; t < kB; ++t)
        if (kept[t]) sh.kk[sh.r++] = j + t;
    }
    // trailing rows i > j + 3, on the matrix cores: every entry (i, c), c <= i,
    // subtracts sum_t f_t(i) y_t(c), a rank-4 product, one
    // v_mfma_f64_16x16x4f64 per 16 x 16 tile.  A lane of the A fragment holds
    // -f_k(i) of row i (k = lane / 16), a lane of the B fragment y_k(c) of
    // column c; the result lane holds column c of four rows.  A tile reads and
    // writes only its own entries, and the pivot rows (read by every tile) and
    // the rows' block columns of X (the f sources; those entries of Z are
    // written instead) are not written in this step.
    const int jl = j + kB - 1;
    const int w = n - 1 - jl;
    {
      const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
      const int li = lane & 15, lk = lane >> 4;
      const int tm = (w + 15) / 16, tn = (n + 15) / 16;
      for (int id = wv; id < tm * tn; id += nwv) {
        const int ti = id / tn, tj = id - (id / tn) * tn;
        const int i0 = jl + 1 + 16 * ti, c0 = 16 * tj;
        if (c0 > i0 + 15) continue;  // above the diagonal
        double fa = 0.0, fb = 0.0;
        const int i = i0 + li;
        if (i < n) {
          double f[kB];
#pragma unroll
          for (int t = 0; t < kB; ++t) {
            double x = Ra[tri(i, j + t)];
#pragma unroll
            for (int r = 0; r < t; ++r) x -= f[r] * a[t][r];  // a[t][r]: pivot row r at column t, step r
            f[t] = x * ip[t];
          }
          fa = -(lk == 0 ? f[0] : lk == 1 ? f[1] : lk == 2 ? f[2] : f[3]);
        }
        const int c = c0 + li;
        const bool zpart = c <= jl;
        if (c < n) {
          double y[kB];
#pragma unroll
          for (int t = 0; t < kB; ++t) {
            double v = zpart ? (c <= j + t ? Rb[tri(j + t, c)] : 0.0) : Ra[tri(c, j + t)];
#pragma unroll
            for (int r = 0; r < t; ++r) v -= l[t][r] * y[r];
            y[t] = v;
          }
          fb = lk == 0 ? y[0] : lk == 1 ? y[1] : lk == 2 ? y[2] : y[3];
        }
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb, acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = i0 + lk + 4 * v;
          if (row < n && c <= row) {
            if (zpart)
              Rb[tri(row, c)] = (c < j ? Rb[tri(row, c)] : 0.0) + acc[v];
            else
              Ra[tri(row, c)] += acc[v];
          }
        }
      }
    }
    __syncthreads();
  }
  // the blocks' pivot rows t = 1..3: their Z rows take the block's earlier
  // steps, z_t = z_t - sum_{r<t} l_tr z_r (columns c < j + t, rows j..j+t-1
  // final), and their pivots are stored
  for (int e = tid; e < (j / kB) * (j + kB); e += nt) {
    const int jb = kB * (e / (j + kB)), c = e - (e / (j + kB)) * (j + kB);
    if (c >= jb + kB - 1) continue;
    double z[kB];
    z[0] = c <= jb ? Rb[tri(jb, c)] : 0.0;
#pragma unroll
    for (int t = 1; t < kB; ++t) {
      double v = c <= jb + t ? Rb[tri(jb + t, c)] : 0.0;
#pragma unroll
      for (int r = 0; r < t; ++r) v -= lblk[(jb + t) * 3 + r] * z[r];
      z[t] = v;
      if (c < jb + t) Rb[tri(jb + t, c)] = v;
    }
  }
  for (int e = tid; e < j; e += nt)
    if (e % kB != 0) Ra[tri(e, e)] = sh.p1[e];
  __syncthreads();
  for (; j < n; ++j) {  // a last single column
    const double piv = Ra[tri(j, j)];
    if (piv > 1e-10) {
      const int w = n - 1 - j;
      const double ip = 1.0 / piv;
      for (int idx = tid; idx < w * kCW; idx += nt) {
        const int i = j + 1 + idx / kCW, cl = idx % kCW;
        double src[kCE], dst[kCE];
#pragma unroll
        for (int u = 0; u < kCE; ++u) {
          const int c = cl + kCW * u;
          src[u] = dst[u] = 0.0;
          if (c <= i) {
            src[u] = c <= j ? Rb[tri(j, c)] : Ra[tri(c, j)];
            dst[u] = c <= j ? Rb[tri(i, c)] : Ra[tri(i, c)];
          }
        }
        const double f = Ra[tri(i, j)] * ip;
#pragma unroll
        for (int u = 0; u < kCE; ++u) {
          const int c = cl + kCW * u;
          if (c <= i) {
            const double v = dst[u] - f * src[u];
            if (c <= j)
              Rb[tri(i, c)] = v;
            else
              Ra[tri(i, c)] = v;
          }
        }
      }
      if (tid == 0) sh.kk[sh.r++] = j;
    }
    __syncthreads();
  }
  for (int j = tid; j < n; j += nt) {
    sh.d[j] = Ra[tri(j, j)];
    sh.p1[j] = sqrt(sh.d[j]);  // kept pivots only are read (the blocks' pivots are no longer needed)
  }
  __syncthreads();
  ts[2] = wall_clock64();
  int r = sh.r;
  const bool chol = r >= m;
  for (int a = tid; a < n; a += nt) sh.dropmap[a] = -1;
  __syncthreads();
  for (int q = tid; q < r; q += nt) sh.dropmap[sh.kk[q]] = q;
  double* cur = Rb;
  double* nxt = Ra;
  if (chol) {
    // Li = D^-1/2 Z on the kept rows and columns into Ra (and Lg)
    for (int e = tid; e < r * r; e += nt) {
      const int a = e / r, b = e - (e / r) * r;
      if (b <= a) {
        const int ka = sh.kk[a], kb = sh.kk[b];
        const double v = Rb[tri(ka, kb)] / sh.p1[ka];
        Ra[tri(a, b)] = v;
        Lg[tri(a, b)] = v;
      }
    }
    __syncthreads();
    // Bk = the scaled shifted matrix on the kept rows and columns (kk is
    // increasing, so a >= b reads the lower triangle), packed, into Rb
    for (int e = tid; e < r * r; e += nt) {
      const int a = e / r, b = e - (e / r) * r;
      if (b <= a) Rb[tri(a, b)] = R0[tri(sh.kk[a], sh.kk[b])];
    }
    __syncthreads();
    // W1 = Li Bk into R0 (r x r), then C = W1 Li^T: only its lower triangle is
    // kept (C is symmetric; the packed Jacobi matrix stores the lower part)
    lds_mfma_gemm(
        r, r, r, [&](int i, int k) { return k <= i ? Ra[tri(i, k)] : 0.0; },
        [&](int k, int j) { return Rb[sym(k, j)]; },
        [&](int i, int j, double v) { R0[i * r + j] = v; }, [](int, int) { return false; });
    __syncthreads();
    lds_mfma_gemm(
        r, r, r, [&](int i, int k) { return R0[i * r + k]; },
        [&](int k, int j) { return k <= j ? Ra[tri(j, k)] : 0.0; },
        [&](int i, int j, double v) {
          if (j <= i) Rb[tri(i, j)] = v;
        },
        [](int ti, int tj) { return tj > ti; });
    __syncthreads();
  } else {
    // ---- SVQB: eigendecompose the scaled Gram matrix, drop tiny directions
    for (int e = tid; e < nz * nz; e += nt) {
      const int i = e / nz, j = e - (e / nz) * nz;
      if (j <= i) Rb[tri(i, j)] = GM[e] * sh.sv[i] * sh.sv[j];
    }
    __syncthreads();
    (void)block_jacobi(cur, R0, nz, sh.j, 1e-30);
    if (tid == 0) {
      double dmax = 0.0;
      for (int j = 0; j < nz; ++j) dmax = fmax(dmax, cur[tri(j, j)]);
      int rr = 0;
      for (int j = 0; j < nz; ++j) {
        const double dj = cur[tri(j, j)];
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
    double* T = Lg;  // [nz][r]: basis coefficients
    for (int e = tid; e < nz * r; e += nt) {
      const int i = e / r, q = e - (e / r) * r;
      T[e] = sh.sv[i] * R0[sh.kk[q] * (nz + (nz & 1)) + i] / sqrt(sh.d[q]);
    }
    __syncthreads();
    for (int e = tid; e < nz * r; e += nt) {
      const int i = e / r, q = e - (e / r) * r;
      double acc = 0.0;
      for (int k = 0; k < nz; ++k) acc += (GA[i * nz + k] - sigma * GM[i * nz + k]) * T[k * r + q];
      W1[e] = acc;
    }
    __syncthreads();
    cur = Rb;
    nxt = Ra;
    for (int e = tid; e < r * r; e += nt) {
      const int p = e / r, q = e - (e / r) * r;
      if (q > p) continue;
      double a1 = 0.0, a2 = 0.0;
      for (int i = 0; i < nz; ++i) {
        a1 += T[i * r + p] * W1[i * r + q];
        a2 += T[i * r + q] * W1[i * r + p];
      }
      Rb[tri(p, q)] = 0.5 * (a1 + a2);
    }
    __syncthreads();
  }
  // ---- warm start of the coarse block.  The previous call on this scratch
  // left an orthonormal basis Q of the coarse (W_c) part that nearly
  // diagonalises it, for the same kept columns: C is rotated to T^T C T,
  // T = diag(I_m, Q), and Jacobi starts from V = T^T.  Q is only a change of
  // basis of the same space, so the Ritz pairs are unchanged (up to rounding);
  // Jacobi mostly has the U'-U' and U'-W_c couplings left, which the previous
  // cycle's correction made small.
  double* Qg = scratch + 5 * nz * nz;
  int* whdr = reinterpret_cast<int*>(Qg + kWarmMax * kWarmMax);
  const int nw = r - m;
  const bool uprefix = chol && nw >= 1 && nw <= kWarmMax && nw * nw <= r * (r + 1) / 2;
  bool use_warm = false;
  if (uprefix && warm) {
    const bool hdr_ok = whdr[0] == 1 && whdr[1] == r;
    bool bad = false;
    for (int q = tid; q < r; q += nt) bad = bad || whdr[4 + q] != sh.kk[q];
    use_warm = hdr_ok && !block_any(bad, sh);
  }
  double* Qs = nxt;  // free: the inverse factor is also in Lg
  if (use_warm) {
    for (int e = tid; e < nw * nw; e += nt) Qs[e] = Qg[e];
    __syncthreads();
    // H = Q^T C[W rows, :] (nw x r) into R0 (free until Jacobi starts)
    for (int e = tid; e < nw * r; e += nt) {
      const int i = e / r, j = e - (e / r) * r;
      double acc = 0.0;
      for (int k = 0; k < nw; ++k) acc += Qs[k * nw + i] * cur[sym(m + k, j)];
      R0[e] = acc;
    }
    __syncthreads();
    // rows >= m of T^T C T, in place: [H_U | H_W Q]
    for (int e = tid; e < nw * r; e += nt) {
      const int i = e / r, j = e - (e / r) * r;
      if (j < m) {
        cur[tri(m + i, j)] = R0[e];
      } else if (j - m <= i) {
        double acc = 0.0;
        for (int k = 0; k < nw; ++k) acc += R0[i * r + m + k] * Qs[k * nw + (j - m)];
        cur[tri(m + i, j)] = acc;
      }
    }
    __syncthreads();
  }
  ts[3] = wall_clock64();
  const int sw = use_warm ? block_jacobi(cur, R0, r, sh.j, rtol2, Qs, m) : block_jacobi(cur, R0, r, sh.j, rtol2);
  ts[4] = wall_clock64();
  const int mm = m < r ? m : r;
  select_nearest_zero(cur, r, mm, sh);
  if (chol) {  // the inverse factor back into LDS (nxt is free)
    for (int e = tid; e < r * (r + 1) / 2; e += nt) nxt[e] = Lg[e];
    __syncthreads();
  }
  // Y (rows in the caller's order [W_c, U']) = basis coefficients of the selection
  const int ldv = r + (r & 1);
  if (chol) {
    // Y[kk[q]][c] = sv[kk[q]] (Li^T V_sel)[q][c] on the matrix cores; rows of
    // dropped columns and columns beyond the selection are zero
    lds_mfma_gemm(
        r, mm, r, [&](int q, int b) { return b >= q ? nxt[tri(b, q)] : 0.0; },
        [&](int b, int c) { return R0[sh.sel[c] * ldv + b]; },
        [&](int q, int c, double v) {
          const int a = sh.kk[q];
          Y[orig(a) * m + c] = sh.sv[a] * v;
        },
        [](int, int) { return false; });
    for (int e = tid; e < nz * m; e += nt) {
      const int a = e / m, c = e - (e / m) * m;
      if (sh.dropmap[a] < 0 || c >= mm) Y[orig(a) * m + c] = 0.0;
    }
  } else {
    for (int e = tid; e < nz * m; e += nt) {
      const int a = e / m, c = e - (e / m) * m;  // a: permuted row
      double acc = 0.0;
      if (c < mm) {
        const int col = sh.sel[c];
        for (int q = 0; q < r; ++q) acc += Lg[a * r + q] * R0[col * ldv + q];
      }
      Y[orig(a) * m + c] = acc;
    }
  }
  for (int c = tid; c < m; c += nt) theta[c] = c < mm ? sh.d[sh.sel[c]] + sigma : 0.0;
  // ---- the coarse-block basis for the next call: the W_c rows of the
  // eigenvectors at the W_c positions, made orthonormal by Newton-Schulz
  // steps P <- P (3 I - P^T P) / 2 (a sub-block of an orthogonal matrix, so
  // its singular values are <= 1 and the steps cannot diverge); kept only if
  // P^T P = I to 1e-13, else the next call starts cold.
  bool made = false;
  if (uprefix) {
    __syncthreads();  // Li (nxt) and the eigenvectors (R0) have been read
    double* P = nxt;
    double* Gm = cur;
    double* P2 = R0;
    for (int e = tid; e < nw * nw; e += nt) {
      const int k = e / nw, j = e - (e / nw) * nw;
      P[e] = R0[(m + j) * ldv + (m + k)];
    }
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      for (int e = tid; e < nw * nw; e += nt) {
        const int i = e / nw, j = e - (e / nw) * nw;
        double acc = 0.0;
        for (int k = 0; k < nw; ++k) acc += P[k * nw + i] * P[k * nw + j];
        Gm[e] = acc;
      }
      __syncthreads();
      for (int e = tid; e < nw * nw; e += nt) {
        const int k = e / nw, j = e - (e / nw) * nw;
        double acc = 0.0;
        for (int i = 0; i < nw; ++i) acc += P[k * nw + i] * Gm[i * nw + j];
        P2[e] = 1.5 * P[e] - 0.5 * acc;
      }
      __syncthreads();
      double* t = P;
      P = P2;
      P2 = t;
    }
    bool bad = false;
    for (int e = tid; e < nw * nw; e += nt) {
      const int i = e / nw, j = e - (e / nw) * nw;
      double acc = 0.0;
      for (int k = 0; k < nw; ++k) acc += P[k * nw + i] * P[k * nw + j];
      bad = bad || !(fabs(acc - (i == j ? 1.0 : 0.0)) <= 1e-13);
    }
    made = !block_any(bad, sh);
    for (int e = tid; e < nw * nw; e += nt) Qg[e] = P[e];
    for (int q = tid; q < r; q += nt) whdr[4 + q] = sh.kk[q];
  }
  ts[5] = wall_clock64();
  if (tid == 0) {
    whdr[0] = made ? 1 : 0;
    whdr[1] = r;
    whdr[2] = nw;
    status[0] = (r < m) ? 1 : (sw < 0 ? 2 : 0);
    status[1] = sw;
    status[2] = chol ? 0 : 1;
    status[3] = n - (chol ? r : n);
    status[9] = sh.j.rounds;
    status[10] = use_warm ? 1 : 0;
    status[11] = made ? 1 : 0;
    for (int i = 0; i < 5; ++i) status[4 + i] = int(ts[i + 1] - ts[i]);  // 100 MHz ticks
  }
}

__global__ void __launch_bounds__(kThreads) k_ritz(int n_c, int m, double sigma, double rtol2, int warm,
                                                   const double* __restrict__ G,
                                                   const double* __restrict__ GW, double* Y,
                                                   double* theta, double* scratch, int* status,
                                                   const double* __restrict__ rho2) {
  extern __shared__ double lds[];
  ritz_body(lds, n_c, m, sigma, rtol2, warm, G, GW, Y, theta, scratch, status, rho2);
}

// The Ritz steps of a grouped solve in one launch: workgroup i runs request
// i's step (its own Gram, Y, theta, scratch and status), each on a CU of its
// own, so the group's steps run side by side.
__global__ void __launch_bounds__(kThreads) k_ritz_batch(RitzBatch b, int warm) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  ritz_body(lds, b.n_c, b.m[i], b.sigma, b.rtol2, warm, b.G[i], b.GW, b.Y[i], b.theta[i], b.scratch[i],
            b.status[i], b.rho2[i]);
}

// Symmetric eigendecomposition of one n x n matrix (n <= 96), ascending.
__global__ void __launch_bounds__(kThreads) k_syev(int n, const double* __restrict__ A, double* w,
                                                   double* Vout, int* status) {
  extern __shared__ double lds[];
  RitzShared& sh = *reinterpret_cast<RitzShared*>(lds);
  double* R0 = lds + shared_doubles();
  double* cur = R0 + vsize(n);
  double* nxt = cur + n * (n + 1) / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, j = e - (e / n) * n;
    if (j <= i) cur[tri(i, j)] = 0.5 * (A[i * n + j] + A[j * n + i]);
  }
  __syncthreads();
  const int sw = block_jacobi(cur, R0, n, sh.j, 1e-30);
  for (int j = tid; j < n; j += nt) sh.d[j] = cur[tri(j, j)];
  __syncthreads();
  for (int j = tid; j < n; j += nt) {
    const double mj = sh.d[j];
    int pos = 0;
    for (int i = 0; i < n; ++i) {
      const double mi = sh.d[i];
      if (mi < mj || (mi == mj && i < j)) ++pos;
    }
    sh.sel[pos] = j;
  }
  __syncthreads();
  for (int c = tid; c < n; c += nt) w[c] = sh.d[sh.sel[c]];
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, c = e - (e / n) * n;
    Vout[e] = R0[sh.sel[c] * (n + (n & 1)) + i];
  }
  if (tid == 0) *status = sw < 0 ? 2 : 0;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

// Both kernels take up to 160 KiB of dynamic LDS (they have no static LDS).
// Set once per process (std::call_once: solves on several threads may reach
// here together); the outcome is kept and every later call returns it.
int set_lds_attr() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    for (const void* f : {(const void*)k_ritz, (const void*)k_ritz_batch, (const void*)k_syev}) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        err = e;
        return;
      }
    }
  });
  if (err != hipSuccess) {
    set_error("cannot reserve 160 KiB of LDS for the Ritz kernels: %s", hipGetErrorString(err));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

}  // namespace

// GA, GM, an unused slot, Lg, W1 (nz^2 each), then the coarse-block basis kept between
// calls (kWarmMax^2) and its header (valid, r, nw, -, kept columns: <= 128 ints)
int ritz_scratch_doubles(int nz) { return 5 * nz * nz + kWarmMax * kWarmMax + 64; }

int launch_ritz(const RitzArgs& a, hipStream_t s) {
  if (a.nz > kMaxN || a.nz != a.n_c + a.m) {
    set_error("ritz: nz = %d exceeds %d", a.nz, kMaxN);
    return BMG_EINVAL;
  }
  BMG_TRY(set_lds_attr());
  BMG_LAUNCH((k_ritz), 1, kThreads, lds_bytes(a.nz), s, a.n_c, a.m, a.sigma, a.rtol2, a.warm, a.G, a.GW, a.Y,
             a.theta, a.scratch, a.status, a.rho2);
  return check_launch();
}

int launch_ritz_batch(const RitzBatch& b, int warm, hipStream_t s) {
  int nz = 0;
  for (int i = 0; i < b.n; ++i) nz = std::max(nz, b.n_c + b.m[i]);
  if (b.n < 1 || b.n > kRitzBatchMax || nz > kMaxN) {
    set_error("ritz batch: %d requests (at most %d), nz = %d (at most %d)", b.n, kRitzBatchMax, nz, kMaxN);
    return BMG_EINVAL;
  }
  BMG_TRY(set_lds_attr());
  BMG_LAUNCH((k_ritz_batch), b.n, kThreads, lds_bytes(nz), s, b, warm);
  return check_launch();
}

int launch_syev(int n, const double* A, double* w, double* V, int* status, hipStream_t s) {
  if (n < 1 || n > kMaxN) {
    set_error("syev: n = %d outside [1, %d]", n, kMaxN);
    return BMG_EINVAL;
  }
  BMG_TRY(set_lds_attr());
  k_syev<<<1, kThreads, lds_bytes(n), s>>>(n, A, w, V, status);
  return check_launch();
}

}  // namespace bmg
