// Kernels of the interior-shift scheme: the coarse solve by the spectral
// inverse of a dense level, the per-level adaptive shifts, and the start block
// built from coarse eigenvectors.
//
// Coarse eigendecomposition.  A level l_c (a few thousand vertices) carries
// all generalized eigenpairs of (A_lc, M_lc) (Alg. 2 step 1 at that level).
// Its eigenvectors are stored one per row, phi[j][i] = x_j(i), M-orthonormal,
// so (A_lc - s M_lc)^-1 = Phi^T diag(1 / (lambda - s)) Phi with Phi = [x_0 .. x_{n-1}]^T
// and the coarse solve of the correction cycle is two dense passes over phi:
//   t[j][c] = g_j sum_i phi[j][i] f[i][c]       (rows of phi; "N")
//   e[i][c] = sum_j phi[j][i] t[j][c]            (columns of phi; "T")
// with g_j the truncated inverse 1/(lambda_j - s) (0 within tau of s: modes
// that close to the shift are left to the Ritz step).  Each pass is a tiled
// product of the n x n matrix with an n x m block (m <= 96): a workgroup
// computes a 64-row tile of the output for one slice of the contraction,
// staging a 64 x 32 tile of phi and a 32 x m tile of the block in LDS; the
// slices' partial sums are added in a fixed order by a second kernel (the
// results do not depend on scheduling).  phi is read once per pass, so a pass
// is bound by reading the n^2 matrix (FP32: 420 MB at n = 10242).
//
// Adaptive shifts (Remark 4.1 and Sec. 5.2: the coarse shift moves by the
// mean of Rayleigh quotients, which follows the drift of the discrete
// spectrum between levels).  For each level l below the finest, the values of
// the block at the level-l vertices (the first N_l rows: every level keeps
// the vertex numbers of the coarser ones) give per-column quadratic forms
// u^T A_l u and u^T M_l u; the level's shift is sigma + mean_c(u_c^T A_l u_c /
// u_c^T M_l u_c - theta_c).
#include <cmath>
#include <type_traits>

#include "bmg_internal.h"

namespace bmg {
namespace {

int check_launch_c() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return BMG_EDEVICE;
  }
  return BMG_OK;
}

int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return int(g);
}

constexpr int kTile = 64;   // output rows per workgroup
constexpr int kKc = 32;     // contraction step staged in LDS
constexpr int kMaxQ = 24;   // columns per thread (m / 4, m <= 96)

// part[s][r][c] = sum over k in slice s of A(r, k) x[k][c], with
// A(r, k) = mat[r n + k] (TRANS = false) or mat[k n + r] (TRANS = true).
template <typename T, bool TRANS>
__global__ void __launch_bounds__(256) k_dense_slices(int n, int m, int kc, const T* __restrict__ mat,
                                                      const T* __restrict__ x, T* __restrict__ part) {
  __shared__ T As[kTile][kKc + 1];
  __shared__ T Xs[kKc][kMaxQ * 4];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * kTile;
  const int s = blockIdx.y;
  const int k_begin = s * kc;
  const int k_end = min(n, k_begin + kc);
  const int rr = tid & (kTile - 1);
  const int cg = tid >> 6;  // 0..3
  const int mq = m >> 2;
  const int c0 = cg * mq;
  T acc[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) acc[q] = T(0);
  for (int k0 = k_begin; k0 < k_end; k0 += kKc) {
    // phi tile: 64 rows x 32 contraction indices
    for (int e = tid; e < kTile * kKc; e += 256) {
      int r, kk;
      if (TRANS) {
        kk = e / kTile;
        r = e - kk * kTile;
      } else {
        r = e / kKc;
        kk = e - r * kKc;
      }
      const int gr = r0 + r, gk = k0 + kk;
      T v = T(0);
      if (gr < n && gk < k_end) v = TRANS ? mat[int64_t(gk) * n + gr] : mat[int64_t(gr) * n + gk];
      As[r][kk] = v;
    }
    // block tile: 32 rows of x
    for (int e = tid; e < kKc * m; e += 256) {
      const int kk = e / m, c = e - kk * m;
      const int gk = k0 + kk;
      Xs[kk][c] = gk < k_end ? x[int64_t(gk) * m + c] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kKc; ++kk) {
      const T a = As[rr][kk];
#pragma unroll
      for (int q = 0; q < kMaxQ; ++q)
        if (q < mq) acc[q] += a * Xs[kk][c0 + q];
    }
    __syncthreads();
  }
  const int gr = r0 + rr;
  if (gr < n) {
    T* out = part + (int64_t(s) * n + gr) * m + c0;
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q)
      if (q < mq) out[q] = acc[q];
  }
}

// y[r][c] = g[r] * sum_s part[s][r][c] (g null: 1), slices added in order
template <typename T>
__global__ void k_slices_sum(int n, int m, int S, const T* __restrict__ part, const T* __restrict__ g,
                             T* __restrict__ y) {
  const int64_t cnt = int64_t(n) * m;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * blockDim.x) {
    T acc = part[e];
    for (int s = 1; s < S; ++s) acc += part[int64_t(s) * cnt + e];
    y[e] = g ? g[e / m] * acc : acc;
  }
}

// truncated inverse spectrum about the device-held shift *sh
template <typename T>
__global__ void k_spec_g(int n, const double* __restrict__ lam, const double* __restrict__ sh,
                         double tau, T* __restrict__ g) {
  const double s = sh[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double x = lam[i] - s;
    g[i] = std::fabs(x) >= tau ? T(1.0 / x) : T(0);
  }
}

// S = A - (*sh) M with the shift read from device memory
template <typename T>
__global__ void k_shift_dev(int64_t cnt, const T* __restrict__ a, const T* __restrict__ mm,
                            const double* __restrict__ sh, T* __restrict__ S) {
  const T sigma = T(sh[0]);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x)
    S[i] = a[i] - sigma * mm[i];
}

// blk[i][c] = phi[sel[c]][i]: the selected eigenvectors as an [n][m] block
__global__ void k_gather_rows(int n, int m, const double* __restrict__ phi, const int* __restrict__ sel,
                              double* __restrict__ blk) {
  const int64_t cnt = int64_t(n) * m;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / m;
    const int c = int(e - i * m);
    blk[e] = phi[int64_t(sel[c]) * n + i];
  }
}

// Injection of a coarse level's rows into a finer level's block: storage row
// r of level l is row rs[n-1][...rs[0][r]] of the finer block, rs[t] the
// general restriction tables (rself) of the stored-permuted levels between
// (each maps a row of the level below to its copy); with n = 0 it is row r
// (nested numbering: the coarse vertices come first).
constexpr int kInjMax = 4;
struct InjChain {
  const int* rs[kInjMax];
  int n;
};

__device__ __forceinline__ int64_t inject(const InjChain& c, int64_t r) {
  for (int t = 0; t < c.n; ++t) r = c.rs[t][r];
  return r;
}

// Per-block partial sums of u^T A u and u^T M u for u the injection of the
// FP64 block U [*][m] into a level of n rows: part[b][c] (A) and part[b][m + c]
// (M).  A thread owns two columns of one row at a time (rows grid-stride);
// the block's rows are added in a fixed order.
template <int WT>
__global__ void __launch_bounds__(256) k_rq_part(int64_t n, int W, int m, const int* __restrict__ cols,
                                                 const double* __restrict__ a,
                                                 const double* __restrict__ mm,
                                                 const double* __restrict__ U, double* __restrict__ part,
                                                 InjChain inj) {
  __shared__ double red[256][4];
  const int cpr = m >> 1;
  const int rpb = 256 / cpr;
  const int rloc = threadIdx.x / cpr;
  const int ch = threadIdx.x - rloc * cpr;
  double qa0 = 0, qa1 = 0, qm0 = 0, qm1 = 0;
  if (rloc < rpb) {
    for (int64_t i = int64_t(blockIdx.x) * rpb + rloc; i < n; i += int64_t(gridDim.x) * rpb) {
      const int64_t base = i * W;
      double ax0 = 0, ax1 = 0, mx0 = 0, mx1 = 0;
      const int width = WT > 0 ? WT : W;
      for (int k = 0; k < width; ++k) {
        const int64_t j = inject(inj, cols[base + k]);
        const double av = a[base + k], mv = mm[base + k];
        const double2 xv = *reinterpret_cast<const double2*>(U + j * m + 2 * ch);
        ax0 += av * xv.x;
        ax1 += av * xv.y;
        mx0 += mv * xv.x;
        mx1 += mv * xv.y;
      }
      const double2 ui = *reinterpret_cast<const double2*>(U + inject(inj, i) * m + 2 * ch);
      qa0 += ui.x * ax0;
      qa1 += ui.y * ax1;
      qm0 += ui.x * mx0;
      qm1 += ui.y * mx1;
    }
  }
  red[threadIdx.x][0] = qa0;
  red[threadIdx.x][1] = qa1;
  red[threadIdx.x][2] = qm0;
  red[threadIdx.x][3] = qm1;
  __syncthreads();
  if (threadIdx.x < cpr) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int r = 0; r < rpb; ++r) {
      const int t = r * cpr + threadIdx.x;
      s0 += red[t][0];
      s1 += red[t][1];
      s2 += red[t][2];
      s3 += red[t][3];
    }
    double* out = part + int64_t(blockIdx.x) * 2 * m;
    out[2 * threadIdx.x] = s0;
    out[2 * threadIdx.x + 1] = s1;
    out[m + 2 * threadIdx.x] = s2;
    out[m + 2 * threadIdx.x + 1] = s3;
  }
}

// shifts[l] = sigma + mean_c(qA_c / qM_c - theta_c) for lo <= l < top from the
// partial sums part[l][b][2m]; shifts[top] = sigma.  One workgroup.
__global__ void __launch_bounds__(256) k_offsets(int lo, int top, int m, int nblk, double sigma,
                                                 const double* __restrict__ part,
                                                 const double* __restrict__ theta,
                                                 double* __restrict__ shifts) {
  __shared__ double v[128];
  for (int l = lo; l < top; ++l) {
    const double* p = part + int64_t(l) * nblk * 2 * m;
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
      double qa = 0, qm = 0;
      for (int b = 0; b < nblk; ++b) {
        qa += p[int64_t(b) * 2 * m + c];
        qm += p[int64_t(b) * 2 * m + m + c];
      }
      v[c] = qa / qm - theta[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0;
      for (int c = 0; c < m; ++c) s += v[c];
      shifts[l] = sigma + s / m;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) shifts[top] = sigma;
}

// rq[c] = qA_c / qM_c and rq[m + c] = 1 / sqrt(qM_c) from the partial sums
// part[b][2m] (zero columns: both 0).  One workgroup; blocks added in order.
__global__ void __launch_bounds__(256) k_rq_final(int m, int nblk, const double* __restrict__ part,
                                                  double* __restrict__ rq) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    double qa = 0, qm = 0;
    for (int b = 0; b < nblk; ++b) {
      qa += part[int64_t(b) * 2 * m + c];
      qm += part[int64_t(b) * 2 * m + m + c];
    }
    rq[c] = qm > 0 ? qa / qm : 0.0;
    rq[m + c] = qm > 0 ? 1.0 / sqrt(qm) : 0.0;
  }
}

// U[i][c] *= scale[c]
__global__ void __launch_bounds__(256) k_scale_cols(int64_t n, int m, double* __restrict__ U,
                                                    const double* __restrict__ scale) {
  const int64_t total = n * m;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x)
    U[e] *= scale[e % m];
}

}  // namespace

int launch_rq_normalise(const DevLevel& L, double* U, int m, double* part, double* rq, hipStream_t s) {
  if (m % 2 != 0 || m < 2 || m > 512) {
    set_error("Rayleigh quotients: m = %d must be even and at most 512", m);
    return BMG_EINVAL;
  }
  const int nblk = kRqBlocks;
  if (L.W == 7)
    k_rq_part<7><<<nblk, 256, 0, s>>>(L.n, L.W, m, L.cols, L.a64, L.m64, U, part, InjChain{});
  else
    k_rq_part<0><<<nblk, 256, 0, s>>>(L.n, L.W, m, L.cols, L.a64, L.m64, U, part, InjChain{});
  k_rq_final<<<1, 256, 0, s>>>(m, nblk, part, rq);
  const int64_t total = L.n * m;
  k_scale_cols<<<int(std::min<int64_t>((total + 255) / 256, 4096)), 256, 0, s>>>(L.n, m, U, rq + m);
  return check_launch_c();
}

int spec_slices(int n) {
  const int tiles = (n + kTile - 1) / kTile;
  int S = (1024 + tiles - 1) / tiles;
  if (S < 1) S = 1;
  if (S > 16) S = 16;
  return S;
}

template <typename T>
int launch_spec_apply(int n, const T* phi, const T* g, const T* f, T* t, T* part, T* e, int m,
                      hipStream_t s) {
  if (m % 4 != 0 || m < 4 || m > 4 * kMaxQ) {
    set_error("spectral coarse solve: m = %d must be a multiple of 4 in [4, %d]", m, 4 * kMaxQ);
    return BMG_EINVAL;
  }
  const int S = spec_slices(n);
  int kc = (n + S - 1) / S;
  kc = (kc + kKc - 1) / kKc * kKc;
  const int S_used = (n + kc - 1) / kc;
  const dim3 grid((n + kTile - 1) / kTile, S_used);
  BMG_LAUNCH((k_dense_slices<T, false>), grid, 256, 0, s, n, m, kc, phi, f, part);
  BMG_LAUNCH((k_slices_sum<T>), grid_for(int64_t(n) * m), 256, 0, s, n, m, S_used, part, g, t);
  BMG_LAUNCH((k_dense_slices<T, true>), grid, 256, 0, s, n, m, kc, phi, t, part);
  BMG_LAUNCH((k_slices_sum<T>), grid_for(int64_t(n) * m), 256, 0, s, n, m, S_used, part,
             static_cast<const T*>(nullptr), e);
  return check_launch_c();
}

template <typename T>
int launch_spec_g(int n, const double* lam, const double* shift, double tau, T* g, hipStream_t s) {
  k_spec_g<T><<<grid_for(n), 256, 0, s>>>(n, lam, shift, tau, g);
  return check_launch_c();
}

template <typename T>
int launch_shift_dev(const DevLevel& L, const double* shift, T* S, hipStream_t s) {
  const int64_t cnt = L.n * L.W;
  const T* a = std::is_same<T, float>::value ? reinterpret_cast<const T*>(L.a32)
                                             : reinterpret_cast<const T*>(L.a64);
  const T* mm = std::is_same<T, float>::value ? reinterpret_cast<const T*>(L.m32)
                                              : reinterpret_cast<const T*>(L.m64);
  k_shift_dev<T><<<grid_for(cnt), 256, 0, s>>>(cnt, a, mm, shift, S);
  return check_launch_c();
}

int launch_gather_rows(int n, int m, const double* phi, const int* sel, double* blk, hipStream_t s) {
  k_gather_rows<<<grid_for(int64_t(n) * m), 256, 0, s>>>(n, m, phi, sel, blk);
  return check_launch_c();
}

int launch_offsets(const std::vector<DevLevel>& dev, int lo, int top, const double* U, int m,
                   double sigma, const double* theta, double* part, double* shifts, hipStream_t s) {
  const int nblk = kRqBlocks;
  if (m % 2 != 0 || m < 2 || m > 96) {
    set_error("adaptive shifts: m = %d must be even and at most 96", m);
    return BMG_EINVAL;
  }
  for (int l = lo; l < top; ++l) {
    const DevLevel& L = dev[l];
    double* p = part + int64_t(l) * nblk * 2 * m;
    InjChain inj{};
    for (int q = l + 1; q <= top; ++q) {
      if (dev[q].rself == nullptr) continue;
      if (inj.n == kInjMax) {
        set_error("adaptive shifts: more than %d stored-permuted levels above level %d", kInjMax, l);
        return BMG_EINVAL;
      }
      inj.rs[inj.n++] = dev[q].rself;
    }
    if (L.W == 7)
      k_rq_part<7><<<nblk, 256, 0, s>>>(L.n, L.W, m, L.cols, L.a64, L.m64, U, p, inj);
    else
      k_rq_part<0><<<nblk, 256, 0, s>>>(L.n, L.W, m, L.cols, L.a64, L.m64, U, p, inj);
  }
  k_offsets<<<1, 256, 0, s>>>(lo, top, m, nblk, sigma, part, theta, shifts);
  return check_launch_c();
}

#define BMG_INST_C(T)                                                                          \
  template int launch_spec_apply<T>(int, const T*, const T*, const T*, T*, T*, T*, int,      \
                                    hipStream_t);                                             \
  template int launch_spec_g<T>(int, const double*, const double*, double, T*, hipStream_t); \
  template int launch_shift_dev<T>(const DevLevel&, const double*, T*, hipStream_t);
BMG_INST_C(double)
BMG_INST_C(float)
#undef BMG_INST_C

}  // namespace bmg
