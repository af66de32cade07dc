// Two-grid eigensolver with a spectral shift (Alg. 1), applied in a cascade
// between neighbouring levels (Remark 3.1), with the fine source problem of
// eq. (pb-f-s) approximated by Kaczmarz relaxation (Sec. 5.3; the remark after
// Alg. 1 allows a smoother started from the previous level's approximation in
// place of a direct solve).
//
// For each followed pair c, level k takes u = P u_{k-1}, the right-hand side
// M_k u and nu multicolour Kaczmarz sweeps (alternating directions, forward
// first) on (A_k - theta_c M_k) x = M_k u from x = u, where theta_c is the
// pair's eigenvalue approximation on level k - 1 (on level_H: the coarse
// eigenvalue; Alg. 1's fixed shift mu cancels, since the fine problem uses
// mu + lambda_H).  The new approximation is the Rayleigh quotient of x, and x
// scaled to unit M-norm is passed on.  All columns run at once, each with its
// own shift.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bmg_internal.h"

namespace bmg {

int two_grid(bmg_hierarchy* h, int level_H, int n, const int32_t* idx, int top, int nu, double* evals,
             double* evecs, hipStream_t s) {
  TraceRange trace("bmg_two_grid");
  const int nl = int(h->dev.size());
  BMG_CHECK(level_H >= 0 && level_H < nl, "level_H = %d out of range", level_H);
  if (top < 0) top = nl - 1;
  BMG_CHECK(top >= level_H && top < nl, "top = %d must be in [level_H, %d]", top, nl - 1);
  BMG_CHECK(n >= 1 && n <= 512, "n = %d must be in [1, 512]", n);
  BMG_CHECK(nu >= 0 && nu <= 64, "nu = %d must be in [0, 64]", nu);
  BMG_CHECK(idx != nullptr && evals != nullptr, "idx and evals must be non-NULL");
  const int64_t nH = h->host[level_H].n;
  BMG_CHECK(nH <= kLevelEigMax, "level_H has %lld vertices; the coarse eigensolve takes at most %d",
            (long long)nH, kLevelEigMax);
  for (int c = 0; c < n; ++c)
    BMG_CHECK(idx[c] >= 0 && idx[c] < nH, "idx[%d] = %d outside the %lld coarse pairs", c, idx[c],
              (long long)nH);
  BMG_HIP(hipSetDevice(h->device));
  const LevelEig* le = nullptr;
  BMG_TRY(level_eig(h, level_H, s, &le));
  const int m = (n + 1) & ~1;  // even: the kernels take two columns per thread
  const int64_t N = h->dev[top].n;
  std::vector<void*> bufs;
  auto alloc = [&](double** p, size_t count) -> int {
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of %zu bytes failed", count * sizeof(double));
      return BMG_ENOMEM;
    }
    bufs.push_back(*p);
    return BMG_OK;
  };
  auto run = [&]() -> int {
    double *U = nullptr, *X = nullptr, *F = nullptr, *AX = nullptr, *shifts = nullptr, *part = nullptr,
           *rq = nullptr;
    int* sel = nullptr;
    BMG_TRY(alloc(&U, size_t(N) * m));
    BMG_TRY(alloc(&X, size_t(N) * m));
    BMG_TRY(alloc(&F, size_t(N) * m));
    BMG_TRY(alloc(&AX, size_t(N) * m));
    BMG_TRY(alloc(&shifts, size_t(m)));
    BMG_TRY(alloc(&part, size_t(kRqBlocks) * 2 * m));
    BMG_TRY(alloc(&rq, size_t(2 * m)));
    BMG_TRY(alloc(reinterpret_cast<double**>(&sel), size_t(m)));  // m ints fit m doubles
    // coarse pairs: rows of the level's eigenvector table; a padding column is zero
    std::vector<int> selh(m, 0);
    std::vector<double> theta(m, 0.0);
    for (int c = 0; c < n; ++c) {
      selh[c] = idx[c];
      theta[c] = le->lam[size_t(idx[c])];
    }
    BMG_HIP(hipMemcpyAsync(sel, selh.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
    BMG_TRY(launch_gather_rows(int(nH), m, le->d_phi64, sel, U, s));
    if (m > n) {
      // zero the padding column: gather wrote eigenvector idx[0] there
      std::vector<double> zero(size_t(nH), 0.0);
      BMG_HIP(hipMemcpy2DAsync(U + (m - 1), sizeof(double) * m, zero.data(), sizeof(double), sizeof(double),
                               size_t(nH), hipMemcpyHostToDevice, s));
      BMG_HIP(hipStreamSynchronize(s));
    }
    for (int c = 0; c < n; ++c) evals[size_t(level_H) * n + c] = theta[c];
    for (int k = level_H + 1; k <= top; ++k) {
      const DevLevel& D = h->dev[k];
      BMG_TRY(launch_fill<double>(X, D.n * m, 0.0, s));
      BMG_TRY(launch_prolong_add<double>(D, U, X, m, s));  // X = P u
      BMG_TRY(launch_spmm_am(D, X, AX, F, m, s));           // F = M P u
      BMG_HIP(hipMemcpyAsync(shifts, theta.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
      for (int sw = 0; sw < nu; ++sw) {
        const bool fwd = sw % 2 == 0;
        for (int q = 0; q < D.n_colours2; ++q)
          BMG_TRY(launch_kaczmarz_shifts_colour(D, fwd ? q : D.n_colours2 - 1 - q, shifts, X, F, m, s));
      }
      BMG_TRY(launch_rq_normalise(D, X, m, part, rq, s));
      BMG_HIP(hipMemcpyAsync(theta.data(), rq, sizeof(double) * m, hipMemcpyDeviceToHost, s));
      BMG_HIP(hipStreamSynchronize(s));  // theta feeds the next level's shifts
      for (int c = 0; c < n; ++c) evals[size_t(k) * n + c] = theta[c];
      std::swap(U, X);
    }
    if (evecs) {
      // column-major [n][N]: column c = pair c
      std::vector<double> hb(size_t(N) * m);
      BMG_HIP(hipMemcpyAsync(hb.data(), U, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
      BMG_HIP(hipStreamSynchronize(s));
      // storage row r of the top level is vertex perm[r]
      const std::vector<int32_t>& perm = h->dev[top].perm_h;
      for (int c = 0; c < n; ++c)
        for (int64_t r = 0; r < N; ++r)
          evecs[size_t(c) * N + (perm.empty() ? r : perm[size_t(r)])] = hb[size_t(r) * m + c];
    }
    return BMG_OK;
  };
  const int st = run();
  (void)hipStreamSynchronize(s);
  for (void* p : bufs) dev_free(p);
  return st;
}

}  // namespace bmg
