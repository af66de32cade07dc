// extern "C" entry points of libbmg (declared in include/bmg.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "bmg_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

namespace bmg {

namespace {
thread_local std::string g_err;
}

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* get_error() { return g_err.c_str(); }

int solve(bmg_hierarchy* h, int k, double sigma, double tol, const bmg_solve_opts* opts,
          double* evals, double* evecs, int64_t ld, int evecs_on_device, void* stream,
          bmg_solve_stats* stats);
int apply_vcycle(bmg_hierarchy* h, int level, int dtype, int m, double sigma, int smoother,
                 int nu1, int nu2, int l_c, double omega, const void* x, void* y, hipStream_t s);

}  // namespace bmg

namespace bmg {
namespace {
// Runs fn(S) with a temporary S = A_l - sigma M_l of the requested precision.
template <typename F>
int with_shift(const DevLevel& D, double sigma, bool f32, hipStream_t s, F&& fn) {
  const size_t bytes = (f32 ? sizeof(float) : sizeof(double)) * D.n * D.W;
  void* S = nullptr;
  BMG_HIP(hipMalloc(&S, bytes));
  int st = f32 ? launch_shift<float>(D, sigma, static_cast<float*>(S), s)
               : launch_shift<double>(D, sigma, static_cast<double*>(S), s);
  if (st == BMG_OK) st = fn(static_cast<const void*>(S));
  (void)hipStreamSynchronize(s);
  dev_free(S);
  return st;
}
}  // namespace
}  // namespace bmg

using namespace bmg;

extern "C" {

const char* bmg_status_string(int status) {
  switch (status) {
    case BMG_OK: return "ok";
    case BMG_EINVAL: return "invalid argument";
    case BMG_ENOMEM: return "out of device memory";
    case BMG_EDEVICE: return "HIP device error";
    case BMG_ENOCONV: return "not converged";
    case BMG_EBUSY: return "busy";
    case BMG_ECANCELED: return "canceled";
    default: return "unknown status";
  }
}

const char* bmg_last_error(void) { return get_error(); }

void bmg_solve_opts_default(bmg_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m = 0;
  o->nu1 = 2;
  o->nu2 = 2;
  o->smoother = BMG_SMOOTH_GS;
  o->precision = BMG_FP64;
  o->max_cycles = 200;
  o->n_c = 0;
  o->l_c = -1;
  o->omega = 0.85;
  o->angle_tol = 1e-7;
  o->seed = 0;
  o->initial_block = nullptr;
  o->timed_kernel = -1;
  o->scheme = BMG_SCHEME_AUTO;
  o->ramp_cycles = 0;
  o->ramp_level = -1;
}

static int build_impl(const bmg_surface_desc* desc, int32_t n_refine, void* stream,
                      bmg_hierarchy** out, bool to_device) {
  BMG_CHECK(out != nullptr, "out must be non-NULL");
  *out = nullptr;
  TraceRange trace("bmg_build_hierarchy");
  bmg_hierarchy* h = new (std::nothrow) bmg_hierarchy();
  if (!h) return BMG_ENOMEM;
  if (desc) h->kind = desc->kind;
  int st = build_host_levels(desc, n_refine, h->host);
  for (size_t l = 0; st == BMG_OK && l < h->host.size(); ++l)
    st = assemble_level(h->host[l], l ? &h->host[l - 1] : nullptr);
  if (st == BMG_OK && to_device) {
    // works whether or not another runtime user initialised the device first
    int count = 0;
    hipError_t e = hipInit(0);
    if (e == hipSuccess) e = hipGetDeviceCount(&count);
    if (e == hipSuccess && count < 1) e = hipErrorNoDevice;
    if (e == hipSuccess) e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = hipSetDevice(h->device);
    if (e != hipSuccess) {
      set_error("no usable HIP device: %s", hipGetErrorString(e));
      st = BMG_EDEVICE;
    }
  }
  if (st == BMG_OK) {
    // Alg. 2 step 1: all eigenpairs of the level-0 pencil.  Up to
    // kHostEigMax vertices on the host (Jacobi); larger coarse meshes (the
    // torus grid) on the device with rocSOLVER, so only a device build takes them.
    const HostLevel& L0 = h->host[0];
    const int n0 = int(L0.n);
    if (n0 > kDeviceEigMax || (n0 > kHostEigMax && !to_device)) {
      set_error("coarse mesh has %d vertices; the setup eigensolver accepts at most %d (%d for a "
                "host-only build)", n0, kDeviceEigMax, kHostEigMax);
      st = BMG_EINVAL;
    } else {
      std::vector<double> A(size_t(n0) * n0, 0.0), M(size_t(n0) * n0, 0.0);
      for (int i = 0; i < n0; ++i)
        for (int k = 0; k < L0.W; ++k) {
          const int j = L0.cols[size_t(i) * L0.W + k];
          A[size_t(i) * n0 + j] += L0.a[size_t(i) * L0.W + k];
          M[size_t(i) * n0 + j] += L0.mm[size_t(i) * L0.W + k];
        }
      h->n0 = n0;
      st = n0 > kHostEigMax ? device_sygv(n0, A, M, h->lam0, h->phi0, static_cast<hipStream_t>(stream))
                            : dense_sygv(n0, A, M, h->lam0, h->phi0);
    }
  }
  if (st == BMG_OK && to_device) st = upload_hierarchy(h, static_cast<hipStream_t>(stream));
  if (st != BMG_OK) {
    free_device(h);
    delete h;
    return st;
  }
  *out = h;
  return BMG_OK;
}

int bmg_build_hierarchy(const bmg_surface_desc* desc, int32_t n_refine, void* stream,
                        bmg_hierarchy** out) {
  return build_impl(desc, n_refine, stream, out, true);
}

int bmg_build_hierarchy_host(const bmg_surface_desc* desc, int32_t n_refine, bmg_hierarchy** out) {
  return build_impl(desc, n_refine, nullptr, out, false);
}

void bmg_free_hierarchy(bmg_hierarchy* h) {
  if (!h) return;
  bmg::DeviceSyncGuard sync;
  if (!h->dev.empty()) (void)hipDeviceSynchronize();
  free_workspaces(h);
  free_device(h);
  delete h;
}

int bmg_hierarchy_info(const bmg_hierarchy* h, int32_t level, bmg_level_info* out) {
  BMG_CHECK(h && out, "NULL argument");
  BMG_CHECK(level >= 0 && level < int(h->host.size()), "level %d out of range", level);
  const HostLevel& H = h->host[level];
  out->n_levels = int32_t(h->host.size());
  out->level = level;
  out->n_vert = H.n;
  out->n_tri = H.n_tri;
  out->nnz = H.nnz;
  out->ell_width = H.W;
  out->n_colours = H.n_colours;
  out->area = H.area;
  out->device_bytes = level < int(h->dev.size()) ? h->dev[level].bytes : 0;
  return BMG_OK;
}

int bmg_hierarchy_export(const bmg_hierarchy* h, int32_t level, int32_t what, void* host_out,
                         int64_t capacity, int64_t* bytes_needed) {
  BMG_CHECK(h != nullptr, "NULL hierarchy");
  BMG_CHECK(level >= 0 && level < int(h->host.size()), "level %d out of range", level);
  const HostLevel& H = h->host[level];
  const void* src = nullptr;
  int64_t bytes = 0;
  std::vector<double> tmp;
  switch (what) {
    case BMG_EXPORT_XYZ: src = H.xyz.data(); bytes = 8 * int64_t(H.xyz.size()); break;
    case BMG_EXPORT_TRI: src = H.tri.data(); bytes = 4 * int64_t(H.tri.size()); break;
    case BMG_EXPORT_PARENTS: src = H.parents.data(); bytes = 4 * int64_t(H.parents.size()); break;
    case BMG_EXPORT_ELL_COLS: src = H.cols.data(); bytes = 4 * int64_t(H.cols.size()); break;
    case BMG_EXPORT_ELL_A: src = H.a.data(); bytes = 8 * int64_t(H.a.size()); break;
    case BMG_EXPORT_ELL_M: src = H.mm.data(); bytes = 8 * int64_t(H.mm.size()); break;
    case BMG_EXPORT_COLOURS: src = H.colour.data(); bytes = 4 * int64_t(H.colour.size()); break;
    case BMG_EXPORT_LUMPED: src = H.lumped.data(); bytes = 8 * int64_t(H.lumped.size()); break;
    case BMG_EXPORT_COLOURS2: src = H.colour2.data(); bytes = 4 * int64_t(H.colour2.size()); break;
    case BMG_EXPORT_COARSE_EIG:
      BMG_CHECK(level == 0, "the coarse eigendecomposition exists on level 0 only");
      tmp = h->lam0;
      tmp.insert(tmp.end(), h->phi0.begin(), h->phi0.end());
      src = tmp.data();
      bytes = 8 * int64_t(tmp.size());
      break;
    default: BMG_CHECK(false, "unknown export item %d", what);
  }
  if (bytes_needed) *bytes_needed = bytes;
  BMG_CHECK(host_out != nullptr || bytes == 0, "host_out is NULL");
  BMG_CHECK(capacity >= bytes, "capacity %lld < %lld bytes", (long long)capacity, (long long)bytes);
  if (bytes) std::memcpy(host_out, src, size_t(bytes));
  return BMG_OK;
}

int bmg_solve(bmg_hierarchy* h, int32_t k, double sigma, double tol, const bmg_solve_opts* opts,
              double* evals, double* evecs, int64_t ld, int32_t evecs_on_device, void* stream,
              bmg_solve_stats* stats) {
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy has no device data");
  return bmg::solve(h, k, sigma, tol, opts, evals, evecs, ld, evecs_on_device, stream, stats);
}

int bmg_solve_group(bmg_hierarchy* h, double sigma, int32_t n, bmg_group_request* reqs, const void* hip_stream) {
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy has no device data");
  return bmg::solve_group(h, sigma, n, reqs, const_cast<void*>(hip_stream));
}

int bmg_estimate(bmg_hierarchy* h, int32_t level, int32_t k, const double* evals, const double* evecs,
                 int64_t ld, double* eta, double* parts, double* eta2_T, void* stream) {
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy has no device data");
  return bmg::estimate(h, level, k, evals, evecs, ld, eta, parts, eta2_T, static_cast<hipStream_t>(stream));
}

int bmg_two_grid(bmg_hierarchy* h, int32_t level_H, int32_t n, const int32_t* idx, int32_t top,
                 int32_t nu, double* evals, double* evecs, void* stream) {
  BMG_CHECK(h != nullptr && !h->dev.empty(), "hierarchy has no device data");
  return bmg::two_grid(h, level_H, n, idx, top, nu, evals, evecs, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

using namespace bmg;

// One operator on row blocks in the levels' storage order.
int apply_stored(bmg_hierarchy* h, const bmg_apply_args* a, const void* x, const void* f, void* y,
                 hipStream_t s) {
  const int l = a->level;
  const int m = a->m;
  const DevLevel& D = h->dev[l];
  const bool f32 = a->dtype == 1;
  auto need_m = [&](int mult) -> int {
    BMG_CHECK(m >= mult && m % mult == 0 && m <= 4096, "m = %d must be a positive multiple of %d", m, mult);
    return BMG_OK;
  };
  switch (a->op) {
    case BMG_OP_A:
    case BMG_OP_M: {
      BMG_TRY(need_m(2));
      BMG_CHECK(x != nullptr && !f32, "A/M products take FP64 x");
      // y = A x or M x: run the fused kernel with a scratch second output
      double* other = nullptr;
      BMG_HIP(hipMalloc(&other, sizeof(double) * D.n * m));
      int st = a->op == BMG_OP_A ? launch_spmm_am(D, (const double*)x, (double*)y, other, m, s)
                                 : launch_spmm_am(D, (const double*)x, other, (double*)y, m, s);
      (void)hipStreamSynchronize(s);
      dev_free(other);
      return st;
    }
    case BMG_OP_SHIFTED:
    case BMG_OP_RESIDUAL: {
      BMG_TRY(need_m(4));
      BMG_CHECK(x != nullptr && (a->op == BMG_OP_SHIFTED || f != nullptr), "x (and f) required");
      const int mode = a->op == BMG_OP_SHIFTED ? ROW_SHIFTED : ROW_RESIDUAL;
      return with_shift(D, a->sigma, f32, s, [&](const void* S) {
        return f32 ? launch_shifted<float>(D, (const float*)S, mode, (const float*)x, (const float*)f,
                                           (float*)y, m, s)
                   : launch_shifted<double>(D, (const double*)S, mode, (const double*)x,
                                            (const double*)f, (double*)y, m, s);
      });
    }
    case BMG_OP_SMOOTH_FWD:
    case BMG_OP_SMOOTH_BWD: {
      BMG_TRY(need_m(4));
      BMG_CHECK(f != nullptr, "f required");
      const bool fwd = a->op == BMG_OP_SMOOTH_FWD;
      if (a->smoother == BMG_SMOOTH_JACOBI) {
        BMG_CHECK(x != nullptr && x != y, "Jacobi needs x (input) distinct from y (output)");
        BMG_CHECK(a->omega > 0 && a->omega < 2, "omega must be in (0, 2)");
        return with_shift(D, a->sigma, f32, s, [&](const void* S) {
          return f32 ? launch_jacobi<float>(D, (const float*)S, a->omega, (const float*)x,
                                            (const float*)f, (float*)y, false, m, s)
                     : launch_jacobi<double>(D, (const double*)S, a->omega, (const double*)x,
                                             (const double*)f, (double*)y, false, m, s);
        });
      }
      if (a->smoother == BMG_SMOOTH_KACZMARZ) {
        return with_shift(D, a->sigma, f32, s, [&](const void* S) -> int {
          for (int k = 0; k < D.n_colours2; ++k) {
            const int c = fwd ? k : D.n_colours2 - 1 - k;
            if (f32)
              BMG_TRY(launch_kaczmarz_colour<float>(D, (const float*)S, c, (float*)y, (const float*)f, m, s));
            else
              BMG_TRY(launch_kaczmarz_colour<double>(D, (const double*)S, c, (double*)y, (const double*)f, m, s));
          }
          return BMG_OK;
        });
      }
      BMG_CHECK(a->smoother == BMG_SMOOTH_GS, "unknown smoother");
      return with_shift(D, a->sigma, f32, s, [&](const void* S) -> int {
        for (int k = 0; k < D.n_colours; ++k) {
          const int c = fwd ? k : D.n_colours - 1 - k;
          if (f32)
            BMG_TRY(launch_gs_colour<float>(D, (const float*)S, c, (float*)y, (const float*)f, m, s));
          else
            BMG_TRY(launch_gs_colour<double>(D, (const double*)S, c, (double*)y, (const double*)f, m, s));
        }
        return BMG_OK;
      });
    }
    case BMG_OP_RESTRICT:
    case BMG_OP_PROLONG_ADD: {
      BMG_TRY(need_m(4));
      BMG_CHECK(l >= 1, "transfers need level >= 1");
      BMG_CHECK(x != nullptr, "x required");
      if (a->op == BMG_OP_RESTRICT)
        return f32 ? launch_restrict<float>(D, (const float*)x, (float*)y, m, s)
                   : launch_restrict<double>(D, (const double*)x, (double*)y, m, s);
      return f32 ? launch_prolong_add<float>(D, (const float*)x, (float*)y, m, s)
                 : launch_prolong_add<double>(D, (const double*)x, (double*)y, m, s);
    }
    case BMG_OP_VCYCLE: {
      BMG_TRY(need_m(4));
      BMG_CHECK(x != nullptr, "x required");
      BMG_CHECK(a->smoother == BMG_SMOOTH_GS || a->smoother == BMG_SMOOTH_JACOBI ||
                    a->smoother == BMG_SMOOTH_KACZMARZ,
                "unknown smoother");
      BMG_CHECK(a->nu1 >= 0 && a->nu2 >= 0 && a->nu1 <= 64 && a->nu2 <= 64, "nu out of range");
      BMG_CHECK(a->omega > 0 && a->omega < 2, "omega must be in (0, 2)");
      return apply_vcycle(h, l, a->dtype, m, a->sigma, a->smoother, a->nu1, a->nu2, a->l_c,
                          a->omega, x, y, s);
    }
    case BMG_OP_GAUSSIAN:
      BMG_CHECK(m >= 1 && m <= 4096, "m out of range");
      return launch_gaussian((double*)y, D.n, m, a->seed, s);
    case BMG_OP_GRAM: {
      BMG_CHECK(x && f && !f32, "GRAM takes FP64 x and f");
      BMG_CHECK(m >= 1 && m <= 96 && a->m2 >= 1 && a->m2 <= 192, "GRAM needs m <= 96, m2 <= 192");
      GramPlan p = gram_plan(D.n, m, a->m2);
      double* part = nullptr;
      BMG_HIP(hipMalloc(&part, sizeof(double) * p.nblk * p.per_block));
      int st = launch_gram(p, D.n, (const double*)x, m, nullptr, 0, (const double*)f, a->m2, nullptr,
                           0, part, (double*)y, s);
      (void)hipStreamSynchronize(s);
      dev_free(part);
      return st;
    }
    case BMG_OP_SYEV: {
      BMG_CHECK(x != nullptr && !f32, "SYEV takes an FP64 matrix");
      BMG_CHECK(m >= 1 && m <= 96, "SYEV needs 1 <= m <= 96");
      int* st_d = nullptr;
      BMG_HIP(hipMalloc(&st_d, sizeof(int)));
      double* w = (double*)y;
      int st = launch_syev(m, (const double*)x, w, w + m, st_d, s);
      int hs = 0;
      (void)hipMemcpyAsync(&hs, st_d, sizeof(int), hipMemcpyDeviceToHost, s);
      (void)hipStreamSynchronize(s);
      dev_free(st_d);
      if (st == BMG_OK && hs != 0) {
        set_error("Jacobi sweep limit reached");
        return BMG_ENOCONV;
      }
      return st;
    }
    case BMG_OP_EIGRES: {
      BMG_TRY(need_m(4));
      BMG_CHECK(x && f, "EIGRES needs x and f (theta)");
      return f32 ? launch_eigres<float>(D, (const double*)x, (const double*)f, 1.0, (float*)y, nullptr, eigres_blocks(D, m), m, s)
                 : launch_eigres<double>(D, (const double*)x, (const double*)f, 1.0, (double*)y, nullptr, eigres_blocks(D, m), m, s);
    }
    case BMG_OP_GRAM_AM: {
      BMG_CHECK(f && !f32, "GRAM_AM takes FP64 blocks");
      BMG_CHECK(m >= 2 && m % 2 == 0 && a->m2 >= 0 && a->m2 + m <= 96 && 2 * m <= 192 &&
                    (a->m2 == 0 || x != nullptr),
                "GRAM_AM needs even m, 0 <= m2, m2 + m <= 96, and x when m2 > 0");
      GramPlan p = gram_plan(D.n, a->m2 + m, 2 * m);
      double* part = nullptr;
      BMG_HIP(hipMalloc(&part, sizeof(double) * p.nblk * p.per_block));
      int st = launch_gram_am(p, D, (const double*)x, a->m2, (const double*)f, m, part, (double*)y, s);
      (void)hipStreamSynchronize(s);
      dev_free(part);
      return st;
    }
    case BMG_OP_UPDATE: {
      BMG_CHECK(f && !f32, "UPDATE takes FP64 blocks and an FP64 Y in f");
      BMG_CHECK(m >= 4 && m % 4 == 0 && m <= 96, "UPDATE needs m a multiple of 4 in [4, 96]");
      BMG_CHECK(a->m2 >= 0 && a->m2 + m <= 96 && (a->m2 == 0 || x != nullptr),
                "UPDATE needs 0 <= m2, m2 + m <= 96 and x when m2 > 0");
      return launch_update_zy(D.n, (const double*)x, a->m2, (const double*)y, m, (const double*)f,
                              (double*)y, m, s);
    }
    case BMG_OP_COARSE_SOLVE: {
      BMG_CHECK(x != nullptr, "x required");
      BMG_CHECK(m >= 4 && m % 4 == 0 && m <= 96, "COARSE_SOLVE needs m a multiple of 4 in [4, 96]");
      BMG_CHECK(std::isfinite(a->sigma), "sigma must be finite");
      const LevelEig* e = nullptr;
      BMG_TRY(level_eig(h, l, s, &e));
      const int n = e->n;
      const size_t vb = f32 ? sizeof(float) : sizeof(double);
      void *g = nullptr, *t = nullptr, *part = nullptr;
      double* sh = nullptr;
      int st = BMG_OK;
      if (hipMalloc(&g, vb * n) != hipSuccess || hipMalloc(&t, vb * n * m) != hipSuccess ||
          hipMalloc(&part, vb * n * m * spec_slices(n)) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&sh), sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc failed");
        st = BMG_ENOMEM;
      }
      const double tau = 1e-2 * std::max(1.0, std::fabs(a->sigma));
      if (st == BMG_OK && hipMemcpyAsync(sh, &a->sigma, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("copy failed");
        st = BMG_EDEVICE;
      }
      if (st == BMG_OK)
        st = f32 ? launch_spec_g<float>(n, e->d_lam, sh, tau, (float*)g, s)
                 : launch_spec_g<double>(n, e->d_lam, sh, tau, (double*)g, s);
      if (st == BMG_OK)
        st = f32 ? launch_spec_apply<float>(n, e->d_phi32, (const float*)g, (const float*)x, (float*)t,
                                            (float*)part, (float*)y, m, s)
                 : launch_spec_apply<double>(n, e->d_phi64, (const double*)g, (const double*)x,
                                             (double*)t, (double*)part, (double*)y, m, s);
      (void)hipStreamSynchronize(s);
      for (void* p : {g, t, part, (void*)sh})
        if (p) dev_free(p);
      return st;
    }
    case BMG_OP_SHIFT_OFFSETS: {
      BMG_CHECK(x && f && !f32, "SHIFT_OFFSETS takes an FP64 block x and FP64 theta in f");
      BMG_CHECK(m >= 2 && m % 2 == 0 && m <= 96, "SHIFT_OFFSETS needs even m in [2, 96]");
      BMG_CHECK(a->l_c >= 0 && a->l_c <= l, "SHIFT_OFFSETS needs 0 <= l_c <= level");
      double* part = nullptr;
      BMG_HIP(hipMalloc(&part, sizeof(double) * (l + 1) * kRqBlocks * 2 * m));
      int st = launch_offsets(h->dev, a->l_c, l, (const double*)x, m, a->sigma, (const double*)f, part,
                              (double*)y, s);
      (void)hipStreamSynchronize(s);
      dev_free(part);
      return st;
    }
    default:
      BMG_CHECK(false, "unknown op %d", a->op);
  }
}

// The row blocks an operator reads or writes: which argument (0 x, 1 f, 2 y),
// the level (0: the op's level, -1: the one below), direction, columns, and
// whether the block is FP64 whatever the op's precision.
struct RowBlock {
  int arg, dl;
  bool in, out;
  int cols;
  bool f64;
};

std::vector<RowBlock> row_blocks(const bmg_apply_args* a, const void* x) {
  const int m = a->m;
  switch (a->op) {
    case BMG_OP_A:
    case BMG_OP_M: return {{0, 0, true, false, m, true}, {2, 0, false, true, m, true}};
    case BMG_OP_SHIFTED: return {{0, 0, true, false, m, false}, {2, 0, false, true, m, false}};
    case BMG_OP_RESIDUAL:
      return {{0, 0, true, false, m, false}, {1, 0, true, false, m, false}, {2, 0, false, true, m, false}};
    case BMG_OP_SMOOTH_FWD:
    case BMG_OP_SMOOTH_BWD: {
      std::vector<RowBlock> b{{1, 0, true, false, m, false}, {2, 0, true, true, m, false}};
      if (x) b.push_back({0, 0, true, false, m, false});
      return b;
    }
    case BMG_OP_RESTRICT: return {{0, 0, true, false, m, false}, {2, -1, false, true, m, false}};
    case BMG_OP_PROLONG_ADD: return {{0, -1, true, false, m, false}, {2, 0, true, true, m, false}};
    case BMG_OP_VCYCLE: return {{0, 0, true, false, m, false}, {2, 0, false, true, m, false}};
    case BMG_OP_EIGRES: return {{0, 0, true, false, m, true}, {2, 0, false, true, m, false}};
    case BMG_OP_GRAM_AM: {
      std::vector<RowBlock> b{{1, 0, true, false, m, true}};
      if (x) b.push_back({0, 0, true, false, a->m2, true});
      return b;
    }
    case BMG_OP_SHIFT_OFFSETS: return {{0, 0, true, false, m, true}};
    default: return {};  // no row blocks, or row-local / order-free ops (Gaussian in vertex order, Gram, update)
  }
}

}  // namespace

extern "C" {

int bmg_apply(const bmg_hierarchy* hc, const bmg_apply_args* a, const void* x, const void* f,
              void* y, void* stream) {
  using namespace bmg;
  BMG_CHECK(hc && a, "NULL argument");
  bmg_hierarchy* h = const_cast<bmg_hierarchy*>(hc);
  BMG_CHECK(!h->dev.empty(), "hierarchy has no device data");
  const int nl = int(h->dev.size());
  const int l = a->level;
  BMG_CHECK(l >= 0 && l < nl, "level %d out of range", l);
  BMG_CHECK(a->dtype == 0 || a->dtype == 1, "dtype must be 0 (FP64) or 1 (FP32)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  BMG_CHECK(y != nullptr, "y must be non-NULL");
  BMG_HIP(hipSetDevice(h->device));
  // Blocks cross this boundary in vertex order; a level stored in another
  // order gets its blocks permuted into temporaries and back.
  std::vector<RowBlock> blocks = row_blocks(a, x);
  bool permuted = false;
  for (const RowBlock& b : blocks) {
    const int lv = l + b.dl;
    if (lv >= 0 && h->dev[lv].perm != nullptr) permuted = true;
  }
  if (!permuted) return apply_stored(h, a, x, f, y, s);
  BMG_CHECK(a->m >= 1 && a->m <= 4096 && a->m2 >= 0 && a->m2 <= 4096, "m out of range");
  const void* args[3] = {x, f, y};
  void* tmp[3] = {nullptr, nullptr, nullptr};
  int st = BMG_OK;
  auto permute = [&](const RowBlock& b, const int* map, const void* src, void* dst) -> int {
    const int64_t n = h->dev[l + b.dl].n;
    if (b.f64 || a->dtype == 0)
      return launch_permute_rows<double>(n, b.cols, map, static_cast<const double*>(src), static_cast<double*>(dst), s);
    return launch_permute_rows<float>(n, b.cols, map, static_cast<const float*>(src), static_cast<float*>(dst), s);
  };
  for (const RowBlock& b : blocks) {
    if (l + b.dl < 0) continue;
    const DevLevel& D = h->dev[l + b.dl];
    if (D.perm == nullptr || args[b.arg] == nullptr) continue;
    const size_t eb = (b.f64 || a->dtype == 0) ? sizeof(double) : sizeof(float);
    if (hipMalloc(&tmp[b.arg], eb * size_t(D.n) * b.cols) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of a storage-order temporary failed");
      st = BMG_ENOMEM;
      break;
    }
    if (b.in && (st = permute(b, D.perm, args[b.arg], tmp[b.arg])) != BMG_OK) break;  // storage row r <- vertex perm[r]
  }
  if (st == BMG_OK)
    st = apply_stored(h, a, tmp[0] ? tmp[0] : x, tmp[1] ? tmp[1] : f, tmp[2] ? tmp[2] : y, s);
  if (st == BMG_OK)
    for (const RowBlock& b : blocks) {
      if (l + b.dl < 0) continue;
      const DevLevel& D = h->dev[l + b.dl];
      if (!b.out || tmp[b.arg] == nullptr) continue;
      if ((st = permute(b, D.iperm, tmp[b.arg], y)) != BMG_OK) break;  // vertex i <- storage row iperm[i]
    }
  (void)hipStreamSynchronize(s);
  for (void* p : tmp)
    if (p) dev_free(p);
  return st;
}

}  // extern "C"
