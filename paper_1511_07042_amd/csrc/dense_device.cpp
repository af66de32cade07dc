// Setup-time generalized symmetric-definite eigensolver for coarse meshes too
// large for the host Jacobi solver (the 64 x 32 torus grid has 2048
// vertices): A_l x = lambda M_l x (Alg. 2 step 1) with rocSOLVER's dsygvd on
// the device.  It runs once per hierarchy and level, outside every cycle.  The library
// is opened on first use (dlopen), so processes whose coarse meshes are small
// never load it.
#include <dlfcn.h>

#include <cstring>
#include <mutex>

#include <rocsolver/rocsolver.h>

#include "bmg_internal.h"

namespace bmg {
namespace {

struct Solver {
  decltype(&rocblas_create_handle) create = nullptr;
  decltype(&rocblas_destroy_handle) destroy = nullptr;
  decltype(&rocblas_set_stream) set_stream = nullptr;
  decltype(&rocsolver_dsygvd) sygvd = nullptr;
  bool ok = false;
  std::string why;
};

void* open_lib(const char* const* names) {
  for (const char* const* n = names; *n; ++n)
    if (void* h = dlopen(*n, RTLD_NOW | RTLD_LOCAL)) return h;
  return nullptr;
}

const Solver& solver() {
  static Solver s;
  static std::once_flag once;
  std::call_once(once, [] {
    static const char* blas[] = {"librocblas.so", "librocblas.so.5", "/opt/rocm/lib/librocblas.so",
                                 nullptr};
    static const char* lapack[] = {"librocsolver.so", "librocsolver.so.0",
                                   "/opt/rocm/lib/librocsolver.so", nullptr};
    void* hb = open_lib(blas);
    void* hs = open_lib(lapack);
    if (!hb || !hs) {
      s.why = "rocBLAS / rocSOLVER not found";
      return;
    }
    s.create = reinterpret_cast<decltype(s.create)>(dlsym(hb, "rocblas_create_handle"));
    s.destroy = reinterpret_cast<decltype(s.destroy)>(dlsym(hb, "rocblas_destroy_handle"));
    s.set_stream = reinterpret_cast<decltype(s.set_stream)>(dlsym(hb, "rocblas_set_stream"));
    s.sygvd = reinterpret_cast<decltype(s.sygvd)>(dlsym(hs, "rocsolver_dsygvd"));
    s.ok = s.create && s.destroy && s.set_stream && s.sygvd;
    if (!s.ok) s.why = "rocBLAS / rocSOLVER entry points missing";
  });
  return s;
}

}  // namespace

// lam ascending [n]; *vecs (device, [n][n]) with row j the M-orthonormal
// eigenvector of lam[j] (rocSOLVER's column-major result read row by row).
// A and M are dense row-major (symmetric).
int device_sygv_keep(int n, const std::vector<double>& A, const std::vector<double>& M,
                     std::vector<double>& lam, double** vecs, hipStream_t s) {
  *vecs = nullptr;
  const Solver& so = solver();
  if (!so.ok) {
    set_error("coarse eigensolve of %d vertices needs rocSOLVER: %s", n, so.why.c_str());
    return BMG_EDEVICE;
  }
  const size_t nn = size_t(n) * n;
  double *dA = nullptr, *dB = nullptr, *dD = nullptr, *dE = nullptr;
  rocblas_int* dinfo = nullptr;
  rocblas_handle hdl = nullptr;
  int st = BMG_OK;
  int info = 0;
  auto fail = [&](const char* what) {
    (void)hipGetLastError();
    set_error("coarse eigensolve: %s failed", what);
    st = BMG_EDEVICE;
  };
  if (hipMalloc(&dA, nn * 8) != hipSuccess || hipMalloc(&dB, nn * 8) != hipSuccess ||
      hipMalloc(&dD, size_t(n) * 8) != hipSuccess || hipMalloc(&dE, size_t(n) * 8) != hipSuccess ||
      hipMalloc(&dinfo, sizeof(rocblas_int)) != hipSuccess) {
    fail("device allocation");
  }
  // symmetric inputs: row-major equals column-major
  if (st == BMG_OK && (hipMemcpyAsync(dA, A.data(), nn * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
                       hipMemcpyAsync(dB, M.data(), nn * 8, hipMemcpyHostToDevice, s) != hipSuccess))
    fail("upload");
  if (st == BMG_OK) {
    DeviceSyncGuard sync;  // the handle's set-up may synchronise the device
    if (so.create(&hdl) != rocblas_status_success) fail("rocblas_create_handle");
  }
  if (st == BMG_OK && so.set_stream(hdl, s) != rocblas_status_success) fail("rocblas_set_stream");
  if (st == BMG_OK && so.sygvd(hdl, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_lower, n,
                               dA, n, dB, n, dD, dE, dinfo) != rocblas_status_success)
    fail("rocsolver_dsygvd");
  if (st == BMG_OK) {
    lam.assign(n, 0.0);
    if (hipMemcpyAsync(lam.data(), dD, size_t(n) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&info, dinfo, sizeof(rocblas_int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      fail("download");
  }
  if (hdl) {
    DeviceSyncGuard sync;  // and so may its teardown
    (void)so.destroy(hdl);
  }
  (void)hipStreamSynchronize(s);
  for (void* p : {(void*)dB, (void*)dD, (void*)dE, (void*)dinfo})
    if (p) dev_free(p);
  if (st == BMG_OK && info != 0) {
    set_error("coarse eigensolve: dsygvd info = %d (mass matrix not positive definite?)", info);
    st = BMG_EINVAL;
  }
  if (st != BMG_OK) {
    if (dA) dev_free(dA);
    return st;
  }
  *vecs = dA;
  return BMG_OK;
}

// lam ascending [n]; X row-major [n][n] with column j the M-orthonormal
// eigenvector of lam[j].
int device_sygv(int n, const std::vector<double>& A, const std::vector<double>& M,
                std::vector<double>& lam, std::vector<double>& X, hipStream_t s) {
  double* d = nullptr;
  BMG_TRY(device_sygv_keep(n, A, M, lam, &d, s));
  const size_t nn = size_t(n) * n;
  std::vector<double> rows(nn);
  const hipError_t e1 = hipMemcpyAsync(rows.data(), d, nn * 8, hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  dev_free(d);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    (void)hipGetLastError();
    set_error("coarse eigensolve: download failed");
    return BMG_EDEVICE;
  }
  // row j is eigenvector j: transpose to column j
  X.assign(nn, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) X[size_t(i) * n + j] = rows[size_t(j) * n + i];
  return BMG_OK;
}

}  // namespace bmg
