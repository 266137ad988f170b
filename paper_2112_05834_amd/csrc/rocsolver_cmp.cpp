// The vendor-library leg of the linear-algebra comparison: batched LU with
// partial pivoting and the solve by rocSOLVER (getrf / getrs, strided
// batched), on the same matrices as the library's own per-wave LU. It is
// not on the integration path: chem_lu_batch_rocsolver exists to time and
// check the library's LU against the vendor routine (paper: Methodology,
// the Analytical Jacobian paragraph, LAPACK in place of generic matrix
// routines; Fig. 2). rocSOLVER and rocBLAS are loaded at the first call with
// dlopen, so libchem.so does not depend on them.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/chem.h"

namespace chem {
// the message chem_last_error() returns (kept by the C ABI's translation unit)
void set_last_error(const std::string& msg);
}  // namespace chem

namespace {

// rocBLAS / rocSOLVER ABI (LP64 build: 32-bit rocblas_int, 64-bit strides)
using rb_handle = void*;
using rb_status = int;
using rb_int = int32_t;
using rb_stride = int64_t;
constexpr int kRbOpNone = 111;

using fn_create = rb_status (*)(rb_handle*);
using fn_set_stream = rb_status (*)(rb_handle, hipStream_t);
using fn_getrf = rb_status (*)(rb_handle, rb_int, rb_int, double*, rb_int, rb_stride, rb_int*, rb_stride, rb_int*,
                               rb_int);
using fn_getrs = rb_status (*)(rb_handle, int, rb_int, rb_int, double*, rb_int, rb_stride, const rb_int*,
                               rb_stride, double*, rb_int, rb_stride, rb_int);

struct Lib {
  bool tried = false;
  std::string err;
  fn_create create = nullptr;
  fn_set_stream set_stream = nullptr;
  fn_getrf getrf = nullptr;
  fn_getrs getrs = nullptr;
  std::vector<rb_handle> handles;   // per device
};

std::mutex g_mu;
Lib g_lib;

void* open_any(const char* const* names) {
  for (int i = 0; names[i]; ++i)
    if (void* h = dlopen(names[i], RTLD_NOW | RTLD_LOCAL)) return h;
  return nullptr;
}

// Loads the libraries once; returns false with g_lib.err set if they are not there.
bool load() {
  if (g_lib.tried) return g_lib.err.empty();
  g_lib.tried = true;
  static const char* const kBlas[] = {"librocblas.so", "librocblas.so.5", "/opt/rocm/lib/librocblas.so", nullptr};
  static const char* const kSolver[] = {"librocsolver.so", "librocsolver.so.0", "/opt/rocm/lib/librocsolver.so",
                                        nullptr};
  void* blas = open_any(kBlas);
  void* solver = blas ? open_any(kSolver) : nullptr;
  if (!blas || !solver) {
    g_lib.err = "rocBLAS / rocSOLVER could not be loaded";
    return false;
  }
  g_lib.create = reinterpret_cast<fn_create>(dlsym(blas, "rocblas_create_handle"));
  g_lib.set_stream = reinterpret_cast<fn_set_stream>(dlsym(blas, "rocblas_set_stream"));
  g_lib.getrf = reinterpret_cast<fn_getrf>(dlsym(solver, "rocsolver_dgetrf_strided_batched"));
  g_lib.getrs = reinterpret_cast<fn_getrs>(dlsym(solver, "rocsolver_dgetrs_strided_batched"));
  if (!g_lib.create || !g_lib.set_stream || !g_lib.getrf || !g_lib.getrs) {
    g_lib.err = "rocBLAS / rocSOLVER entry points not found";
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

int chem_lu_batch_rocsolver(int32_t n, int64_t batch, double* A, int32_t* piv, int32_t* info, double* b,
                            void* stream) {
  if (n < 1 || batch < 0 || batch > 0x7fffffffLL || (batch > 0 && (!A || !piv || !info))) {
    chem::set_last_error("chem_lu_batch_rocsolver: bad argument");
    return CHEM_EINVAL;
  }
  if (batch == 0) return CHEM_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    chem::set_last_error("chem_lu_batch_rocsolver: hipGetDevice failed");
    return CHEM_EHIP;
  }
  rb_handle h = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!load()) {
      chem::set_last_error("chem_lu_batch_rocsolver: " + g_lib.err);
      return CHEM_EUNSUPPORTED;
    }
    if (g_lib.handles.size() <= static_cast<size_t>(dev)) g_lib.handles.resize(dev + 1, nullptr);
    if (!g_lib.handles[dev] && g_lib.create(&g_lib.handles[dev]) != 0) {
      g_lib.handles[dev] = nullptr;
      chem::set_last_error("chem_lu_batch_rocsolver: rocblas_create_handle failed");
      return CHEM_EHIP;
    }
    h = g_lib.handles[dev];
  }
  if (g_lib.set_stream(h, static_cast<hipStream_t>(stream)) != 0) {
    chem::set_last_error("chem_lu_batch_rocsolver: rocblas_set_stream failed");
    return CHEM_EHIP;
  }
  const rb_stride sa = static_cast<rb_stride>(n) * n;
  if (g_lib.getrf(h, n, n, A, n, sa, piv, n, info, static_cast<rb_int>(batch)) != 0) {
    chem::set_last_error("chem_lu_batch_rocsolver: rocsolver_dgetrf_strided_batched failed");
    return CHEM_EHIP;
  }
  if (b && g_lib.getrs(h, kRbOpNone, n, 1, A, n, sa, piv, n, b, n, n, static_cast<rb_int>(batch)) != 0) {
    chem::set_last_error("chem_lu_batch_rocsolver: rocsolver_dgetrs_strided_batched failed");
    return CHEM_EHIP;
  }
  return CHEM_OK;
}

}  // extern "C"
