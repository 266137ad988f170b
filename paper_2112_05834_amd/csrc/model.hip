// Learned cost model driver (features; MLP and binning come with their oracle).
#include "model.hpp"

#include <cmath>
#include <cstdio>
#include <string>

namespace chem_model {

namespace {
thread_local std::string g_err;

// features of one cell: (T-1500)/700, ln(p/1e5), mean log10 max(Y,1e-30)/10,
// log10(dt/1e-6); one thread per cell
__global__ void k_features(int ns, long long n, double dt, const double* __restrict__ phi, float* __restrict__ f) {
  const long long c = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  if (c >= n) return;
  const double* p = phi + c * (ns + 2);
  double ell = 0.0;
  for (int i = 0; i < ns; ++i) ell += log10(fmax(p[2 + i], 1e-30));
  ell /= ns;
  f[4 * c + 0] = static_cast<float>((p[0] - 1500.0) / 700.0);
  f[4 * c + 1] = static_cast<float>(log(p[1] / 1e5));
  f[4 * c + 2] = static_cast<float>(ell / 10.0);
  f[4 * c + 3] = static_cast<float>(log10(dt / 1e-6));
}
}  // namespace

const char* last_error() { return g_err.c_str(); }

int init(Model& m) {
  m = Model{};
  return 0;
}

void release(Model& m) {
  hipFree(m.master);
  hipFree(m.wbf16);
  hipFree(m.adam_m);
  hipFree(m.adam_v);
  hipFree(m.grad);
  hipFree(m.scratch);
  hipFree(m.feats);
  hipFree(m.pred);
  hipFree(m.perm);
  hipFree(m.counts);
  hipFree(m.flag);
  m = Model{};
}

int features(const chemk::MechArgs& ma, long long n, double dt, const double* phi, float* feats, hipStream_t st) {
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_features, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, ma.ns, n, dt, phi, feats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_err = std::string("features launch: ") + hipGetErrorString(e);
    return CHEM_EHIP;
  }
  return 0;
}

int train(Model&, long long, const float*, const float*, const chem_train_opts&, hipStream_t) {
  g_err = "model training not available in this build";
  return CHEM_EUNSUPPORTED;
}

int predict(Model& m, long long, const float*, float*, hipStream_t) {
  g_err = m.trained ? "prediction not available in this build" : "model not trained";
  return CHEM_ESTATE;
}

int plan(Model& m, const chemk::MechArgs&, chemk::Variant, long long, double, const double*, const float*,
         hipStream_t, const int** perm, int* used) {
  *perm = nullptr;
  *used = 0;
  (void)m;
  return 0;
}

int save(const Model& m, const char*) {
  g_err = m.trained ? "save not available in this build" : "model not trained";
  return CHEM_ESTATE;
}

int load(Model&, const char*) {
  g_err = "load not available in this build";
  return CHEM_EUNSUPPORTED;
}

}  // namespace chem_model
