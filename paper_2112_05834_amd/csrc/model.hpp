// Learned cost model: features, 4->64->64->1 MLP (BF16 operands, FP32
// accumulation), training, and cost binning of the persistent queue.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/chem.h"
#include "kernels.hpp"

namespace chem_model {

constexpr int kIn = 4, kH = 64, kBins = 8;

struct Model {
  bool trained = false;
  // device buffers
  float* master = nullptr;      // FP32 master weights, packed (see model.hip)
  uint16_t* wbf16 = nullptr;    // BF16 copy used by inference
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;
  float* scratch = nullptr;     // activations for training
  long long scratch_n = 0;
  // binning
  float* feats = nullptr;       // [cap][4]
  float* pred = nullptr;        // [cap]
  int* perm = nullptr;          // [cap]
  int* counts = nullptr;        // per-block bin counts
  int* flag = nullptr;          // [0] = all predictions finite
  long long cap = 0;
  long long counts_cap = 0;
  // host copies of normalisation and bin edges
  float mu[kIn], sd[kIn];
  float edges[kBins - 1];
};

const char* last_error();
int init(Model& m);
void release(Model& m);
int features(const chemk::MechArgs& ma, long long n, double dt, const double* phi, float* feats, hipStream_t st);
int train(Model& m, long long n, const float* feats, const float* target, const chem_train_opts& t, hipStream_t st);
int predict(Model& m, long long n, const float* feats, float* pred, hipStream_t st);
// Queue order for the persistent kernel; *perm = NULL (queue order) when the
// model is not trained. With a cost override the given costs are binned.
int plan(Model& m, const chemk::MechArgs& ma, chemk::Variant v, long long n, double dt, const double* phi,
         const float* cost_override, hipStream_t st, const int** perm, int* used);
int save(const Model& m, const char* path);
int load(Model& m, const char* path);

}  // namespace chem_model
