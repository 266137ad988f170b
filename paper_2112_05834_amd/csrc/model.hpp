// Learned cost model: features, 4->64->64->1 ReLU MLP (BF16 operands, FP32
// accumulation, FP32 master weights, Adam), octile bin edges, and the
// longest-first binned order of the persistent work queue.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/chem.h"
#include "kernels.hpp"

namespace chem_model {

constexpr int kIn = 4, kH = 64, kBins = 8;
// Parameter vector layout (FP32 master and BF16 copy alike):
// W1 [64][4], b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
constexpr int kOffW1 = 0, kOffB1 = 256, kOffW2 = 320, kOffB2 = 4416, kOffW3 = 4480, kOffB3 = 4544;
constexpr int kParams = 4545;
constexpr int kBinBlock = 4096;   // cells per block of the binning kernels

struct Model {
  bool has_params = false;        // weights present (trained, loaded or set)
  bool has_edges = false;
  // device
  float* master = nullptr;        // [kParams] FP32
  uint16_t* wbf16 = nullptr;      // [kParams] BF16 bits of master
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* norm = nullptr;          // [8] mu[4], sd[4]
  float* dedges = nullptr;        // [7]
  float* partial = nullptr;       // [partial_cap][kParams + 1] per-block gradients and loss
  long long partial_cap = 0;
  unsigned int* sel = nullptr;    // radix-select state and histograms
  double* stats = nullptr;        // reduction scratch
  // binning buffers, sized by reserve()
  float* feats = nullptr;         // [cap][4]
  float* cost = nullptr;          // [cap]
  int* perm = nullptr;            // [cap]
  int* counts = nullptr;          // [blocks][kBins + 1] and [blocks][kBins] offsets, flag
  long long cap = 0;
  long long counts_cap = 0;
  long long last_nblk = 0;        // block count of the last binning (locates its flag)
  // host copies
  float mu[kIn], sd[kIn];
  float edges[kBins - 1];
};

const char* last_error();
int init(Model& m);
void release(Model& m);
// Make the binning buffers hold n cells (allocates; call outside graph capture).
int reserve(Model& m, long long n);
int features(const chemk::MechArgs& ma, long long n, double dt, const double* phi, float* feats, hipStream_t st);
int train(Model& m, long long n, const float* feats, const float* target, const chem_train_opts& t, hipStream_t st);
int predict(Model& m, long long n, const float* feats, float* pred, hipStream_t st);
// Loss and gradient of the current weights over n samples taken as one batch.
int grad(Model& m, long long n, const float* feats, const float* target, float* grad, float* loss, hipStream_t st);
int get_params(const Model& m, float* params, float* norm, float* edges);
int set_params(Model& m, const float* params, const float* norm, const float* edges);
// Octile edges of n device costs, written to host edges[7]. Synchronises.
int octiles(Model& m, long long n, const float* cost, float* edges, hipStream_t st);
// Queue order for n costs and edges (host array; NULL = the model's edges).
int order(Model& m, long long n, const float* cost, const float* edges, int* perm, hipStream_t st);
// Queue order for the persistent kernel. *perm = NULL (plain queue order)
// and *used = 0 when there is no model and no cost override.
int plan(Model& m, const chemk::MechArgs& ma, long long n, double dt, const double* phi,
         const float* cost_override, hipStream_t st, const int** perm, int* used);
// Whether the last plan's costs were all finite (reads the device flag).
int last_plan_finite(const Model& m, int* finite);
int save(const Model& m, const char* path);
int load(Model& m, const char* path);

}  // namespace chem_model
