// Learned cost model: the paper balances the uneven per-cell chemistry cost
// across processes ("DLBFoam: Dynamic load balancing"); here the cost of each
// cell is predicted from four state features by a small MLP, and the
// persistent kernel's work queue is ordered by predicted cost, longest first,
// in eight bins. The order changes which wave integrates which cell and when,
// never the arithmetic of a cell, so results are bit-identical to unbinned.
//
// MLP: 4 -> 64 -> 64 -> 1, ReLU, predicting ln(accepted + rejected steps).
// Contraction operands are BF16 (round to nearest even), accumulation and
// stored activations FP32, master weights FP32, Adam. The 64x64 layer and its
// two backward contractions run on the 32x32x8 BF16 matrix instruction, one
// wave per 32 samples, in transposed form (weights as the A operand,
// activations as B): then the accumulator layout of the forward product is
// exactly the B operand layout of the backward product, so the error never
// has to be transposed through LDS. Weight-gradient sums over samples are
// taken in a fixed order (LDS columns, then blocks in index order), so
// training is deterministic.
#include "model.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace chem_model {

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define MTRY(expr, what)                                                   \
  do {                                                                     \
    hipError_t _e = (expr);                                                \
    if (_e != hipSuccess) return fail(CHEM_EHIP, std::string(what) + ": " + hipGetErrorString(_e)); \
  } while (0)

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kPartStride = kParams + 1;   // per-block gradient + loss
constexpr int kSelPrefix = 0, kSelRank = 8, kSelHist = 16;
constexpr int kSelWords = kSelHist + 7 * 256;
constexpr int kStatBlocks = 256;

// ---- BF16 ------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ float bf16r(float x) { return bf16_val(bf16_bits(x)); }
// ReLU that lets NaN through (a non-finite prediction must stay visible)
__device__ __forceinline__ float relu(float a) { return a <= 0.f ? 0.f : a; }

__device__ __forceinline__ v16f mfma(v4s a, v4s b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// ---- small parameters, staged in LDS per block ------------------------------
struct Small {
  float w1[kH][kIn];   // BF16 values of W1
  float b1[kH], b2[kH];
  float w3[kH];        // BF16 values of w3
  float b3;
  float mu[kIn], sd[kIn];
};

__device__ void load_small(Small& S, const float* master, const uint16_t* wb, const float* norm) {
  for (int p = threadIdx.x; p < kH * kIn; p += blockDim.x) S.w1[p / kIn][p % kIn] = bf16_val(wb[kOffW1 + p]);
  for (int p = threadIdx.x; p < kH; p += blockDim.x) {
    S.b1[p] = master[kOffB1 + p];
    S.b2[p] = master[kOffB2 + p];
    S.w3[p] = bf16_val(wb[kOffW3 + p]);
  }
  if (threadIdx.x == 0) S.b3 = master[kOffB3];
  if (threadIdx.x < kIn) {
    S.mu[threadIdx.x] = norm[threadIdx.x];
    S.sd[threadIdx.x] = norm[kIn + threadIdx.x];
  }
}

// W2 as the A operand of the forward product a2^T = W2 h1^T: lane (s, hh)
// holds W2[32 mt + s][8 kk + 4 hh + 0..3].
__device__ __forceinline__ void load_w2(const uint16_t* wb, int s, int hh, v4s (&w)[2][8]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      w[mt][kk] = *reinterpret_cast<const v4s*>(wb + kOffW2 + (32 * mt + s) * kH + 8 * kk + 4 * hh);
}

// W2^T as the A operand of dh1^T = W2^T d2^T: lane (s, hh) holds
// W2[8 kk + 4 hh + 0..3][32 mt + s].
__device__ __forceinline__ void load_w2t(const uint16_t* wb, int s, int hh, v4s (&w)[2][8]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        w[mt][kk][q] = static_cast<short>(wb[kOffW2 + (8 * kk + 4 * hh + q) * kH + 32 * mt + s]);
}

// Forward pass of one sample per lane pair: lane (s, hh) computes the hidden
// units k = 8 kk + 4 hh + q of layer 1 (exactly the B operand it supplies)
// and receives units j = 32 mt + 8 (r/4) + 4 hh + r%4 of layer 2.
// On return a2[mt][r] holds the BF16 value of h2, m1/m2 the ReLU masks.
__device__ __forceinline__ float forward(const Small& S, const v4s (&w2)[2][8], const float (&xb)[kIn], int hh,
                                         v4s (&hA)[8], uint32_t& m1, v16f (&a2)[2], uint32_t& m2) {
  m1 = 0;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 8 * kk + 4 * hh + q;
      float a = S.b1[k];
#pragma unroll
      for (int c = 0; c < kIn; ++c) a = fmaf(xb[c], S.w1[k][c], a);
      if (a > 0.f) m1 |= 1u << (4 * kk + q);
      hA[kk][q] = static_cast<short>(bf16_bits(relu(a)));
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    v16f acc = {};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc = mfma(w2[mt][kk], hA[kk], acc);
    a2[mt] = acc;
  }
  m2 = 0;
  float yp = 0.f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = 32 * mt + 8 * (r >> 2) + 4 * hh + (r & 3);
      const float a = a2[mt][r] + S.b2[j];
      if (a > 0.f) m2 |= 1u << (16 * mt + r);
      const float hb = bf16r(relu(a));
      a2[mt][r] = hb;
      yp = fmaf(hb, S.w3[j], yp);
    }
  }
  return (yp + __shfl_xor(yp, 32)) + S.b3;
}

__device__ __forceinline__ void load_x(const Small& S, const float* feats, long long idx, bool valid,
                                       float (&xb)[kIn]) {
#pragma unroll
  for (int c = 0; c < kIn; ++c) xb[c] = valid ? bf16r((feats[4 * idx + c] - S.mu[c]) / S.sd[c]) : 0.f;
}

// ---- inference ----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_predict(const float* __restrict__ master, const uint16_t* __restrict__ wb,
                                                 const float* __restrict__ norm, const float* __restrict__ feats,
                                                 long long n, float* __restrict__ out) {
  __shared__ Small S;
  load_small(S, master, wb, norm);
  __syncthreads();
  const int l = threadIdx.x & 63, s = l & 31, hh = l >> 5;
  v4s w2[2][8];
  load_w2(wb, s, hh, w2);
  const long long chunks = (n + 31) / 32;
  const long long waves = static_cast<long long>(gridDim.x) * (blockDim.x / 64);
  for (long long c = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); c < chunks; c += waves) {
    const long long idx = 32 * c + s;
    const bool valid = idx < n;
    float xb[kIn];
    load_x(S, feats, idx, valid, xb);
    v4s hA[8];
    uint32_t m1, m2;
    v16f a2[2];
    const float y = forward(S, w2, xb, hh, hA, m1, a2, m2);
    if (valid && hh == 0) out[idx] = y;
  }
}

// ---- training: forward + backward of one minibatch ------------------------------
// Block = one wave; it takes samples [blockIdx.x*spw, ...) of the minibatch in
// chunks of 32 and writes its summed gradient and squared error to
// partial[blockIdx.x]. Sample i of the minibatch is data index
// ((start + i) * mul + add) mod n.
__global__ __launch_bounds__(64) void k_train(const float* __restrict__ master, const uint16_t* __restrict__ wb,
                                              const float* __restrict__ norm, const float* __restrict__ feats,
                                              const float* __restrict__ target, long long n, long long start,
                                              long long bcur, unsigned long long mul, unsigned long long add,
                                              int spw, float* __restrict__ partial) {
  __shared__ Small S;
  __shared__ float sA[32 * kH], sB[32 * kH];
  __shared__ uint16_t sD2[32 * kH], sH1[32 * kH];
  __shared__ float sX[32][kIn], sD3[32];
  load_small(S, master, wb, norm);
  __syncthreads();
  const int t = threadIdx.x, s = t & 31, hh = t >> 5;
  v4s w2[2][8], w2t[2][8];
  load_w2(wb, s, hh, w2);
  load_w2t(wb, s, hh, w2t);
  v16f gacc[2][2] = {};
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, gw1[kIn] = {0.f, 0.f, 0.f, 0.f}, lsum = 0.f;
  const float inv_b = 1.0f / static_cast<float>(bcur);
  const long long i0 = static_cast<long long>(blockIdx.x) * spw;
  const long long i1 = i0 + spw < bcur ? i0 + spw : bcur;
  for (long long base = i0; base < i1; base += 32) {
    const long long i = base + s;
    const bool valid = i < i1;
    const long long idx = valid ? static_cast<long long>((static_cast<unsigned long long>(start + i) * mul + add) %
                                                         static_cast<unsigned long long>(n))
                                : 0;
    float xb[kIn];
    load_x(S, feats, idx, valid, xb);
    const float tv = valid ? target[idx] : 0.f;
    v4s hA[8];
    uint32_t m1, m2;
    v16f a2[2];
    const float y = forward(S, w2, xb, hh, hA, m1, a2, m2);
    const float r = y - tv;
    const float d3 = valid ? (2.f * r) * inv_b : 0.f;
    const float d3b = bf16r(d3);
    if (valid && hh == 0) lsum = fmaf(r, r, lsum);
    // layer-2 error, its BF16 copy as the next B operand, LDS columns for sums
    v4s d2B[8];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int j = 32 * mt + 8 * (rr >> 2) + 4 * hh + (rr & 3);
        const float d2 = ((m2 >> (16 * mt + rr)) & 1u) ? d3b * S.w3[j] : 0.f;
        const uint16_t d2b = bf16_bits(d2);
        d2B[4 * mt + (rr >> 2)][rr & 3] = static_cast<short>(d2b);
        sA[s * kH + j] = d2;
        sB[s * kH + j] = a2[mt][rr] * d3b;
        sD2[s * kH + j] = d2b;
      }
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int q = 0; q < 4; ++q) sH1[s * kH + 8 * kk + 4 * hh + q] = static_cast<uint16_t>(hA[kk][q]);
    if (hh == 0) {
#pragma unroll
      for (int c = 0; c < kIn; ++c) sX[s][c] = xb[c];
      sD3[s] = d3;
    }
    __syncthreads();
    // bias and output-layer sums, one hidden unit per thread
    for (int q = 0; q < 32; ++q) {
      gb2 += sA[q * kH + t];
      gw3 += sB[q * kH + t];
    }
    if (t == 0)
      for (int q = 0; q < 32; ++q) gb3 += sD3[q];
    // dW2[j][k] = sum_s d2[s][j] h1[s][k]: A = d2^T, B = h1, K = samples
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      v4s A[2], B[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int sq = 8 * ks + 4 * hh + q;
        A[0][q] = static_cast<short>(sD2[sq * kH + s]);
        A[1][q] = static_cast<short>(sD2[sq * kH + 32 + s]);
        B[0][q] = static_cast<short>(sH1[sq * kH + s]);
        B[1][q] = static_cast<short>(sH1[sq * kH + 32 + s]);
      }
#pragma unroll
      for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) gacc[jt][kt] = mfma(A[jt], B[kt], gacc[jt][kt]);
    }
    // dh1^T = W2^T d2^T
    v16f dh[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      v16f acc = {};
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) acc = mfma(w2t[mt][kk], d2B[kk], acc);
      dh[mt] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int k = 32 * mt + 8 * (rr >> 2) + 4 * hh + (rr & 3);
        const float d1 = ((m1 >> (16 * mt + rr)) & 1u) ? dh[mt][rr] : 0.f;
        sA[s * kH + k] = d1;
        sB[s * kH + k] = bf16r(d1);
      }
    }
    __syncthreads();
    for (int q = 0; q < 32; ++q) {
      gb1 += sA[q * kH + t];
      const float d1b = sB[q * kH + t];
#pragma unroll
      for (int c = 0; c < kIn; ++c) gw1[c] = fmaf(d1b, sX[q][c], gw1[c]);
    }
    __syncthreads();
  }
  // squared-error sum over the wave, fixed pairing
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off);
  float* P = partial + static_cast<long long>(blockIdx.x) * kPartStride;
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int j = 32 * jt + 8 * (rr >> 2) + 4 * hh + (rr & 3);
        const int k = 32 * kt + s;
        P[kOffW2 + j * kH + k] = gacc[jt][kt][rr];
      }
#pragma unroll
  for (int c = 0; c < kIn; ++c) P[kOffW1 + t * kIn + c] = gw1[c];
  P[kOffB1 + t] = gb1;
  P[kOffB2 + t] = gb2;
  P[kOffW3 + t] = gw3;
  if (t == 0) {
    P[kOffB3] = gb3;
    P[kParams] = lsum;
  }
}

// Sum the block gradients in block order; optionally apply one Adam step
// (Kingma and Ba) to the FP32 master weights and refresh their BF16 copy.
__global__ void k_reduce_adam(const float* __restrict__ partial, int nblk, long long bcur, float* __restrict__ master,
                              uint16_t* __restrict__ wb, float* __restrict__ am, float* __restrict__ av, float lr,
                              float b1, float b2, float eps, float bc1, float bc2, int update,
                              float* __restrict__ grad_out, float* __restrict__ loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += partial[static_cast<long long>(b) * kPartStride + p];
  if (p == kParams) {
    if (loss_out) loss_out[0] = g / static_cast<float>(bcur);
    return;
  }
  if (grad_out) grad_out[p] = g;
  if (update) {
    const float m = b1 * am[p] + (1.f - b1) * g;
    const float v = b2 * av[p] + (1.f - b2) * g * g;
    am[p] = m;
    av[p] = v;
    const float th = master[p] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    master[p] = th;
    wb[p] = bf16_bits(th);
  }
}

// ---- initialisation, normalisation -----------------------------------------
__device__ __forceinline__ unsigned long long splitmix(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// He-uniform weights from a counter-based hash of (seed, index), zero biases,
// output bias = mean target, zero Adam moments.
__global__ void k_init_params(unsigned long long seed, const double* __restrict__ stats, float* __restrict__ master,
                              uint16_t* __restrict__ wb, float* __restrict__ am, float* __restrict__ av) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const double u = static_cast<double>(splitmix(seed * 0x100000001b3ull + static_cast<unsigned long long>(p)) >> 11) *
                   (1.0 / 9007199254740992.0);
  float bound = 0.f;
  if (p < kOffB1) bound = sqrtf(6.f / kIn);
  else if (p >= kOffW2 && p < kOffB2) bound = sqrtf(6.f / kH);
  else if (p >= kOffW3 && p < kOffB3) bound = sqrtf(3.f / kH);
  float v = static_cast<float>((2.0 * u - 1.0) * bound);
  if (p == kOffB3) v = static_cast<float>(stats[4]);
  master[p] = v;
  wb[p] = bf16_bits(v);
  am[p] = 0.f;
  av[p] = 0.f;
}

// Per-block sums of the 4 features and the target (pass 0) or of squared
// deviations from the means in stats[0..3] (pass 1), FP64, fixed grid.
__global__ __launch_bounds__(256) void k_stats(const float* __restrict__ feats, const float* __restrict__ target,
                                               long long n, int pass, const double* __restrict__ stats,
                                               double* __restrict__ part) {
  __shared__ double red[5][256];
  double acc[5] = {0, 0, 0, 0, 0};
  double mu[4] = {0, 0, 0, 0};
  if (pass == 1)
    for (int c = 0; c < 4; ++c) mu[c] = stats[c];
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    for (int c = 0; c < 4; ++c) {
      const double x = feats[4 * i + c];
      acc[c] += pass == 0 ? x : (x - mu[c]) * (x - mu[c]);
    }
    if (pass == 0) acc[4] += target[i];
  }
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

// Combine the block sums in block order: pass 0 -> means (stats[0..4]),
// pass 1 -> standard deviations and the FP32 normalisation vector.
__global__ void k_stats_final(const double* __restrict__ part, int nblk, long long n, int pass,
                              double* __restrict__ stats, float* __restrict__ norm) {
  const int c = threadIdx.x;
  if (c >= 5) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[b * 5 + c];
  if (pass == 0) {
    stats[c] = s / static_cast<double>(n);
    if (c < 4) norm[c] = static_cast<float>(stats[c]);
  } else if (c < 4) {
    double sd = sqrt(s / static_cast<double>(n));
    if (sd < 1e-6) sd = 1.0;
    stats[5 + c] = sd;
    norm[4 + c] = static_cast<float>(sd);
  }
}

// ---- features -------------------------------------------------------------------
// (T-1500)/700, ln(p/1e5), mean log10 max(Y,1e-30)/10, log10(dt/1e-6); one
// thread per cell
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

// ---- octile edges: radix select of the 7 order statistics -------------------------
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unfkey(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_sel_init(long long n, uint32_t* __restrict__ sel) {
  for (int e = threadIdx.x; e < kSelWords; e += blockDim.x) sel[e] = 0;
  __syncthreads();
  if (threadIdx.x < 7) sel[kSelRank + threadIdx.x] = static_cast<uint32_t>(((threadIdx.x + 1) * n) / 8);
}

// Histogram of the next 8 key bits among keys that match each target's prefix.
__global__ __launch_bounds__(256) void k_sel_hist(int pass, const float* __restrict__ cost, long long n,
                                                  uint32_t* __restrict__ sel) {
  __shared__ uint32_t lh[7 * 256];
  __shared__ uint32_t pre[7];
  for (int e = threadIdx.x; e < 7 * 256; e += 256) lh[e] = 0;
  if (threadIdx.x < 7) pre[threadIdx.x] = sel[kSelPrefix + threadIdx.x];
  __syncthreads();
  const int sh = 24 - 8 * pass;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    const uint32_t k = fkey(cost[i]);
    const uint32_t d = (k >> sh) & 255u;
    for (int t = 0; t < 7; ++t)
      if (pass == 0 || (k >> (sh + 8)) == pre[t]) atomicAdd(&lh[t * 256 + d], 1u);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 7 * 256; e += 256)
    if (lh[e]) atomicAdd(&sel[kSelHist + e], lh[e]);
}

// Pick each target's digit, narrow its rank, clear the histograms; after the
// last pass write the edges.
__global__ void k_sel_pick(int pass, uint32_t* __restrict__ sel, float* __restrict__ edges) {
  const int t = threadIdx.x;
  if (t < 7) {
    uint32_t cum = 0, d = 255;
    const uint32_t rank = sel[kSelRank + t];
    for (uint32_t b = 0; b < 256; ++b) {
      const uint32_t c = sel[kSelHist + t * 256 + b];
      if (rank < cum + c) {
        d = b;
        break;
      }
      cum += c;
    }
    sel[kSelRank + t] = rank - cum;
    const uint32_t pre = (sel[kSelPrefix + t] << 8) | d;
    sel[kSelPrefix + t] = pre;
    if (pass == 3) edges[t] = unfkey(pre);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 7 * 256; e += blockDim.x) sel[kSelHist + e] = 0;
}

// ---- binned queue order ----------------------------------------------------------
struct Edges {
  float e[kBins - 1];
};

__device__ __forceinline__ int bin_of(float c, const Edges& E) {
  int b = 0;
#pragma unroll
  for (int k = 0; k < kBins - 1; ++k) b += c >= E.e[k] ? 1 : 0;
  return b;
}

// counts layout: cnt [nblk][9] (8 bins, all-finite), off [nblk][8], flag
__global__ __launch_bounds__(256) void k_bin_count(const float* __restrict__ cost, long long n, Edges E,
                                                   int* __restrict__ cnt) {
  __shared__ int lc[kBins];
  __shared__ int fin;
  if (threadIdx.x < kBins) lc[threadIdx.x] = 0;
  if (threadIdx.x == 0) fin = 1;
  __syncthreads();
  const long long b0 = static_cast<long long>(blockIdx.x) * kBinBlock;
  for (int q = threadIdx.x; q < kBinBlock; q += 256) {
    const long long i = b0 + q;
    if (i >= n) break;
    const float c = cost[i];
    if (!isfinite(c)) fin = 0;
    atomicAdd(&lc[bin_of(c, E)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kBins) cnt[blockIdx.x * 9 + threadIdx.x] = lc[threadIdx.x];
  if (threadIdx.x == 0) cnt[blockIdx.x * 9 + 8] = fin;
}

// Queue offsets: bin 7 first; within a bin, blocks in index order.
__global__ void k_bin_scan(int* __restrict__ cnt, int nblk) {
  __shared__ int tot[kBins];
  int* off = cnt + nblk * 9;
  int* flag = off + nblk * kBins;
  const int b = threadIdx.x;
  if (b < kBins) {
    int s = 0;
    for (int k = 0; k < nblk; ++k) s += cnt[k * 9 + b];
    tot[b] = s;
  }
  if (b == kBins) {
    int f = 1;
    for (int k = 0; k < nblk; ++k) f &= cnt[k * 9 + 8];
    flag[0] = f;
  }
  __syncthreads();
  if (b < kBins) {
    int run = 0;
    for (int h = kBins - 1; h > b; --h) run += tot[h];
    for (int k = 0; k < nblk; ++k) {
      off[k * kBins + b] = run;
      run += cnt[k * 9 + b];
    }
  }
}

// Stable scatter: cells of one bin keep their index order. With a non-finite
// cost anywhere the order is the identity.
__global__ __launch_bounds__(256) void k_bin_scatter(const float* __restrict__ cost, long long n, Edges E,
                                                     const int* __restrict__ cnt, int nblk, int* __restrict__ perm) {
  __shared__ int run[kBins];
  __shared__ int wc[4][kBins];
  const int* off = cnt + nblk * 9;
  const int* flag = off + nblk * kBins;
  const long long b0 = static_cast<long long>(blockIdx.x) * kBinBlock;
  if (!flag[0]) {
    for (int q = threadIdx.x; q < kBinBlock; q += 256)
      if (b0 + q < n) perm[b0 + q] = static_cast<int>(b0 + q);
    return;
  }
  if (threadIdx.x < kBins) run[threadIdx.x] = off[blockIdx.x * kBins + threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = 0; base < kBinBlock; base += 256) {
    const long long i = b0 + base + threadIdx.x;
    const bool valid = i < n;
    const int b = valid ? bin_of(cost[i], E) : -1;
    int rank = 0;
#pragma unroll
    for (int h = 0; h < kBins; ++h) {
      const unsigned long long m = __ballot(b == h);
      if (b == h) rank = __popcll(m & below);
      if (lane == 0) wc[wv][h] = __popcll(m);
    }
    __syncthreads();
    if (valid) {
      int pos = run[b] + rank;
      for (int w = 0; w < wv; ++w) pos += wc[w][b];
      perm[pos] = static_cast<int>(i);
    }
    __syncthreads();
    if (threadIdx.x < kBins) run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
    __syncthreads();
  }
}

// ---- host helpers ------------------------------------------------------------------
int ensure_core(Model& m) {
  if (m.master) return 0;
  MTRY(hipMalloc(&m.master, kParams * sizeof(float)), "hipMalloc model");
  MTRY(hipMalloc(&m.wbf16, (kParams + 3) * sizeof(uint16_t)), "hipMalloc model");
  MTRY(hipMalloc(&m.adam_m, kParams * sizeof(float)), "hipMalloc model");
  MTRY(hipMalloc(&m.adam_v, kParams * sizeof(float)), "hipMalloc model");
  MTRY(hipMalloc(&m.norm, 8 * sizeof(float)), "hipMalloc model");
  MTRY(hipMalloc(&m.dedges, 8 * sizeof(float)), "hipMalloc model");
  MTRY(hipMalloc(&m.sel, kSelWords * sizeof(uint32_t)), "hipMalloc model");
  MTRY(hipMalloc(&m.stats, (16 + 5 * kStatBlocks) * sizeof(double)), "hipMalloc model");
  return 0;
}

int ensure_partial(Model& m, long long nblk) {
  if (m.partial_cap >= nblk) return 0;
  hipFree(m.partial);
  m.partial = nullptr;
  m.partial_cap = 0;
  MTRY(hipMalloc(&m.partial, static_cast<size_t>(nblk) * kPartStride * sizeof(float)), "hipMalloc gradients");
  m.partial_cap = nblk;
  return 0;
}

hipError_t launch_err() { return hipGetLastError(); }

// samples per training wave: at least 128, at most 1024 waves per minibatch
int samples_per_wave(long long b) {
  long long spw = (b + 1023) / 1024;
  spw = (spw + 31) / 32 * 32;
  return static_cast<int>(spw < 128 ? 128 : spw);
}

int run_octiles(Model& m, long long n, const float* cost, float* dedges, hipStream_t st) {
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, st, n, m.sel);
  long long g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  for (int pass = 0; pass < 4; ++pass) {
    hipLaunchKernelGGL(k_sel_hist, dim3(static_cast<unsigned>(g)), dim3(256), 0, st, pass, cost, n, m.sel);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, st, pass, m.sel, dedges);
  }
  MTRY(launch_err(), "octile launch");
  return 0;
}

int run_order(Model& m, long long n, const float* cost, const Edges& E, int* perm, hipStream_t st) {
  const long long nblk = (n + kBinBlock - 1) / kBinBlock;
  if (nblk > m.counts_cap) return fail(CHEM_ESTATE, "binning buffers too small");
  m.last_nblk = nblk;
  hipLaunchKernelGGL(k_bin_count, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, cost, n, E, m.counts);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(64), 0, st, m.counts, static_cast<int>(nblk));
  hipLaunchKernelGGL(k_bin_scatter, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, cost, n, E, m.counts,
                     static_cast<int>(nblk), perm);
  MTRY(launch_err(), "binning launch");
  return 0;
}

int run_predict(Model& m, long long n, const float* feats, float* out, hipStream_t st) {
  long long g = (n + 127) / 128;
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_predict, dim3(static_cast<unsigned>(g)), dim3(256), 0, st, m.master, m.wbf16, m.norm, feats,
                     n, out);
  MTRY(launch_err(), "predict launch");
  return 0;
}

// one minibatch: gradient (and Adam step when update)
int run_batch(Model& m, long long n, const float* feats, const float* target, long long start, long long bcur,
              unsigned long long mul, unsigned long long add, bool update, const chem_train_opts* t, int step,
              float* grad_out, float* loss_out, hipStream_t st) {
  const int spw = samples_per_wave(bcur);
  const long long nblk = (bcur + spw - 1) / spw;
  if (int rc = ensure_partial(m, nblk)) return rc;
  hipLaunchKernelGGL(k_train, dim3(static_cast<unsigned>(nblk)), dim3(64), 0, st, m.master, m.wbf16, m.norm, feats,
                     target, n, start, bcur, mul, add, spw, m.partial);
  float lr = 0, b1 = 0, b2 = 0, eps = 0, bc1 = 1, bc2 = 1;
  if (update) {
    lr = t->lr;
    b1 = t->beta1;
    b2 = t->beta2;
    eps = t->eps;
    bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), step));
    bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), step));
  }
  hipLaunchKernelGGL(k_reduce_adam, dim3((kParams + 1 + 255) / 256), dim3(256), 0, st, m.partial,
                     static_cast<int>(nblk), bcur, m.master, m.wbf16, m.adam_m, m.adam_v, lr, b1, b2, eps, bc1, bc2,
                     update ? 1 : 0, grad_out, loss_out);
  MTRY(launch_err(), "training launch");
  return 0;
}

unsigned long long host_mix(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

unsigned long long gcd(unsigned long long a, unsigned long long b) {
  while (b) {
    const unsigned long long r = a % b;
    a = b;
    b = r;
  }
  return a;
}

}  // namespace

const char* last_error() { return g_err.c_str(); }

int init(Model& m) {
  m = Model{};
  for (int c = 0; c < kIn; ++c) {
    m.mu[c] = 0.f;
    m.sd[c] = 1.f;
  }
  return 0;
}

void release(Model& m) {
  hipFree(m.master);
  hipFree(m.wbf16);
  hipFree(m.adam_m);
  hipFree(m.adam_v);
  hipFree(m.norm);
  hipFree(m.dedges);
  hipFree(m.partial);
  hipFree(m.sel);
  hipFree(m.stats);
  hipFree(m.feats);
  hipFree(m.cost);
  hipFree(m.perm);
  hipFree(m.counts);
  init(m);
}

int reserve(Model& m, long long n) {
  if (int rc = ensure_core(m)) return rc;
  if (n > m.cap) {
    hipFree(m.feats);
    hipFree(m.cost);
    hipFree(m.perm);
    m.feats = nullptr;
    m.cost = nullptr;
    m.perm = nullptr;
    m.cap = 0;
    MTRY(hipMalloc(&m.feats, static_cast<size_t>(n) * 4 * sizeof(float)), "hipMalloc binning");
    MTRY(hipMalloc(&m.cost, static_cast<size_t>(n) * sizeof(float)), "hipMalloc binning");
    MTRY(hipMalloc(&m.perm, static_cast<size_t>(n) * sizeof(int)), "hipMalloc binning");
    m.cap = n;
  }
  const long long nblk = (n + kBinBlock - 1) / kBinBlock;
  if (nblk > m.counts_cap) {
    hipFree(m.counts);
    m.counts = nullptr;
    m.counts_cap = 0;
    MTRY(hipMalloc(&m.counts, static_cast<size_t>(nblk * (9 + kBins) + 1) * sizeof(int)), "hipMalloc binning");
    m.counts_cap = nblk;
  }
  return 0;
}

int features(const chemk::MechArgs& ma, long long n, double dt, const double* phi, float* feats, hipStream_t st) {
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_features, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, ma.ns, n, dt, phi, feats);
  MTRY(launch_err(), "features launch");
  return 0;
}

int train(Model& m, long long n, const float* feats, const float* target, const chem_train_opts& t, hipStream_t st) {
  if (n > 0x7fffffffLL) return fail(CHEM_EINVAL, "too many training samples");
  if (int rc = ensure_core(m)) return rc;
  if (int rc = reserve(m, n)) return rc;
  m.has_params = false;
  m.has_edges = false;
  // feature standardisation and mean target
  double* part = m.stats + 16;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_stats, dim3(kStatBlocks), dim3(256), 0, st, feats, target, n, pass, m.stats, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, kStatBlocks, n, pass, m.stats, m.norm);
  }
  hipLaunchKernelGGL(k_init_params, dim3((kParams + 255) / 256), dim3(256), 0, st,
                     static_cast<unsigned long long>(t.seed), m.stats, m.master, m.wbf16, m.adam_m, m.adam_v);
  MTRY(launch_err(), "model init launch");
  const long long B = t.batch < n ? t.batch : n;
  const long long steps = (n + B - 1) / B;
  int step = 0;
  for (int ep = 0; ep < t.epochs; ++ep) {
    // epoch order: i -> (i*mul + add) mod n with mul coprime to n
    const unsigned long long h = host_mix(t.seed ^ (0x5851f42d4c957f2dull * (ep + 1)));
    unsigned long long mul = 1, add = 0;
    if (n > 1) {
      mul = 1 + host_mix(h) % static_cast<unsigned long long>(n - 1);
      while (gcd(mul, static_cast<unsigned long long>(n)) != 1) mul = mul % static_cast<unsigned long long>(n - 1) + 1;
      add = h % static_cast<unsigned long long>(n);
    }
    for (long long k = 0; k < steps; ++k) {
      const long long start = k * B;
      const long long bcur = start + B <= n ? B : n - start;
      if (int rc = run_batch(m, n, feats, target, start, bcur, mul, add, true, &t, ++step, nullptr, nullptr, st))
        return rc;
    }
  }
  // bin edges: octiles of the training predictions
  if (int rc = run_predict(m, n, feats, m.cost, st)) return rc;
  if (int rc = run_octiles(m, n, m.cost, m.dedges, st)) return rc;
  MTRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  MTRY(hipMemcpy(m.edges, m.dedges, 7 * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  float norm[8];
  MTRY(hipMemcpy(norm, m.norm, sizeof(norm), hipMemcpyDeviceToHost), "hipMemcpy");
  for (int c = 0; c < kIn; ++c) {
    m.mu[c] = norm[c];
    m.sd[c] = norm[kIn + c];
  }
  m.has_params = true;
  m.has_edges = true;
  return 0;
}

int predict(Model& m, long long n, const float* feats, float* pred, hipStream_t st) {
  if (!m.has_params) return fail(CHEM_ESTATE, "model has no weights (train, load or set them first)");
  return run_predict(m, n, feats, pred, st);
}

int grad(Model& m, long long n, const float* feats, const float* target, float* g, float* loss, hipStream_t st) {
  if (!m.has_params) return fail(CHEM_ESTATE, "model has no weights (train, load or set them first)");
  if (n > 0x7fffffffLL) return fail(CHEM_EINVAL, "too many samples");
  return run_batch(m, n, feats, target, 0, n, 1, 0, false, nullptr, 0, g, loss, st);
}

int get_params(const Model& m, float* params, float* norm, float* edges) {
  if (!m.has_params) return fail(CHEM_ESTATE, "model has no weights");
  if (params) MTRY(hipMemcpy(params, m.master, kParams * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  if (norm) {
    std::memcpy(norm, m.mu, sizeof(m.mu));
    std::memcpy(norm + kIn, m.sd, sizeof(m.sd));
  }
  if (edges) {
    if (!m.has_edges) return fail(CHEM_ESTATE, "model has no bin edges");
    std::memcpy(edges, m.edges, sizeof(m.edges));
  }
  return 0;
}

int set_params(Model& m, const float* params, const float* norm, const float* edges) {
  if (!params) return fail(CHEM_EINVAL, "set_params: null weights");
  if (int rc = ensure_core(m)) return rc;
  std::vector<uint16_t> wb(kParams + 3, 0);
  for (int p = 0; p < kParams; ++p) {
    uint32_t u;
    std::memcpy(&u, &params[p], 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      wb[p] = 0x7fc0;
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      wb[p] = static_cast<uint16_t>(u >> 16);
    }
  }
  float nv[8];
  for (int c = 0; c < kIn; ++c) {
    nv[c] = norm ? norm[c] : 0.f;
    nv[kIn + c] = norm ? norm[kIn + c] : 1.f;
    m.mu[c] = nv[c];
    m.sd[c] = nv[kIn + c];
  }
  MTRY(hipMemcpy(m.master, params, kParams * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  MTRY(hipMemcpy(m.wbf16, wb.data(), kParams * sizeof(uint16_t), hipMemcpyHostToDevice), "hipMemcpy");
  MTRY(hipMemcpy(m.norm, nv, sizeof(nv), hipMemcpyHostToDevice), "hipMemcpy");
  MTRY(hipMemset(m.adam_m, 0, kParams * sizeof(float)), "hipMemset");
  MTRY(hipMemset(m.adam_v, 0, kParams * sizeof(float)), "hipMemset");
  m.has_params = true;
  m.has_edges = edges != nullptr;
  if (edges) {
    std::memcpy(m.edges, edges, sizeof(m.edges));
    MTRY(hipMemcpy(m.dedges, m.edges, sizeof(m.edges), hipMemcpyHostToDevice), "hipMemcpy");
  }
  return 0;
}

int octiles(Model& m, long long n, const float* cost, float* edges, hipStream_t st) {
  if (n < 1 || n > 0x7fffffffLL) return fail(CHEM_EINVAL, "octiles: bad size");
  if (int rc = ensure_core(m)) return rc;
  if (int rc = run_octiles(m, n, cost, m.dedges + 0, st)) return rc;
  MTRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  float e[8];
  MTRY(hipMemcpy(e, m.dedges, 7 * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  std::memcpy(edges, e, 7 * sizeof(float));
  // restore the model's own edges on the device
  if (m.has_edges) MTRY(hipMemcpy(m.dedges, m.edges, sizeof(m.edges), hipMemcpyHostToDevice), "hipMemcpy");
  return 0;
}

int order(Model& m, long long n, const float* cost, const float* edges, int* perm, hipStream_t st) {
  if (n < 1 || n > 0x7fffffffLL) return fail(CHEM_EINVAL, "order: bad size");
  Edges E;
  if (edges) {
    std::memcpy(E.e, edges, sizeof(E.e));
  } else {
    if (!m.has_edges) return fail(CHEM_ESTATE, "model has no bin edges");
    std::memcpy(E.e, m.edges, sizeof(E.e));
  }
  if (int rc = reserve(m, n)) return rc;
  return run_order(m, n, cost, E, perm, st);
}

int plan(Model& m, const chemk::MechArgs& ma, long long n, double dt, const double* phi, const float* over,
         hipStream_t st, const int** perm, int* used) {
  *perm = nullptr;
  *used = 0;
  if (!m.has_edges || (!over && !m.has_params)) return 0;
  if (m.cap < n || m.counts_cap < (n + kBinBlock - 1) / kBinBlock)
    return fail(CHEM_ESTATE, "binning buffers not reserved for this many cells");
  Edges E;
  std::memcpy(E.e, m.edges, sizeof(E.e));
  const float* cost = over;
  if (!over) {
    if (int rc = features(ma, n, dt, phi, m.feats, st)) return rc;
    if (int rc = run_predict(m, n, m.feats, m.cost, st)) return rc;
    cost = m.cost;
  }
  if (int rc = run_order(m, n, cost, E, m.perm, st)) return rc;
  *perm = m.perm;
  *used = 1;
  return 0;
}

int last_plan_finite(const Model& m, int* finite) {
  *finite = 0;
  if (!m.counts || m.last_nblk < 1) return 0;
  int f = 0;
  MTRY(hipMemcpy(&f, m.counts + m.last_nblk * (9 + kBins), sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
  *finite = f;
  return 0;
}

namespace {
constexpr char kMagic[8] = {'C', 'H', 'E', 'M', 'M', 'L', 'P', '1'};
}

int save(const Model& m, const char* path) {
  if (!m.has_params) return fail(CHEM_ESTATE, "model has no weights");
  std::vector<float> p(kParams);
  MTRY(hipMemcpy(p.data(), m.master, kParams * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(CHEM_EINVAL, std::string("cannot write ") + path);
  const uint32_t flags = m.has_edges ? 1u : 0u;
  const uint32_t np = kParams;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 && std::fwrite(&flags, 4, 1, f) == 1 &&
            std::fwrite(p.data(), 4, kParams, f) == static_cast<size_t>(kParams) &&
            std::fwrite(m.mu, 4, kIn, f) == kIn && std::fwrite(m.sd, 4, kIn, f) == kIn &&
            std::fwrite(m.edges, 4, kBins - 1, f) == kBins - 1;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? 0 : fail(CHEM_EINVAL, std::string("write failed: ") + path);
}

int load(Model& m, const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(CHEM_EINVAL, std::string("cannot read ") + path);
  char magic[8];
  uint32_t np = 0, flags = 0;
  std::vector<float> p(kParams);
  float mu[kIn], sd[kIn], ed[kBins - 1];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(&np, 4, 1, f) == 1 &&
            np == static_cast<uint32_t>(kParams) && std::fread(&flags, 4, 1, f) == 1 &&
            std::fread(p.data(), 4, kParams, f) == static_cast<size_t>(kParams) &&
            std::fread(mu, 4, kIn, f) == kIn && std::fread(sd, 4, kIn, f) == kIn &&
            std::fread(ed, 4, kBins - 1, f) == kBins - 1;
  std::fclose(f);
  if (!ok) return fail(CHEM_EINVAL, std::string("not a cost-model file: ") + path);
  float norm[8];
  std::memcpy(norm, mu, sizeof(mu));
  std::memcpy(norm + kIn, sd, sizeof(sd));
  return set_params(m, p.data(), norm, (flags & 1u) ? ed : nullptr);
}

}  // namespace chem_model
