// Zonal reference mapping around the integrator (paper: Methodology, the
// DLBFoam paragraph), read as follows:
// - Z is Bilger's mixture fraction, a linear function of the mass fractions:
//     beta(Y) = sum_i Y_i b_i,  b_i = (sum_e coupling_e a_{e,i}) / W_i,
//     Z = (beta - beta_ox) / (beta_fuel - beta_ox);
// - the zone is every cell with Z <= z_max. It is one band, or with a band
//   width dz > 0 the bands b = floor(max(Z, 0) / dz), so that cells are mapped
//   only from a reference of similar Z. Each band's reference is its cell of
//   lowest index;
// - a zone cell within t_tol of its band reference's temperature is mapped:
//   it takes the reference's change of T and Y over the step. Every other
//   cell is integrated.
//
// All of this is streaming work next to the integration: one thread per cell
// or per element, except the classification, which stages rows through LDS so
// that its loads coalesce. Z is summed in natural
// species order with one fused multiply-add per term, so that a cell's zone
// decision does not depend on how the work is split.
#include "zonal.hpp"

namespace chemz {
namespace {

constexpr unsigned long long kNone = ~0ull;
constexpr int kThreads = 256;

__device__ __forceinline__ double beta_of(const double* Y, const double* coef, int ns) {
  double b = 0.0;
  for (int i = 0; i < ns; ++i) b = fma(Y[i], coef[i], b);
  return b;
}

__device__ __forceinline__ double z_of(const double* Y, const double* coef, int ns, const double* streams) {
  const double bf = streams[0], bo = streams[1];
  return (beta_of(Y, coef, ns) - bo) / (bf - bo);
}

__global__ void k_zone_setup(int ns, int ne, const double* coupling, const int* counts, const double* W,
                             const double* yf, const double* yo, double* coef, double* streams) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int i = 0; i < ns; ++i) {
    double s = 0.0;
    for (int e = 0; e < ne; ++e) s = fma(coupling[e], static_cast<double>(counts[i * ne + e]), s);
    coef[i] = s / W[i];
  }
  streams[0] = beta_of(yf, coef, ns);
  streams[1] = beta_of(yo, coef, ns);
}

__global__ void k_mixture_fraction(long long n, int ns, const double* phi, const double* coef,
                                   const double* streams, double* z) {
  const long long c = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  if (c < n) z[c] = z_of(phi + c * (ns + 2) + 2, coef, ns, streams);
}

__global__ void k_zone_reset(unsigned long long* ctl) {
  if (blockIdx.x == 0 && threadIdx.x < kMaxBands) ctl[threadIdx.x] = kNone;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl[kMaxBands] = 0;
}

// Band flag of one cell, and one atomic per band present in the wave for the
// references: the lowest lane of a band holds the wave's lowest cell of it.
__device__ __forceinline__ void classify_one(const ZoneArgs& a, long long c, double z) {
  const bool zone = c < a.n && z <= a.z_max;
  int band = -1;
  if (zone) band = a.dz > 0.0 ? min(static_cast<int>(floor(fmax(z, 0.0) / a.dz)), a.nb - 1) : 0;
  if (c < a.n) a.flag[c] = static_cast<signed char>(band + 1);
  unsigned long long m = __ballot(zone);
  const unsigned long long lane = static_cast<unsigned long long>(__lane_id());
  while (m) {                       // wave-uniform loop over the bands present
    const int lead = __builtin_ctzll(m);
    const int b = __shfl(band, lead);
    const unsigned long long same = __ballot(band == b);
    if (lane == static_cast<unsigned long long>(lead)) atomicMin(a.ctl + b, static_cast<unsigned long long>(c));
    m &= ~same;
  }
}

// Each thread walks its own row (used above kStageMaxNs species).
__global__ void k_zone_classify(ZoneArgs a) {
  const long long c = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  const double z = c < a.n ? z_of(a.phi_in + c * (a.ns + 2) + 2, a.coef, a.ns, a.streams) : 0.0;
  classify_one(a, c, z);
}

// One block per 64 consecutive cells: their rows, contiguous in HBM, are
// loaded 16 bytes per thread by all four waves, coalesced, into LDS (mass
// fractions only; the row stride is padded to an odd number of doubles so
// that a lane-per-row read spreads over the banks). Wave 0 then sums each
// row in species order, the same chain as the row walk.
constexpr int kStageMaxNs = 127;    // 64 rows of at most 127 doubles: < 64 KB
constexpr int kStageThreads = 256;
__global__ void __launch_bounds__(kStageThreads) k_zone_classify_staged(ZoneArgs a) {
  extern __shared__ double Ys[];    // [64][ns | 1]
  const int ns = a.ns, stride = ns + 2, ls = ns | 1;
  const long long c0 = static_cast<long long>(blockIdx.x) * 64;
  const long long rows = min(64LL, a.n - c0);
  const int t = threadIdx.x;
  // rows hold an even number of doubles and phi is 16-byte aligned, so the
  // block's span is a whole number of 16-byte pairs, none split across rows
  const double2* src = reinterpret_cast<const double2*>(a.phi_in + c0 * stride);
  const int pairs = static_cast<int>(rows) * stride / 2;
  // Row of element e: e < 64 * 129 and the distance from (e + 0.5) / stride
  // to the nearest integer is at least 0.5 / stride, far above the float
  // error of the product, so truncation gives floor(e / stride).
  const float inv = 1.0f / static_cast<float>(stride);
  constexpr int kBatch = 8;   // loads in flight per thread before their stores
  for (int q0 = t; q0 < pairs; q0 += kBatch * kStageThreads) {
    double2 v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = q0 + j * kStageThreads;
      if (q < pairs) v[j] = src[q];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = q0 + j * kStageThreads;
      if (q < pairs) {
        const int e = 2 * q;
        const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv);
        const int k = e - r * stride;   // even: k and k + 1 are in row r
        if (k >= 2) {
          Ys[r * ls + k - 2] = v[j].x;
          Ys[r * ls + k - 1] = v[j].y;
        }
      }
    }
  }
  __syncthreads();
  if (t >= 64) return;
  double z = 0.0;
  if (t < rows) {
    const double bf = a.streams[0], bo = a.streams[1];
    double b = 0.0;
    for (int i = 0; i < ns; ++i) b = fma(Ys[t * ls + i], a.coef[i], b);
    z = (b - bo) / (bf - bo);
  }
  classify_one(a, c0 + t, z);
}

// Mapped flags and the queue order of the integrated cells: each wave claims
// a run of positions, counted down from the end of order, with one atomic.
__global__ void k_zone_select(ZoneArgs a) {
  const long long c = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  const int stride = a.ns + 2;
  bool mapped = false;
  if (c < a.n) {
    const int b = a.flag[c] - 1;
    if (b >= 0) {
      // every zone band has a reference: the lowest of its cells
      const unsigned long long ref = a.ctl[b];
      if (static_cast<unsigned long long>(c) == ref) {
        for (int k = 0; k < stride; ++k) a.stash[b * stride + k] = a.phi_in[c * stride + k];
      } else {
        mapped = fabs(a.phi_in[c * stride] - a.phi_in[static_cast<long long>(ref) * stride]) <= a.t_tol;
      }
    }
    if (!mapped) a.flag[c] = 0;
  }
  const bool keep = c < a.n && !mapped;
  const unsigned long long m = __ballot(keep);
  const int lane = __lane_id();
  unsigned long long base = 0;
  if (lane == 0 && m) base = atomicAdd(a.ctl + kMaxBands, static_cast<unsigned long long>(__popcll(m)));
  base = __shfl(base, 0);
  if (keep) {
    const unsigned long long k = base + static_cast<unsigned long long>(__popcll(m & ((1ull << lane) - 1ull)));
    a.order[a.n - 1 - static_cast<long long>(k)] = static_cast<int>(c);
  }
}

// The persistent kernel pulls queue positions from head up to n: start it at
// the first integrated cell.
__global__ void k_zone_head(long long n, const unsigned long long* ctl, unsigned long long* head) {
  if (blockIdx.x == 0 && threadIdx.x == 0) head[0] = static_cast<unsigned long long>(n) - ctl[kMaxBands];
}

// One thread per element of a mapped cell's row: T and Y move by the
// reference's change, p stays; no steps counted, the reference's status.
__global__ void k_zone_apply(ZoneArgs a) {
  const int stride = a.ns + 2;
  const long long total = a.n * stride;
  for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long c = e / stride;
    const int b = a.flag[c] - 1;     // mapped cells only: their band has a reference
    if (b < 0) continue;
    const unsigned long long ref = a.ctl[b];
    const long long r0 = static_cast<long long>(ref) * stride;
    const int k = static_cast<int>(e - c * stride);
    const double x = a.phi_in[e];
    a.phi_out[e] = k == 1 ? x : x + (a.phi_out[r0 + k] - a.stash[b * stride + k]);
    if (k == 0) {
      if (a.n_acc) a.n_acc[c] = 0;
      if (a.n_rej) a.n_rej[c] = 0;
      if (a.n_jac) a.n_jac[c] = 0;
      if (a.n_fev) a.n_fev[c] = 0;
      if (a.status) a.status[c] = a.status[ref];
    }
  }
}

unsigned grid_for(long long n) {
  return static_cast<unsigned>((n + kThreads - 1) / kThreads);
}

}  // namespace

hipError_t launch_zone_setup(int ns, int ne, const double* coupling, const int* counts, const double* W,
                             const double* y_fuel, const double* y_ox, double* coef, double* streams,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_zone_setup, dim3(1), dim3(64), 0, st, ns, ne, coupling, counts, W, y_fuel, y_ox, coef,
                     streams);
  return hipGetLastError();
}

hipError_t launch_mixture_fraction(long long n, int ns, const double* phi, const double* coef,
                                   const double* streams, double* z, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mixture_fraction, dim3(grid_for(n)), dim3(kThreads), 0, st, n, ns, phi, coef, streams, z);
  return hipGetLastError();
}

hipError_t launch_zone_classify(const ZoneArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zone_reset, dim3(1), dim3(64), 0, st, a.ctl);
  if (hipError_t e = hipGetLastError()) return e;
  if (a.n <= 0) return hipSuccess;
  const bool aligned = (reinterpret_cast<uintptr_t>(a.phi_in) & 15) == 0;
  if (a.ns <= kStageMaxNs && a.ns % 2 == 0 && aligned) {
    const size_t lds = sizeof(double) * 64 * (a.ns | 1);
    hipLaunchKernelGGL(k_zone_classify_staged, dim3(static_cast<unsigned>((a.n + 63) / 64)), dim3(kStageThreads),
                       lds, st, a);
  } else {
    hipLaunchKernelGGL(k_zone_classify, dim3(grid_for(a.n)), dim3(kThreads), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_zone_select(const ZoneArgs& a, hipStream_t st) {
  if (a.n > 0) {
    hipLaunchKernelGGL(k_zone_select, dim3(grid_for(a.n)), dim3(kThreads), 0, st, a);
    if (hipError_t e = hipGetLastError()) return e;
  }
  hipLaunchKernelGGL(k_zone_head, dim3(1), dim3(64), 0, st, a.n, a.ctl, a.head);
  return hipGetLastError();
}

hipError_t launch_zone_apply(const ZoneArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  long long blocks = (a.n * (a.ns + 2) + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zone_apply, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace chemz
