// Per-cell stiff chemistry integration for mechanisms too large for one
// wave (n = Ns + 1 up to 256): one workgroup of 256 threads per cell.
//
// The Jacobian J and the Rosenbrock matrix M = I/(gamma h) - J of a
// 160-species cell are 161 x 161 FP64 (207 KB each): they fit neither one
// wave's registers nor the 160 KB LDS of a CU. Each resident workgroup
// therefore owns a workspace slot in HBM holding J and the LU factors of M
// (column-major, leading dimension ld); the number of slots, and so of cells
// in flight, is bounded by the HBM budget. Everything else of the cell
// (state, stage vectors, concentrations, per-reaction rates) lives in LDS.
//
// The LU is a left-looking blocked getrf that never moves a row in HBM:
// the row interchanges are kept as a permutation, so physical row q of M
// stays at offset q of every column. Panel by panel (12 columns), the panel
// is first brought up to date with every finished column to its left, each
// wave holding three of its columns in registers while the finished columns
// stream through LDS twelve at a time; the four waves then factor the panel
// with one row per lane and write it back. Every element sees the same
// sequence of operations as in an unblocked row-swapping LU, in the same
// order, so the factors do not depend on the blocking.

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace chemk {

namespace {

using namespace dev;

constexpr int kT = kWideThreads;
constexpr int kNB = kWidePanel;
// The LU's blocks sit in LDS as rows of kNB doubles at a stride of kLS: 14
// rather than 12 spreads the transposed stores of consecutive row pairs over
// more LDS banks, and keeps every row 16-byte aligned.
constexpr int kLS = 14;

// Per-cell LDS area. Region A (right-hand-side buffers) and region B (the
// LU's two 12-column buffers) are never live at the same time and share
// storage; so do the stage input ys and the solve right-hand side v, and the
// stage derivative fs and the trial state yn.
struct Wide {
  double *C, *gRT, *hRT, *RB;                   // A: ns, ns, ns, 5 nr
  double *buf0, *buf1;                          // B: the LU's two 12-column buffers, kLS ld each
  double *y, *f0, *fs, *ys, *yn, *v, *u[4];     // 8 distinct vectors of ld
  double* red;                                  // 16
  double* ub;                                   // 144: per wave, 12 x 3 values of the LU's U block
  int* piv;                                     // ld: getrf's interchange at each step
  int* perm;                                    // ld: physical row of each logical row
  int* pos;                                     // ld: logical row of each physical row (-1 beyond n)
  int* ired;                                    // 16
  int* zpm;                                     // 32: zero-pivot columns, one 12-bit mask per panel
  unsigned long long* qslot;                    // 1
};

__host__ __device__ inline int wide_region(int ns, int nr, int ld) {
  const int a = 3 * ns + 5 * nr;
  const int b = 2 * kLS * ld;
  return ((a > b ? a : b) + 1) & ~1;
}

// doubles: region, 8 vectors, reduction scratch, U block; ints: piv, perm,
// pos, ired, zpm; one 64-bit queue slot
__host__ __device__ inline int wide_doubles(int ns, int nr, int ld) {
  return wide_region(ns, nr, ld) + 8 * ld + 16 + 144 + (3 * ld + 48) / 2 + 2;
}

__device__ inline Wide wide_area(double* base, int ns, int nr, int ld) {
  Wide W;
  W.C = base;
  W.gRT = W.C + ns;
  W.hRT = W.gRT + ns;
  W.RB = W.hRT + ns;
  W.buf0 = base;
  W.buf1 = base + kLS * ld;
  double* q = base + wide_region(ns, nr, ld);
  W.y = q;
  W.f0 = q + ld;
  W.fs = q + 2 * ld;
  W.yn = W.fs;
  W.v = q + 3 * ld;
  W.ys = W.v;
  for (int k = 0; k < 4; ++k) W.u[k] = q + (4 + k) * ld;
  W.red = q + 8 * ld;
  W.ub = W.red + 16;
  int* ip = reinterpret_cast<int*>(W.ub + 144);
  W.piv = ip;
  W.perm = ip + ld;
  W.pos = ip + 2 * ld;
  W.ired = ip + 3 * ld;
  W.zpm = ip + 3 * ld + 16;
  W.qslot = reinterpret_cast<unsigned long long*>(ip + 3 * ld + 48);
  return W;
}

// ---- workgroup sum (fixed pairing: butterfly in the wave, then waves
// (0+1)+(2+3)); every thread receives the same value ----
__device__ __forceinline__ double bsum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Loads of J for the chain rule, in batches of kJB: species rows of column t
// (row t of the species block) or of row t (column t); indices past the last
// species read the last one (such values are never used), so that every
// load is issued and each wait covers one batch. The start passes through an
// empty asm so that the addresses are formed here.
constexpr int kJB = 16;
__device__ __forceinline__ void jrow_load(const double* J, int ns, int ld, int t, int k0, double (&v)[kJB]) {
  asm volatile("" : "+s"(k0));
#pragma unroll
  for (int q = 0; q < kJB; ++q) v[q] = J[(1 + min(k0 + q, ns - 1)) * ld + t];
}
__device__ __forceinline__ void jcol_load(const double* J, int ns, int ld, int t, int q0, double (&v)[kJB]) {
  asm volatile("" : "+s"(q0));
#pragma unroll
  for (int q = 0; q < kJB; ++q) v[q] = J[t * ld + 1 + min(q0 + q, ns - 1)];
}

// ---- right-hand side and analytical Jacobian ----------------------------------
// f = dy/dt at y (LDS vector); with JAC also J = df/dy, column-major in HBM:
// element (i, j) at J[j * ld + i]. Thread t owns state component t (0 = T,
// t = 1..Ns species t-1) and, for the Jacobian, row t.
template <bool JAC>
__device__ __forceinline__ void rhs_w(const MechArgs& A, const MechLds& L, const Wide& W, double p, const double* yv, double* fout,
                      double* J, int ld) {
  const int ns = A.ns, nr = A.nr, n = ns + 1;
  const int t = threadIdx.x;
  const bool sp = t >= 1 && t <= ns;
  const int s = sp ? t - 1 : 0;
  const double T = yv[0];
  const double rT = 1.0 / T;
  const double lnT = log(T);
  const double Ys = sp ? yv[t] : 0.0;
  const double rWs = sp ? L.rW[s] : 0.0;
  const double invWbar = bsum(Ys * rWs, W.red);
  const double Wbar = 1.0 / invWbar;
  const double rho = p * Wbar / (kR * T);
  const double Cs = rho * Ys * rWs;
  if (sp) W.C[s] = Cs;
  const double Ctot = bsum(Cs, W.red);
  double cpR = 0.0, hRT = 0.0, dcpR = 0.0;
  if (sp) {
    double gRT;
    nasa7<JAC>(A.nasa + 16 * s, T, rT, lnT, cpR, hRT, gRT, dcpR);
    W.gRT[s] = gRT;
    W.hRT[s] = hRT;
  }
  const double cp = bsum(Ys * cpR * kR * rWs, W.red);
  double dcp = 0.0;
  if (JAC) {
    dcp = bsum(Ys * dcpR * kR * rWs, W.red);
    if (t < ld)
      for (int c = 0; c < n; ++c) J[c * ld + t] = 0.0;
  }
  __syncthreads();
  const double lnRTp = log(kR * T / kPatm);
  for (int rx = t; rx < nr; rx += kT) reaction_rate<JAC>(L, W.C, W.gRT, W.hRT, W.RB, nr, rx, T, rT, lnT, lnRTp, Ctot);
  __syncthreads();

  // species: production rates and, with JAC, the rows d(omega)/dC. Thread t
  // alone adds to row t, with atomic adds that return nothing (nothing waits
  // on them; one thread's adds to one address apply in program order).
  double om = 0.0, wT = 0.0, td = 0.0;
  if (sp) {
    const int e0 = L.sp_off[s], e1 = L.sp_off[s + 1];
    if (!JAC) {
      for (int e = e0; e < e1; ++e) {
        const unsigned ent = L.sp_ent[e];
        const double nu = static_cast<double>(static_cast<int>(ent >> 12) - 8);
        om = om + nu * W.RB[ent & 0xfff];
      }
    } else {
      double* Jr = J + t;
      for (int e = e0; e < e1; ++e) {
        const unsigned ent = L.sp_ent[e];
        const int rx = ent & 0xfff;
        const double nu = static_cast<double>(static_cast<int>(ent >> 12) - 8);
        const uint4 wc = L.rint[rx];
        const double qr = W.RB[rx], kfT = W.RB[nr + rx], krT = W.RB[2 * nr + rx];
        const double q0b = W.RB[3 * nr + rx], dqdT = W.RB[4 * nr + rx];
        const int nre = (wc.x >> 24) & 0xf, npr = (wc.y >> 24) & 0xf;
        double Pf, Pr, dPf[3], dPr[3];
        int sf[3], sr[3];
        mass_action(W.C, wc.x, wc.z, nre, Pf, dPf, sf);
        mass_action(W.C, wc.y, wc.z >> 12, npr, Pr, dPr, sr);
        om = om + nu * qr;
        wT = wT + nu * dqdT;
        const double af = nu * kfT, ar = nu * krT;
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (j < nre) unsafeAtomicAdd(&Jr[(1 + sf[j]) * ld], af * dPf[j]);
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (j < npr) unsafeAtomicAdd(&Jr[(1 + sr[j]) * ld], -(ar * dPr[j]));
        const int type = (wc.x >> 28) & 3;
        if (type >= 1) {
          const double ab = nu * q0b;
          td = td + ab;
          const int eoff = wc.w & 0xffff, neff = (wc.w >> 16) & 0xff;
          for (int q = 0; q < neff; ++q) unsafeAtomicAdd(&Jr[(1 + L.eff_sp[eoff + q]) * ld], ab * L.eff_am1[eoff + q]);
        }
      }
    }
  }
  const double fY = sp ? A.W[s] * om / rho : 0.0;
  const double Q = bsum(hRT * kR * T * om, W.red);
  const double rcp = rho * cp;
  const double fT = -Q / rcp;
  if (t < n) fout[t] = (t == 0) ? fT : fY;
  if (!JAC) {
    __syncthreads();
    return;
  }

  // chain rule from d(omega)/dC and d(omega)/dT to y = (T, Y): the adds
  // complete (release), then every thread sees them past its L1 (acquire)
  __threadfence();
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double sv = 0.0;
  if (sp) {
    // four accumulators (k mod 4); batches of kJB loads, the next batch in
    // flight while one is used
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    double v0[kJB], v1[kJB];
    jrow_load(J, ns, ld, t, 0, v0);
    for (int k0 = 0; k0 < ns; k0 += 2 * kJB) {
      jrow_load(J, ns, ld, t, k0 + kJB, v1);
#pragma unroll
      for (int q = 0; q < kJB; ++q)
        if (k0 + q < ns) a[q & 3] = fma(v0[q], W.C[k0 + q], a[q & 3]);
      jrow_load(J, ns, ld, t, k0 + 2 * kJB, v0);
#pragma unroll
      for (int q = 0; q < kJB; ++q)
        if (k0 + kJB + q < ns) a[q & 3] = fma(v1[q], W.C[k0 + kJB + q], a[q & 3]);
    }
    sv = ((a[0] + a[1]) + (a[2] + a[3])) + td * Ctot;
  }
  const double HS = bsum(hRT * sv, W.red);
  const double HT = bsum(hRT * td, W.red);
  const double dQdT = bsum(sp ? cpR * kR * om + hRT * kR * T * (wT - sv / T) : 0.0, W.red);
  double JT = 0.0;
  if (sp) {
    // column t, rows 1..ns
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    double v0[kJB], v1[kJB];
    jcol_load(J, ns, ld, t, 0, v0);
    for (int q0 = 0; q0 < ns; q0 += 2 * kJB) {
      jcol_load(J, ns, ld, t, q0 + kJB, v1);
#pragma unroll
      for (int q = 0; q < kJB; ++q)
        if (q0 + q < ns) c[q & 3] = fma(W.hRT[q0 + q], v0[q], c[q & 3]);
      jcol_load(J, ns, ld, t, q0 + 2 * kJB, v0);
#pragma unroll
      for (int q = 0; q < kJB; ++q)
        if (q0 + kJB + q < ns) c[q & 3] = fma(W.hRT[q0 + kJB + q], v1[q], c[q & 3]);
    }
    const double cs = (c[0] + c[1]) + (c[2] + c[3]);
    const double dQdY = kR * T * ((rho * rWs) * (cs + HT) - (Wbar * rWs) * HS);
    const double drcp = rho * cpR * kR * rWs - rcp * Wbar * rWs;
    JT = -(dQdY + fT * drcp) / rcp;
  }
  __syncthreads();
  if (sp) {
    const double Wi_rho = A.W[s] / rho;
    // the next batch is loaded before this one is written back; the two
    // never overlap (a clamped load past the last species is not used)
    auto upd = [&](const double (&v)[kJB], int k0) {
#pragma unroll
      for (int q = 0; q < kJB; ++q) {
        const int k = k0 + q;
        if (k < ns) {
          const double rWk = L.rW[k];
          const double D = v[q] + td;
          const double dw = (rho * rWk) * D - (Wbar * rWk) * sv;
          J[(1 + k) * ld + t] = Wi_rho * dw + fY * Wbar * rWk;
        }
      }
    };
    double v0[kJB], v1[kJB];
    jrow_load(J, ns, ld, t, 0, v0);
    for (int k0 = 0; k0 < ns; k0 += 2 * kJB) {
      jrow_load(J, ns, ld, t, k0 + kJB, v1);
      upd(v0, k0);
      jrow_load(J, ns, ld, t, k0 + 2 * kJB, v0);
      upd(v1, k0 + kJB);
    }
    J[t] = Wi_rho * (wT - sv / T) + fY / T;   // (t, 0)
    J[t * ld] = JT;                           // (0, t)
  } else if (t == 0) {
    const double drcp = -rcp / T + rho * dcp;
    J[0] = -(dQdT + fT * drcp) / rcp;
  }
  __syncthreads();
}

// The per-cell area is LDS; pointers into it are generic in the Wide struct.
// Converted to the LDS address space, accesses compile to LDS instructions
// (not flat ones, whose completion is counted together with global loads)
// even where the compiler cannot trace them to the shared array.
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) T* lds(T* p) {
  return (__attribute__((address_space(3))) T*)p;
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(3))) T* lds(const T* p) {
  return (const __attribute__((address_space(3))) T*)p;
}
// a pair of doubles as a native vector (128-bit LDS and global accesses)
typedef double dv2 __attribute__((ext_vector_type(2)));
// the same for the workspace slot in HBM (global loads and stores)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glb(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* glb(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// ---- wave-wide primitives (all 64 lanes active) ---------------------------------
__device__ __forceinline__ double rl_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
// every pattern reads a lane inside the same DPP row
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
// into the rows of ROWMASK only (the others keep old)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_rows_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xf, false);
}
// xor 1, xor 2, the 8- and 16-lane mirrors inside a row, then rows 1 and 3
// take lane 15 of the row below and rows 2 and 3 lane 31: lane 63 ends with
// the result
__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dppd<0xB1>(x));
  x = fmax(x, dppd<0x4E>(x));
  x = fmax(x, dppd<0x141>(x));
  x = fmax(x, dppd<0x140>(x));
  x = fmax(x, dpp_rows<0x142, 0xA>(x, x));
  x = fmax(x, dpp_rows<0x143, 0xC>(x, x));
  return rl_d(x, 63);
}
__device__ __forceinline__ int wave_min(int x) {
  x = ::min(x, dppi<0xB1>(x));
  x = ::min(x, dppi<0x4E>(x));
  x = ::min(x, dppi<0x141>(x));
  x = ::min(x, dppi<0x140>(x));
  x = ::min(x, dpp_rows_i<0x142, 0xA>(x, x));
  x = ::min(x, dpp_rows_i<0x143, 0xC>(x, x));
  return __builtin_amdgcn_readlane(x, 63);
}

// an int kept in a double-sized LDS slot (low word), and back
__device__ __forceinline__ double int_in_double(int v) { return __hiloint2double(0, v); }
__device__ __forceinline__ int int_of_double(double d) { return __double2loint(d); }

// ---- blocked LU with partial pivoting ---------------------------------------------
// M: n x n column-major (leading dimension ld) in HBM, overwritten by L (unit
// lower) and U. No row is moved: logical row i of the factors is physical row
// W.perm[i] (offset perm[i] in every column), W.pos is the inverse (-1 beyond
// n), and W.piv[k] is the logical row interchanged with row k at step k
// (getrf's ipiv, from 0). Returns the first zero pivot column + 1 (0 if none);
// such a column is left unreduced and its multipliers are not applied, as
// getrf does.
//
// Register layout: lane l of a wave holds physical rows l + 64 s, s < kRS.
// Panel p (columns k0 .. k0 + nb - 1) is first updated with every finished
// column k < k0, twelve at a time: wave w owns panel columns 3w .. 3w + 2, and
// the twelve finished columns of block b arrive in LDS as rows of twelve
// multipliers (loaded from HBM while the previous block is applied). For
// block b (columns kb .. kb + 11) the twelve rows at logical kb .. kb + 11
// first solve their unit lower triangle (36 lanes, one per row and column,
// the solved value broadcast along each 16-lane row by DPP); every row below
// then subtracts the twelve multiplier-times-U terms in ascending k. The panel
// then goes through LDS to wave 0, which factors it column by column (pivot
// search by DPP reductions, no barrier) and writes it back.
constexpr int kRS = 4;              // row slots per lane: n <= 256
constexpr int kCW = kNB / 4;        // panel columns per wave in the update
constexpr int kPre = 6;             // two-double loads per thread for one 12-column block (ld <= 256)
static_assert(kT == 256 && kNB == 12, "four waves of three panel columns each");

// A finished block for the LU's update (kNB columns of ld from src): pairs of
// rows that lie above the block (logical position < kb, or padding) are not
// used, and read the block's first pair instead, so that every load is
// issued while they cost no memory traffic of their own. mx[i] is the larger
// logical position of this thread's i-th pair of rows (the same rows in every
// block: pair i is element threadIdx.x + kT i of the column-major block).
__device__ __forceinline__ void lu_block_load(const double* src, int cnt2, int kb, const int (&mx)[kPre],
                                              dv2 (&r)[kPre]) {
  asm volatile("" : "+s"(src));   // addresses formed here, not hoisted and spilled
  const auto* s = glb(reinterpret_cast<const dv2*>(src));
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    const int e = min(static_cast<int>(threadIdx.x) + kT * i, cnt2 - 1);
    r[i] = s[mx[i] >= kb ? e : 0];
  }
}
// the block (column-major, kNB columns of ld) into LDS as rows of kNB:
// element (row q, column m) at dst[q * kLS + m]
__device__ __forceinline__ void block_store_t(double* dst, int ld, int cnt2, const dv2 (&r)[kPre]) {
  auto* d = lds(dst);
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    const int e = static_cast<int>(threadIdx.x) + kT * i;
    if (e < cnt2) {
      const int m = (2 * e) / ld, q = 2 * e - m * ld;   // q even, q + 1 < ld
      d[q * kLS + m] = r[i].x;
      d[(q + 1) * kLS + m] = r[i].y;
    }
  }
}

// apply f(row array, slot) to each of the four per-slot arrays by name (an
// array indexed [s][c] with s known only at run time would go to scratch)
template <int C, class F>
__device__ __forceinline__ void each_slot(double (&r0)[C], double (&r1)[C], double (&r2)[C], double (&r3)[C],
                                          F&& f) {
  f(r0, 0);
  f(r1, 1);
  f(r2, 2);
  f(r3, 3);
}

// this wave's panel columns (k0 + 3w + cc) of the matrix, rows beyond n and
// columns beyond the panel as zero. With FORM the source is J and the
// matrix is g I - J, formed here: each column of M is read in its original
// form only once, by this load.
template <bool FORM>
__device__ __forceinline__ void load_cols(double (&a0)[kCW], double (&a1)[kCW], double (&a2)[kCW],
                                          double (&a3)[kCW], const double* Sg, double g, int n, int ld, int k0,
                                          int nb) {
  asm volatile("" : "+s"(k0));    // addresses formed here, not hoisted and spilled
  const auto* S = glb(Sg);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  each_slot(a0, a1, a2, a3, [&](double (&row)[kCW], const int s) {
    const int q = lane + 64 * s;
#pragma unroll
    for (int cc = 0; cc < kCW; ++cc) {
      const int c = kCW * w + cc;
      const double v = (q < n && c < nb) ? S[(k0 + c) * ld + q] : 0.0;
      row[cc] = FORM ? ((q == k0 + c ? g : 0.0) - v) : v;
    }
  });
}

// one 64-bit value of lane SRC of each 16-lane row, to every lane of that row
template <int SRC>
__device__ __forceinline__ double row_share_c(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + SRC, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + SRC, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// the same with src a constant after unrolling
__device__ __forceinline__ double row_share(double v, int src) {
  switch (src) {
    case 0: return row_share_c<0>(v);
    case 1: return row_share_c<1>(v);
    case 2: return row_share_c<2>(v);
    case 3: return row_share_c<3>(v);
    case 4: return row_share_c<4>(v);
    case 5: return row_share_c<5>(v);
    case 6: return row_share_c<6>(v);
    case 7: return row_share_c<7>(v);
    case 8: return row_share_c<8>(v);
    case 9: return row_share_c<9>(v);
    case 10: return row_share_c<10>(v);
    case 11: return row_share_c<11>(v);
    case 12: return row_share_c<12>(v);
    case 13: return row_share_c<13>(v);
    case 14: return row_share_c<14>(v);
    default: return row_share_c<15>(v);
  }
}

// Apply finished block b (its rows of multipliers in Lt, LDS) to this wave's
// panel columns. zm: the block's zero-pivot columns (skipped).
__device__ __forceinline__ void apply_block(double (&A0)[kCW], double (&A1)[kCW], double (&A2)[kCW],
                                            double (&A3)[kCW], const int (&ps)[kRS], const double* Ltg, int kb,
                                            int zm, int n, const Wide& W) {
  using LD = __attribute__((address_space(3))) double;
  using LD2 = __attribute__((address_space(3))) dv2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const LD* Lt = lds(Ltg);
  LD* T = lds(W.ub) + 36 * w;   // this wave's 12 x 3 table
  // the block's own rows (logical kb .. kb + 11) into the table
  // (a slot with no row below n on any lane is skipped: its test is uniform)
  each_slot(A0, A1, A2, A3, [&](double (&row)[kCW], const int s) {
    if (64 * s >= n) return;
    const int m = ps[s] - kb;
    if (m >= 0 && m < kNB) {
#pragma unroll
      for (int cc = 0; cc < kCW; ++cc) T[m * kCW + cc] = row[cc];
    }
  });
  wsync();
  // their unit lower triangle: lane 16 cc + m holds row m, column cc
  const int cc = lane >> 4, m = lane & 15;
  const bool act = cc < kCW && m < kNB;
  double x = act ? T[m * kCW + cc] : 0.0;
  double lr[kNB];
  {
    const int q = act ? lds(W.perm)[kb + m] : 0;
    const LD2* r = reinterpret_cast<const LD2*>(Lt + q * kLS);
#pragma unroll
    for (int j = 0; j < kNB / 2; ++j) {
      const dv2 v = r[j];
      lr[2 * j] = v.x;
      lr[2 * j + 1] = v.y;
    }
  }
#pragma unroll
  for (int j = 0; j + 1 < kNB; ++j) {
    if (((zm >> j) & 1) == 0) {
      const double u = row_share(x, j);
      const double y = x - lr[j] * u;
      x = m > j ? y : x;
    }
  }
  if (act) T[m * kCW + cc] = x;
  wsync();
  // every row below the block: twelve terms in ascending k; the block's own
  // rows take their solved values
  double U[kNB][kCW];
#pragma unroll
  for (int j = 0; j < kNB; ++j)
#pragma unroll
    for (int c = 0; c < kCW; ++c) U[j][c] = T[j * kCW + c];
  each_slot(A0, A1, A2, A3, [&](double (&row)[kCW], const int s) {
    if (64 * s >= n) return;
    const int q = lane + 64 * s;
    const int rel = ps[s] - kb;
    if (rel >= kNB) {
      const LD2* r = reinterpret_cast<const LD2*>(Lt + q * kLS);
      double l[kNB];
#pragma unroll
      for (int j = 0; j < kNB / 2; ++j) {
        const dv2 v = r[j];
        l[2 * j] = v.x;
        l[2 * j + 1] = v.y;
      }
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (((zm >> j) & 1) == 0) {
#pragma unroll
          for (int c = 0; c < kCW; ++c) row[c] = row[c] - l[j] * U[j][c];
        }
      }
    } else if (rel >= 0) {
#pragma unroll
      for (int c = 0; c < kCW; ++c) row[c] = T[rel * kCW + c];
    }
  });
}

// All four waves: factor panel columns k0 .. k0 + nb - 1. The panel arrives in
// LDS as rows of kNB doubles (H[q * kLS + c], physical row q); lane l of wave
// w holds row q = 64 w + l in registers, rotated so that the current column
// is always P[0] (the loop over columns then needs no run-time register
// index). At each column every wave finds its best candidate (DPP
// reductions) and that row's lane writes the candidate's key, code and row to
// the wave's LDS slot (two sets, by column parity); after one barrier every
// lane picks the same winner from the four slots, reads its row (a broadcast)
// and updates its own row. The finished column goes to M; the row shifts by
// one. Entries past the panel's last column are updated too but never stored.
// Writes the positions to W.pos / W.perm.
constexpr int kCand = 2 + kNB;   // per wave and parity: key, code, row entries

__device__ __forceinline__ void factor_panel(double* Mg, const double* Hg, int n, int ld, int k0, int nb,
                                             const Wide& W) {
  using LD = __attribute__((address_space(3))) double;
  using LD2 = __attribute__((address_space(3))) dv2;
  const LD* H = lds(Hg);
  LD* cand = lds(W.ub);   // 2 x 4 x kCand doubles (the U-block tables are idle here)
  auto* M = glb(Mg);
  const int t = threadIdx.x, w = t >> 6;
  const int q = t;        // this lane's physical row
  int pq = q < n ? lds(W.pos)[q] : -1;
  int info = lds(W.ired)[15];
  double P[kNB];
  {
    const LD2* r = reinterpret_cast<const LD2*>(H + (q < n ? q : 0) * kLS);
#pragma unroll
    for (int j = 0; j < kNB / 2; ++j) {
      const dv2 v = r[j];
      P[2 * j] = q < n ? v.x : 0.0;
      P[2 * j + 1] = q < n ? v.y : 0.0;
    }
  }
  for (int c = 0; c < nb; ++c) {
    const int k = k0 + c;
    // first logical row of the largest |a| among rows k..n-1 (a NaN on the
    // diagonal stays the pivot; elsewhere it never wins); code = logical
    // position * 256 + physical row
    const double av = fabs(P[0]);
    const double key = pq < k ? -1.0 : (av != av ? (pq == k ? INFINITY : -1.0) : av);
    const int code = pq * 256 + q;
    const double wkey = wave_max(key);
    const bool tie = key == wkey;
    const unsigned long long bal = __ballot(tie);
    const int wcode = __popcll(bal) == 1
                          ? __builtin_amdgcn_readlane(code, __ffsll(static_cast<long long>(bal)) - 1)
                          : wave_min(tie ? code : 0x7fffffff);
    LD* slot = cand + ((c & 1) * 4 + w) * kCand;
    if (code == wcode) {
      slot[0] = wkey;
      slot[1] = int_in_double(wcode);
      LD2* r2 = reinterpret_cast<LD2*>(slot + 2);
#pragma unroll
      for (int j = 0; j < kNB / 2; ++j) r2[j] = dv2{P[2 * j], P[2 * j + 1]};
    }
    __syncthreads();
    // the winner among the four waves' candidates: largest key, then the
    // smallest code (all four slots' key, code and first two row entries
    // read at once; the choice runs on selects)
    const LD* set = cand + (c & 1) * 4 * kCand;
    dv2 kc[4], a01[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      kc[v] = reinterpret_cast<const LD2*>(set + v * kCand)[0];
      a01[v] = reinterpret_cast<const LD2*>(set + v * kCand)[1];
    }
    double bk = kc[0].x;
    int bc = int_of_double(kc[0].y), bw = 0;
    dv2 ba = a01[0];
#pragma unroll
    for (int v = 1; v < 4; ++v) {
      const double kv = kc[v].x;
      const int cv = int_of_double(kc[v].y);
      const bool better = kv > bk || (kv == bk && cv < bc);
      bk = better ? kv : bk;
      bc = better ? cv : bc;
      bw = better ? v : bw;
      ba.x = better ? a01[v].x : ba.x;
      ba.y = better ? a01[v].y : ba.y;
    }
    bw = __builtin_amdgcn_readfirstlane(bw);
    const int pv = __builtin_amdgcn_readfirstlane(bc) >> 8, qs = __builtin_amdgcn_readfirstlane(bc) & 255;
    if (t == 0) lds(W.piv)[k] = pv;
    if (q == qs) {
      pq = k;
    } else if (pq == k) {
      pq = pv;
    }
    double pr[kNB];
    pr[0] = ba.x;
    pr[1] = ba.y;
    {
      const LD2* r2 = reinterpret_cast<const LD2*>(set + bw * kCand + 2);
#pragma unroll
      for (int j = 1; j < kNB / 2; ++j) {
        const dv2 v = r2[j];
        pr[2 * j] = v.x;
        pr[2 * j + 1] = v.y;
      }
    }
    const double akk = pr[0];
    if (akk == 0.0) {
      if (!info) info = k + 1;
      if (t == 0) lds(W.zpm)[k0 / kNB] |= 1 << c;
    } else if (pq > k) {
      // below the pivot: multiplier, and the multiplier times the pivot
      // row's later entries subtracted
      const double l = P[0] / akk;
      P[0] = l;
#pragma unroll
      for (int j = 1; j < kNB; ++j) P[j] = P[j] - l * pr[j];
    }
    if (q < n) M[k * ld + q] = P[0];
#pragma unroll
    for (int j = 0; j + 1 < kNB; ++j) P[j] = P[j + 1];
    P[kNB - 1] = 0.0;
  }
  if (q < ld) lds(W.pos)[q] = pq;
  if (pq >= 0) lds(W.perm)[pq] = q;
  if (t == 0) lds(W.ired)[15] = info;
}

// With FORM, the matrix is gm I - J (J: n x n, the same layout) and is formed
// from J as its columns are first read; M then receives only the factors.
template <bool FORM>
__device__ __forceinline__ int lu_w(double* M, const double* J, double gm, int n, int ld, const Wide& W) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int np = (n + kNB - 1) / kNB;
  const int cnt2 = kNB * ld / 2;
  auto* pos = lds(W.pos);
  auto* perm = lds(W.perm);
  auto* zpm = lds(W.zpm);
  auto* ired = lds(W.ired);
  if (t < ld) {
    pos[t] = t < n ? t : -1;
    perm[t] = t;
  }
  if (t < 32) zpm[t] = 0;
  if (t == 0) ired[15] = 0;
  double A0[kCW], A1[kCW], A2[kCW], A3[kCW];
  load_cols<FORM>(A0, A1, A2, A3, FORM ? J : M, gm, n, ld, 0, min(kNB, n));
  dv2 R[kPre];
  int g = 0;   // finished blocks applied so far: block g is in buffer g & 1
  __syncthreads();
  for (int p = 0; p < np; ++p) {
    const int k0 = p * kNB, nb = min(kNB, n - k0);
    int ps[kRS];
#pragma unroll
    for (int s = 0; s < kRS; ++s) {
      const int q = lane + 64 * s;
      ps[s] = q < ld ? pos[q] : -1;
    }
    int mx[kPre];   // positions of this thread's pairs of rows in the block loads
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int q = (2 * min(t + kT * i, cnt2 - 1)) % ld;
      mx[i] = max(pos[q], pos[q + 1]);
    }
    // the panel's columns were loaded during the previous factorisation:
    // wait for them here, once, not inside the block loop where the next
    // block's loads are in flight
    each_slot(A0, A1, A2, A3, [&](double (&row)[kCW], const int s) {
#pragma unroll
      for (int cc = 0; cc < kCW; ++cc) asm volatile("" : "+v"(row[cc]));
    });
    if (p == 1) {
      // the first finished block, not loaded ahead
      lu_block_load(M, cnt2, 0, mx, R);
      block_store_t(W.buf0, ld, cnt2, R);
      __syncthreads();
    }
    for (int b = 0; b < p; ++b) {
      const int kb = b * kNB;
      // the next block: (p, b + 1), or the first one of panel p + 1
      const bool more = b + 1 < p || p + 1 < np;
      if (more) lu_block_load(M + (b + 1 < p ? kb + kNB : 0) * ld, cnt2, b + 1 < p ? kb + kNB : 0, mx, R);
      const int zm = __builtin_amdgcn_readfirstlane(zpm[b]);
      apply_block(A0, A1, A2, A3, ps, (g & 1) ? W.buf1 : W.buf0, kb, zm, n, W);
      if (more) block_store_t((g & 1) ? W.buf0 : W.buf1, ld, cnt2, R);
      __syncthreads();
      ++g;
    }
    // the panel to the factorisation, as rows of kNB, through the buffer the
    // last block used
    double* H = (g & 1) ? W.buf0 : W.buf1;
    auto* HL = lds(H);
    each_slot(A0, A1, A2, A3, [&](double (&row)[kCW], const int s) {
      const int q = lane + 64 * s;
#pragma unroll
      for (int cc = 0; cc < kCW; ++cc)
        if (q < n) HL[q * kLS + kCW * w + cc] = row[cc];
    });
    __syncthreads();
    if (p + 1 < np) load_cols<FORM>(A0, A1, A2, A3, FORM ? J : M, gm, n, ld, k0 + kNB, min(kNB, n - k0 - kNB));
    factor_panel(M, H, n, ld, k0, nb, W);
    __syncthreads();
  }
  return ired[15];
}

// x = M^-1 b with the factors of lu_w. b (LDS) is overwritten: the
// substitutions run in place in physical row order; x (LDS, distinct from b)
// receives the solution. Forward substitution in blocks of kSB columns (each
// element receives its terms in ascending column order), then backward in
// blocks from the bottom. Every thread loads its own physical row's entries
// in the block's columns, two blocks ahead (three register sets, loads
// issued unconditionally so that each wait is for one set only). The rows
// inside the block hand theirs to wave 0 through LDS; wave 0 solves the
// block's triangle on lanes 0..15, the solved value of each step broadcast
// along them by DPP (row_newbcast; the backward steps multiply by the
// diagonal's reciprocal); every thread then updates its row.
constexpr int kSB = 16;

// row t's entries in columns k0 .. k0 + kSB - 1 when the row takes part in
// the block (need); columns past n - 1 read column n - 1, and rows that do not
// take part read row 0, so that every load is issued (each wait then covers
// one register set) while the rows left out cost no memory traffic of their
// own; such values are never used. k0 passes through an empty asm so that
// the addresses are formed here, not hoisted out of the loops and spilled.
__device__ __forceinline__ void solve_load(const double* Mg, int n, int ld, int k0, bool need, double (&v)[kSB]) {
  asm volatile("" : "+s"(k0));
  const auto* M = glb(Mg) + (need ? threadIdx.x : 0);
#pragma unroll
  for (int j = 0; j < kSB; ++j) v[j] = M[min(k0 + j, n - 1) * ld];
}

template <bool FWD>
__device__ __forceinline__ void solve_block(int k0, int n, int pt, const double (&v)[kSB], const Wide& W,
                                            __attribute__((address_space(3))) double* b) {
  using LD = __attribute__((address_space(3))) double;
  using LD2 = __attribute__((address_space(3))) dv2;
  const int t = threadIdx.x;
  const int nb = min(kSB, n - k0);
  LD* T = lds(W.buf1);                  // the block rows' entries, kSB x kSB
  LD* xb = lds(W.ub);                  // the block's solved values
  const int rel = pt - k0;
  if (rel >= 0 && rel < nb) {
    LD2* d = reinterpret_cast<LD2*>(T + rel * kSB);
#pragma unroll
    for (int j = 0; j < kSB / 2; ++j) d[j] = dv2{v[2 * j], v[2 * j + 1]};
  }
  __syncthreads();
  if (t < 64) {
    const int r = t < nb ? lds(W.perm)[k0 + t] : 0;
    double lc[kSB];
    {
      const LD2* rr = reinterpret_cast<const LD2*>(T + (t < nb ? t : 0) * kSB);
#pragma unroll
      for (int j = 0; j < kSB / 2; ++j) {
        const dv2 x = rr[j];
        lc[2 * j] = x.x;
        lc[2 * j + 1] = x.y;
      }
    }
    double xv = t < nb ? b[r] : 0.0;
    // the multipliers are masked rather than the updates, which keeps the
    // selects off the chain of dependent broadcasts (a zero multiplier
    // leaves xv unchanged for finite z)
    if (FWD) {
#pragma unroll
      for (int j = 0; j + 1 < kSB; ++j) {
        if (j + 1 < nb) {
          const double lm = (t > j && t < nb) ? lc[j] : 0.0;
          const double z = row_share(xv, j);
          xv = xv - lm * z;
        }
      }
    } else {
      // the diagonal's reciprocals, all lanes at once; lane j's value is
      // final once the steps above it are done (its multipliers from then
      // on are zero), and is scaled by its reciprocal when broadcast and at
      // the end
      const double rdg = 1.0 / (t < nb ? T[t * kSB + t] : 1.0);
#pragma unroll
      for (int j = kSB - 1; j >= 0; --j) {
        if (j < nb) {
          const double lm = t < j ? lc[j] : 0.0;
          const double z = row_share(xv * rdg, j);
          xv = xv - lm * z;
        }
      }
      xv = xv * rdg;
    }
    if (t < nb) {
      b[r] = xv;
      xb[t] = xv;
    }
  }
  __syncthreads();
  if (FWD ? pt >= k0 + nb : (pt >= 0 && pt < k0)) {
    double a = b[t];
#pragma unroll
    for (int j = 0; j < kSB; ++j)
      if (j < nb) a = a - v[j] * xb[j];
    b[t] = a;
  }
}

__device__ __forceinline__ void solve_w(const double* M, int n, int ld, const Wide& W, double* bg, double* xg) {
  auto* b = lds(bg);
  auto* x = lds(xg);
  const int t = threadIdx.x;
  const int pt = t < n ? lds(W.pos)[t] : -1;   // logical position of physical row t
  const int nblk = (n + kSB - 1) / kSB;
  const int last = (nblk - 1) * kSB;
  double v0[kSB], v1[kSB], v2[kSB];
  // forward: blocks 0, 1, 2, ...; loads past the last block repeat it
  solve_load(M, n, ld, 0, pt >= 0, v0);
  solve_load(M, n, ld, min(kSB, last), pt >= min(kSB, last), v1);
  for (int i = 0; i < nblk; i += 3) {
    solve_load(M, n, ld, min((i + 2) * kSB, last), pt >= min((i + 2) * kSB, last), v2);
    solve_block<true>(i * kSB, n, pt, v0, W, b);
    solve_load(M, n, ld, min((i + 3) * kSB, last), pt >= min((i + 3) * kSB, last), v0);
    if (i + 1 < nblk) solve_block<true>((i + 1) * kSB, n, pt, v1, W, b);
    solve_load(M, n, ld, min((i + 4) * kSB, last), pt >= min((i + 4) * kSB, last), v1);
    if (i + 2 < nblk) solve_block<true>((i + 2) * kSB, n, pt, v2, W, b);
  }
  // backward: blocks nblk - 1, nblk - 2, ...; loads past the first repeat it
  solve_load(M, n, ld, last, pt >= 0 && pt < last + kSB, v0);
  solve_load(M, n, ld, max(last - kSB, 0), pt >= 0 && pt < max(last - kSB, 0) + kSB, v1);
  for (int i = nblk - 1; i >= 0; i -= 3) {
    solve_load(M, n, ld, max((i - 2) * kSB, 0), pt >= 0 && pt < max((i - 2) * kSB, 0) + kSB, v2);
    solve_block<false>(i * kSB, n, pt, v0, W, b);
    solve_load(M, n, ld, max((i - 3) * kSB, 0), pt >= 0 && pt < max((i - 3) * kSB, 0) + kSB, v0);
    if (i - 1 >= 0) solve_block<false>((i - 1) * kSB, n, pt, v1, W, b);
    solve_load(M, n, ld, max((i - 4) * kSB, 0), pt >= 0 && pt < max((i - 4) * kSB, 0) + kSB, v1);
    if (i - 2 >= 0) solve_block<false>((i - 2) * kSB, n, pt, v2, W, b);
  }
  __syncthreads();
  if (t < n) x[t] = b[lds(W.perm)[t]];
  __syncthreads();
}

// ---- the state without the bath gas ----------------------------------------------
// The bath gas is the last species (component ns): its mass fraction is 1 -
// the sum of the other species (a workgroup sum in a fixed order).
__device__ void with_bath_w(double* vec, int ns, double* red) {
  const int t = threadIdx.x;
  const double s = bsum((t >= 1 && t < ns) ? vec[t] : 0.0, red);
  if (t == ns) vec[ns] = 1.0 - s;
  __syncthreads();
}

// Jacobian of the state without the bath gas from the full one (column-major
// in HBM): by the chain rule every species column loses the bath column; the
// bath's row and column are cleared, so its row of M is g e_ns.
__device__ void reduce_bath_w(double* J, int ns, int ld) {
  const int t = threadIdx.x;
  if (t < ns) {
    const double jb = J[ns * ld + t];
    for (int j = 1; j < ns; ++j) J[j * ld + t] = J[j * ld + t] - jb;
    J[ns * ld + t] = 0.0;
  } else if (t == ns) {
    for (int j = 0; j <= ns; ++j) J[j * ld + ns] = 0.0;
  }
  __syncthreads();
}

// ---- adaptive Rosenbrock integration (scheme SCHEME) over [0, dt] for one cell
// (state in W.y) ---------------------------------------------------------------
// GEN: honour the forward-difference Jacobian and the state without the bath
// gas; without it both are compiled out.
template <int SCHEME, bool GEN>
__device__ __forceinline__ void integrate_w(const MechArgs& A, const MechLds& L, const Wide& W, double* J, double* M, int ld,
                            const OptsDev& o, double p, double dt, double& hio, int& nacc_o, int& nrej_o,
                            int& status_o, int& njac_o, int& nfev_o) {
  using TB = Tab<SCHEME>;
  const int ns = A.ns;
  const int n = ns + 1;                 // size of J and M
  const bool nb = GEN && o.no_bath != 0;   // bath gas (component ns) derived, not integrated
  const int ni = nb ? ns : n;           // integrated components
  const int t = threadIdx.x;
  int status = 0;
  if (nb) with_bath_w(W.y, ns, W.red);
  const bool bad = (t < ni && !isfinite(W.y[t])) || !isfinite(p) || !(p > 0.0);
  if (__syncthreads_or(bad)) status = 3;
  double h = hio > 0.0 ? hio : dt;
  double hnext = h, tt = 0.0;
  int nacc = 0, nrej = 0, att = 0, consec = 0;
  int njac = 0, nfev = 0;     // evaluations of J and of f (a difference Jacobian's included)
  bool need = true;
  while (status == 0 && tt < dt) {
    if (att >= o.max_steps) {
      status = 1;
      break;
    }
    if (need) {
      if (GEN && o.jac_fd) {
        rhs_w<false>(A, L, W, p, W.y, W.f0, nullptr, ld);
        // forward differences: column j from f(y + d_j e_j), the perturbed
        // state staged in W.ys and its f in W.fs; without the bath gas the
        // perturbed state's bath component is derived again, and the bath's
        // column and row stay zero
        if (nb && t < n) J[ns * ld + t] = 0.0;
        for (int j = 0; j < ni; ++j) {
          const double yj = W.y[j];
          const double yp = yj + fd_increment(yj);
          const double d = yp - yj;
          if (t < n) W.ys[t] = t == j ? yp : W.y[t];
          __syncthreads();
          if (nb) with_bath_w(W.ys, ns, W.red);
          rhs_w<false>(A, L, W, p, W.ys, W.fs, nullptr, ld);
          if (t < n) J[j * ld + t] = (nb && t == ns) ? 0.0 : (W.fs[t] - W.f0[t]) / d;
          __syncthreads();
        }
      } else {
        rhs_w<true>(A, L, W, p, W.y, W.f0, J, ld);
        if (nb) reduce_bath_w(J, ns, ld);
      }
      need = false;
      ++njac;
      nfev += (GEN && o.jac_fd) ? 1 + ni : 1;
    }
    const double rem = dt - tt;
    double hc = h;
    bool clipped = false;
    if (hc >= rem) {
      hc = rem;
      clipped = true;
    }
    if (hc < kHMin) {
      status = 2;
      break;
    }
    // M = g I - J, formed by the LU as it first reads each column
    const double g = 1.0 / (TB::gamma * hc);
    __syncthreads();
    const int info = lu_w<true>(M, J, g, n, ld, W);
    ++att;
    if (info) {
      status = 4;
      break;
    }
    // stage sums over j < st in ascending order with the scheme's
    // coefficients, zeros included, as the oracle forms them. W.fs keeps the
    // last evaluated f for a stage that reuses it.
    for (int st = 0; st < 4; ++st) {
      const int src = TB::fsrc[st];
      if (src == kFnew) {
        if (t < n) {
          double ys = W.y[t];
          for (int j = 0; j < st; ++j) ys = ys + TB::a[st][j] * W.u[j][t];
          W.ys[t] = ys;
        }
        __syncthreads();
        if (nb) with_bath_w(W.ys, ns, W.red);
        rhs_w<false>(A, L, W, p, W.ys, W.fs, nullptr, ld);
        ++nfev;
      }
      if (t < n) {
        double v = src == kFy ? W.f0[t] : W.fs[t];
        for (int j = 0; j < st; ++j) v = v + (TB::c[st][j] / hc) * W.u[j][t];
        W.v[t] = (nb && t == ns) ? 0.0 : v;   // the bath takes no step of its own
      }
      __syncthreads();
      solve_w(M, n, ld, W, W.v, W.u[st]);
    }
    double yn = 0.0, q = 0.0;
    if (t < n) {
      yn = W.y[t];
      double ev = 0.0;
      for (int j = 0; j < 4; ++j) {
        yn = yn + TB::m[j] * W.u[j][t];
        ev = ev + TB::e[j] * W.u[j][t];
      }
      const double sc = o.atol + o.rtol * fmax(fabs(W.y[t]), fabs(yn));
      q = ev / sc;
      W.yn[t] = yn;
    }
    if (nb) with_bath_w(W.yn, ns, W.red);
    const double acc = bsum(t < ni ? q * q : 0.0, W.red);
    double err = sqrt(acc / ni);
    const bool nonfinite = __syncthreads_or(t < ni && !isfinite(yn));
    double hnew;
    if (nonfinite || !isfinite(err)) {
      err = INFINITY;
      hnew = hc * kFacRej;
    } else {
      double fac = step_factor<SCHEME>(err);
      fac = fmin(kFacMax, fmax(kFacMin, fac));
      hnew = hc * fac;
    }
    if (err <= 1.0) {
      if (consec > 0) hnew = fmin(hnew, hc);
      const double Tn = W.yn[0];
      if (!(Tn >= kTMin && Tn <= kTMax)) {
        status = 5;
        break;
      }
      if (t < n) W.y[t] = W.yn[t];
      ++nacc;
      tt = clipped ? dt : tt + hc;
      hnext = clipped ? fmax(hnew, h) : hnew;
      h = hnew;
      consec = 0;
      need = true;
      __syncthreads();
    } else {
      ++nrej;
      ++consec;
      if (consec >= 2) hnew = hc * kFacRej;
      h = hnew;
    }
  }
  if (status != 0) hnext = h;
  hio = hnext;
  nacc_o = nacc;
  nrej_o = nrej;
  status_o = status;
  njac_o = njac;
  nfev_o = nfev;
}

template <int SCHEME, bool GEN>
__device__ __forceinline__ void run_cell_w(const IntegrateArgs& a, const MechLds& L, const Wide& W, double* J, double* M,
                           long long cell) {
  const int ns = a.m.ns, n = ns + 1, w2 = ns + 2;
  const int t = threadIdx.x;
  const double* pin = a.phi_in + cell * w2;
  const double p = pin[1];
  if (t < n) W.y[t] = t == 0 ? pin[0] : pin[1 + t];
  __syncthreads();
  float ft[4] = {0.f, 0.f, 0.f, 0.f};
  if (a.log.cap > 0) {
    const double lv = (t >= 1 && t <= ns) ? log10(fmax(W.y[t], 1e-30)) : 0.0;
    const double ell = bsum(lv, W.red) / ns;
    ft[0] = static_cast<float>((W.y[0] - 1500.0) / 700.0);
    ft[1] = static_cast<float>(log(p / 1e5));
    ft[2] = static_cast<float>(ell / 10.0);
    ft[3] = static_cast<float>(log10(a.dt / 1e-6));
  }
  double h = a.h_io ? a.h_io[cell] : 0.0;
  int nacc, nrej, st, njac, nfev;
  integrate_w<SCHEME, GEN>(a.m, L, W, J, M, a.ld, a.o, p, a.dt, h, nacc, nrej, st, njac, nfev);
  double* pout = a.phi_out + cell * w2;
  if (t < n) pout[t == 0 ? 0 : 1 + t] = W.y[t];
  if (t == 0) {
    pout[1] = p;
    if (a.h_io) a.h_io[cell] = h;
    if (a.accumulate) {
      if (a.n_acc) a.n_acc[cell] += nacc;
      if (a.n_rej) a.n_rej[cell] += nrej;
      if (a.status && a.status[cell] == 0) a.status[cell] = static_cast<signed char>(st);
      if (a.n_jac) a.n_jac[cell] += njac;
      if (a.n_fev) a.n_fev[cell] += nfev;
    } else {
      if (a.n_acc) a.n_acc[cell] = nacc;
      if (a.n_rej) a.n_rej[cell] = nrej;
      if (a.status) a.status[cell] = static_cast<signed char>(st);
      if (a.n_jac) a.n_jac[cell] = njac;
      if (a.n_fev) a.n_fev[cell] = nfev;
    }
    if (a.log.cap > 0) {
      const unsigned long long k = atomicAdd(a.log.head, 1ull) % static_cast<unsigned long long>(a.log.cap);
      for (int c = 0; c < 4; ++c) a.log.feats[4 * k + c] = ft[c];
      a.log.target[k] = logf(static_cast<float>(nacc + nrej > 0 ? nacc + nrej : 1));
    }
  }
  __syncthreads();
}

// ---- kernels ---------------------------------------------------------------------
// Each workgroup owns workspace slot blockIdx.x. Plain: cells blockIdx.x,
// blockIdx.x + gridDim.x, ... (static); persistent: chunks from the queue.
template <bool PERSIST, int SCHEME, bool GEN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_integrate_wide(IntegrateArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_mech(smem, a.m);
  const MechLds L = mech_views(smem, a.m);
  const Wide W = wide_area(reinterpret_cast<double*>(smem + a.m.lds_bytes), a.m.ns, a.m.nr, a.ld);
  double* J = a.ws + static_cast<long long>(blockIdx.x) * a.ws_stride;
  double* M = J + static_cast<long long>(a.m.ns + 1) * a.ld;
  if (!PERSIST) {
    for (long long cell = blockIdx.x; cell < a.n; cell += gridDim.x) run_cell_w<SCHEME, GEN>(a, L, W, J, M, cell);
  } else {
    for (;;) {
      if (threadIdx.x == 0) W.qslot[0] = atomicAdd(a.head, static_cast<unsigned long long>(a.chunk));
      __syncthreads();
      const unsigned long long idx = W.qslot[0];
      __syncthreads();
      if (idx >= static_cast<unsigned long long>(a.n)) break;
      const long long end = min(static_cast<long long>(idx) + a.chunk, a.n);
      for (long long q = static_cast<long long>(idx); q < end; ++q) {
        const long long cell = a.perm ? static_cast<long long>(a.perm[q]) : q;
        run_cell_w<SCHEME, GEN>(a, L, W, J, M, cell);
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_eval_wide(EvalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_mech(smem, a.m);
  const MechLds L = mech_views(smem, a.m);
  const Wide W = wide_area(reinterpret_cast<double*>(smem + a.m.lds_bytes), a.m.ns, a.m.nr, a.ld);
  double* J = a.ws + static_cast<long long>(blockIdx.x) * a.ws_stride;
  const int ns = a.m.ns, n = ns + 1, ld = a.ld;
  const int t = threadIdx.x;
  for (long long cell = blockIdx.x; cell < a.n; cell += gridDim.x) {
    const double* pin = a.phi + cell * (ns + 2);
    const double p = pin[1];
    if (t < n) W.y[t] = t == 0 ? pin[0] : pin[1 + t];
    __syncthreads();
    if (a.J) {
      rhs_w<true>(a.m, L, W, p, W.y, W.f0, J, ld);
    } else {
      rhs_w<false>(a.m, L, W, p, W.y, W.f0, nullptr, ld);
    }
    if (t < n) a.f[cell * n + t] = W.f0[t];
    if (a.J) {
      const long long nn = static_cast<long long>(n) * n;
      for (long long e = t; e < nn; e += kT) {
        const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<long long>(i) * n);
        a.J[cell * nn + e] = J[j * ld + i];
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_lu_wide(LuArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, ld = a.ld;
  const Wide W = wide_area(reinterpret_cast<double*>(smem), 0, 0, ld);
  double* M = a.ws + static_cast<long long>(blockIdx.x) * a.ws_stride;
  const int t = threadIdx.x;
  const long long nn = static_cast<long long>(n) * n;
  for (long long m = blockIdx.x; m < a.batch; m += gridDim.x) {
    for (long long e = t; e < nn; e += kT) {
      const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<long long>(i) * n);
      M[j * ld + i] = a.A[m * nn + e];
    }
    __syncthreads();
    const int info = lu_w<false>(M, nullptr, 0.0, n, ld, W);
    for (long long e = t; e < nn; e += kT) {
      const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<long long>(i) * n);
      a.A[m * nn + e] = M[j * ld + W.perm[i]];
    }
    if (t < n) a.piv[m * n + t] = W.piv[t];
    if (t == 0) a.info[m] = info;
    if (a.b) {
      if (t < n) W.v[t] = a.b[m * n + t];
      __syncthreads();
      solve_w(M, n, ld, W, W.v, W.u[0]);
      if (t < n) a.b[m * n + t] = W.u[0][t];
    }
    __syncthreads();
  }
}

}  // namespace

int wide_cell_bytes(int ns, int nr, int ld) { return static_cast<int>(sizeof(double)) * wide_doubles(ns, nr, ld); }

template <bool P>
static void* wide_fn(int scheme, bool gen) {
  if (gen)
    return scheme == dev::kRos4 ? reinterpret_cast<void*>(&k_integrate_wide<P, dev::kRos4, true>)
                                : reinterpret_cast<void*>(&k_integrate_wide<P, dev::kRodas3, true>);
  return scheme == dev::kRos4 ? reinterpret_cast<void*>(&k_integrate_wide<P, dev::kRos4, false>)
                              : reinterpret_cast<void*>(&k_integrate_wide<P, dev::kRodas3, false>);
}

hipError_t launch_integrate_wide(bool persistent, int grid, const IntegrateArgs& a, size_t lds_bytes,
                                 hipStream_t st) {
  if (a.o.scheme != dev::kRodas3 && a.o.scheme != dev::kRos4) return hipErrorInvalidValue;
  const bool gen = a.o.jac_fd || a.o.no_bath;
  void* fn = persistent ? wide_fn<true>(a.o.scheme, gen) : wide_fn<false>(a.o.scheme, gen);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  if (e != hipSuccess) return e;
  IntegrateArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(kT), args, lds_bytes, st);
}

int integrate_wide_blocks_per_cu(bool persistent, size_t lds_bytes) {
  void* fn = persistent ? wide_fn<true>(dev::kRodas3, false) : wide_fn<false>(dev::kRodas3, false);
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kT, lds_bytes) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_eval_wide(int grid, const EvalArgs& a, size_t lds_bytes, hipStream_t st) {
  void* fn = reinterpret_cast<void*>(&k_eval_wide);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  if (e != hipSuccess) return e;
  EvalArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(kT), args, lds_bytes, st);
}

hipError_t launch_lu_wide(int grid, const LuArgs& a, size_t lds_bytes, hipStream_t st) {
  void* fn = reinterpret_cast<void*>(&k_lu_wide);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  if (e != hipSuccess) return e;
  LuArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(kT), args, lds_bytes, st);
}

}  // namespace chemk
