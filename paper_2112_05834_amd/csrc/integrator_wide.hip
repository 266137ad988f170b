// Per-cell stiff chemistry integration for mechanisms too large for one
// wave (n = Ns + 1 up to 256): one workgroup of 256 threads per cell.
//
// The Jacobian J and the Rosenbrock matrix M = I/(gamma h) - J of a
// 160-species cell are 161 x 161 FP64 (207 KB each): they fit neither one
// wave's registers nor the 160 KB LDS of a CU. Each resident workgroup
// therefore owns a workspace slot in HBM holding J and M (column-major,
// leading dimension ld); the number of slots, and so of cells in flight, is
// bounded by the HBM budget. Everything else of the cell (state, stage
// vectors, concentrations, per-reaction rates) lives in LDS.
//
// The LU is a right-looking blocked getrf: a panel of 12 columns is factored
// in LDS with partial pivoting (first index of the largest |a|), its row
// interchanges are applied to the other columns, the 12-row block of U is
// solved against the unit-lower diagonal block, and the trailing matrix
// receives the rank-12 update in one pass through HBM. Every element sees
// the same sequence of operations as in an unblocked row-swapping LU, in the
// same order, so the factors do not depend on the blocking.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace chemk {

namespace {

using namespace dev;

constexpr int kT = kWideThreads;
constexpr int kNB = kWidePanel;

// Per-cell LDS area. Region A (right-hand-side buffers) and region B (LU
// panel and U block) are never live at the same time and share storage; so
// do the stage input ys and the solve right-hand side v, and the stage
// derivative fs and the trial state yn.
struct Wide {
  double *C, *gRT, *hRT, *RB;                   // A: ns, ns, ns, 5 nr
  double *panel, *U12;                          // B: kNB ld, kNB ld
  double *y, *f0, *fs, *ys, *yn, *v, *u[4];     // 8 distinct vectors of ld
  double* red;                                  // 16
  int* piv;                                     // ld
  int* perm;                                    // ld
  int* sig;                                     // ld: source row of each row in one panel
  int* ired;                                    // 16
  unsigned long long* qslot;                    // 1
};

__host__ __device__ inline int wide_region(int ns, int nr, int ld) {
  const int a = 3 * ns + 5 * nr;
  const int b = 2 * kNB * ld;
  return ((a > b ? a : b) + 1) & ~1;
}

// doubles: region, 8 vectors, reduction scratch; ints: piv, perm, sig, ired;
// one 64-bit queue slot
__host__ __device__ inline int wide_doubles(int ns, int nr, int ld) {
  return wide_region(ns, nr, ld) + 8 * ld + 16 + (3 * ld + 16) / 2 + 2;
}

__device__ inline Wide wide_area(double* base, int ns, int nr, int ld) {
  Wide W;
  W.C = base;
  W.gRT = W.C + ns;
  W.hRT = W.gRT + ns;
  W.RB = W.hRT + ns;
  W.panel = base;
  W.U12 = base + kNB * ld;
  double* q = base + wide_region(ns, nr, ld);
  W.y = q;
  W.f0 = q + ld;
  W.fs = q + 2 * ld;
  W.yn = W.fs;
  W.v = q + 3 * ld;
  W.ys = W.v;
  for (int k = 0; k < 4; ++k) W.u[k] = q + (4 + k) * ld;
  W.red = q + 8 * ld;
  int* ip = reinterpret_cast<int*>(W.red + 16);
  W.piv = ip;
  W.perm = ip + ld;
  W.sig = ip + 2 * ld;
  W.ired = ip + 3 * ld;
  W.qslot = reinterpret_cast<unsigned long long*>(ip + 3 * ld + 16);
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

// ---- right-hand side and analytical Jacobian ----------------------------------
// f = dy/dt at y (LDS vector); with JAC also J = df/dy, column-major in HBM:
// element (i, j) at J[j * ld + i]. Thread t owns state component t (0 = T,
// t = 1..Ns species t-1) and, for the Jacobian, row t.
template <bool JAC>
__device__ void rhs_w(const MechArgs& A, const MechLds& L, const Wide& W, double p, const double* yv, double* fout,
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
    // four accumulators (k mod 4), eight loads in flight
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < ns; k0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = k0 + q < ns ? J[(1 + k0 + q) * ld + t] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < ns) a[q & 3] = fma(v[q], W.C[k0 + q], a[q & 3]);
    }
    sv = ((a[0] + a[1]) + (a[2] + a[3])) + td * Ctot;
  }
  const double HS = bsum(hRT * sv, W.red);
  const double HT = bsum(hRT * td, W.red);
  const double dQdT = bsum(sp ? cpR * kR * om + hRT * kR * T * (wT - sv / T) : 0.0, W.red);
  double JT = 0.0;
  if (sp) {
    const double* col = J + t * ld + 1;    // column t, rows 1..ns
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < ns; q0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = q0 + q < ns ? col[q0 + q] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q0 + q < ns) c[q & 3] = fma(W.hRT[q0 + q], v[q], c[q & 3]);
    }
    const double cs = (c[0] + c[1]) + (c[2] + c[3]);
    const double dQdY = kR * T * ((rho * rWs) * (cs + HT) - (Wbar * rWs) * HS);
    const double drcp = rho * cpR * kR * rWs - rcp * Wbar * rWs;
    JT = -(dQdY + fT * drcp) / rcp;
  }
  __syncthreads();
  if (sp) {
    const double Wi_rho = A.W[s] / rho;
    for (int k0 = 0; k0 < ns; k0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = k0 + q < ns ? J[(1 + k0 + q) * ld + t] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        if (k < ns) {
          const double rWk = L.rW[k];
          const double D = v[q] + td;
          const double dw = (rho * rWk) * D - (Wbar * rWk) * sv;
          J[(1 + k) * ld + t] = Wi_rho * dw + fY * Wbar * rWk;
        }
      }
    }
    J[t] = Wi_rho * (wT - sv / T) + fY / T;   // (t, 0)
    J[t * ld] = JT;                           // (0, t)
  } else if (t == 0) {
    const double drcp = -rcp / T + rho * dcp;
    J[0] = -(dQdT + fT * drcp) / rcp;
  }
  __syncthreads();
}

// ---- blocked LU with partial pivoting ---------------------------------------------
// M: n x n column-major (leading dimension ld) in HBM, overwritten by L (unit
// lower, below the diagonal) and U. W.piv[k] = row interchanged with row k
// at step k, W.perm = the resulting row order. Returns the first zero pivot
// column + 1 (0 if none); such a column is left unreduced, as getrf does.
// The panel is factored by wave 0 alone (no workgroup barrier per column);
// the whole workgroup applies its interchanges, solves the U block and
// updates the trailing matrix.
__device__ int lu_w(double* M, int n, int ld, const Wide& W) {
  const int t = threadIdx.x;
  if (t < ld) W.perm[t] = t;
  int info = 0;
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int nb = min(kNB, n - k0);
    if (t < ld) {
      const bool in = t >= k0 && t < n;
      for (int c = 0; c < nb; ++c) W.panel[c * ld + t] = in ? M[(k0 + c) * ld + t] : 0.0;
      W.sig[t] = t;
    }
    __syncthreads();
    if (t < 64) {
      for (int c = 0; c < nb; ++c) {
        const int k = k0 + c;
        double* pc = W.panel + c * ld;
        // first index of the largest |a| among rows k..n-1 (a NaN on the
        // diagonal stays the pivot; elsewhere it never wins)
        double key = -1.0;
        int idx = 1 << 30;
        for (int r = k + t; r < n; r += 64) {
          const double av = fabs(pc[r]);
          const double kv = (av != av) ? (r == k ? INFINITY : -1.0) : av;
          if (kv > key) {
            key = kv;
            idx = r;
          }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          const double ok = __shfl_xor(key, off);
          const int oi = __shfl_xor(idx, off);
          if (ok > key || (ok == key && oi < idx)) {
            key = ok;
            idx = oi;
          }
        }
        const int pv = idx;
        if (t == 0) {
          W.piv[k] = pv;
          const int tmp = W.perm[k];
          W.perm[k] = W.perm[pv];
          W.perm[pv] = tmp;
          const int tms = W.sig[k];
          W.sig[k] = W.sig[pv];
          W.sig[pv] = tms;
        }
        if (pv != k && t < nb) {
          double* q = W.panel + t * ld;
          const double tmp = q[k];
          q[k] = q[pv];
          q[pv] = tmp;
        }
        wsync();
        const double akk = pc[k];
        if (akk == 0.0) {
          if (!info) info = k + 1;
          continue;
        }
        for (int r = k + 1 + t; r < n; r += 64) {
          const double l = pc[r] / akk;
          pc[r] = l;
          for (int c2 = c + 1; c2 < nb; ++c2) {
            double* q = W.panel + c2 * ld;
            q[r] = q[r] - l * q[k];
          }
        }
        wsync();
      }
      if (t == 0) W.ired[15] = info;
    }
    __syncthreads();
    info = W.ired[15];
    // panel back to HBM, and its interchanges on the other columns
    if (t < ld && t >= k0 && t < n)
      for (int c = 0; c < nb; ++c) M[(k0 + c) * ld + t] = W.panel[c * ld + t];
    // The panel's interchanges compose to row i <- row sig[i]; only rows
    // k0..k0+nb-1 and their pivot rows can move. All sources are read before
    // any destination is written.
    for (int j = t; j < n; j += kT) {
      if (j >= k0 && j < k0 + nb) continue;
      double* col = M + j * ld;
      double va[kNB], vb[kNB];
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        const int ia = k0 + c, ib = c < nb ? W.piv[k0 + c] : ia;
        va[c] = (c < nb && W.sig[ia] != ia) ? col[W.sig[ia]] : 0.0;
        vb[c] = (c < nb && W.sig[ib] != ib) ? col[W.sig[ib]] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        const int ia = k0 + c, ib = c < nb ? W.piv[k0 + c] : ia;
        if (c < nb && W.sig[ia] != ia) col[ia] = va[c];
        if (c < nb && W.sig[ib] != ib) col[ib] = vb[c];
      }
    }
    __syncthreads();
    const int j0 = k0 + nb, m = n - j0;
    if (m > 0) {
      // U block: L11^-1 A12, one column per thread
      for (int j = j0 + t; j < n; j += kT) {
        double* col = M + j * ld;
        double x[kNB];
#pragma unroll
        for (int q = 0; q < kNB; ++q) x[q] = q < nb ? col[k0 + q] : 0.0;
#pragma unroll
        for (int q = 1; q < kNB; ++q) {
#pragma unroll
          for (int q2 = 0; q2 < q; ++q2)
            if (q < nb) x[q] = x[q] - W.panel[q2 * ld + k0 + q] * x[q2];
        }
#pragma unroll
        for (int q = 0; q < kNB; ++q) {
          if (q < nb) {
            col[k0 + q] = x[q];
            W.U12[(j - j0) * kNB + q] = x[q];
          }
        }
      }
      __syncthreads();
      // trailing update A22 -= L21 U12: threads 0..127 and 128..255 take
      // alternate columns; consecutive threads take consecutive rows
      const int half = t >> 7, rl = t & 127;
      for (int rb = rl; rb < m; rb += 128) {
        const int r = j0 + rb;
        double lr[kNB];
#pragma unroll
        for (int q = 0; q < kNB; ++q) lr[q] = q < nb ? W.panel[q * ld + r] : 0.0;
        // eight columns per round: loads first, then the updates, then stores
        for (int jb = half; jb < m; jb += 16) {
          double av[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int jj = jb + 2 * i;
            av[i] = jj < m ? M[(j0 + jj) * ld + r] : 0.0;
          }
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int jj = jb + 2 * i;
            if (jj < m) {
              const double* u = W.U12 + jj * kNB;
#pragma unroll
              for (int q = 0; q < kNB; ++q)
                if (q < nb) av[i] = av[i] - lr[q] * u[q];
              M[(j0 + jj) * ld + r] = av[i];
            }
          }
        }
      }
      __syncthreads();
    }
  }
  return info;
}

// x = M^-1 b with the factors of lu_w (b, x: LDS vectors, distinct).
// Forward substitution in blocks of kSB columns (each element receives its
// terms in ascending column order), then backward in blocks from the
// bottom. Wave 0 solves the diagonal triangle with the block's factors
// loaded up front; every thread then updates its row with kSB independent
// loads in flight.
constexpr int kSB = 32;

__device__ void solve_w(const double* M, int n, int ld, const Wide& W, const double* b, double* x) {
  const int t = threadIdx.x;
  if (t < n) x[t] = b[W.perm[t]];
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += kSB) {
    const int nb = min(kSB, n - k0);
    if (t < 64) {
      double lc[kSB];
#pragma unroll
      for (int q = 0; q < kSB; ++q) lc[q] = (q + 1 < nb && t > q && t < nb) ? M[(k0 + q) * ld + k0 + t] : 0.0;
      double xv = t < nb ? x[k0 + t] : 0.0;
#pragma unroll
      for (int q = 0; q + 1 < kSB; ++q) {
        if (q + 1 < nb) {
          const double z = __shfl(xv, q);
          if (t > q && t < nb) xv = xv - lc[q] * z;
        }
      }
      if (t < nb) x[k0 + t] = xv;
    }
    __syncthreads();
    for (int r = k0 + nb + t; r < n; r += kT) {
      double lv[kSB];
#pragma unroll
      for (int q = 0; q < kSB; ++q) lv[q] = q < nb ? M[(k0 + q) * ld + r] : 0.0;
      double a = x[r];
#pragma unroll
      for (int q = 0; q < kSB; ++q)
        if (q < nb) a = a - lv[q] * x[k0 + q];
      x[r] = a;
    }
    __syncthreads();
  }
  for (int k0 = ((n - 1) / kSB) * kSB; k0 >= 0; k0 -= kSB) {
    const int nb = min(kSB, n - k0);
    if (t < 64) {
      double uc[kSB];
#pragma unroll
      for (int q = 0; q < kSB; ++q) uc[q] = (q < nb && t < q) ? M[(k0 + q) * ld + k0 + t] : 0.0;
      const double dg = t < nb ? M[(k0 + t) * ld + k0 + t] : 1.0;
      double xv = t < nb ? x[k0 + t] : 0.0;
#pragma unroll
      for (int q = kSB - 1; q >= 0; --q) {
        if (q < nb) {
          const double d = (t == q) ? xv / dg : 0.0;
          const double z = __shfl(d, q);
          if (t == q) {
            xv = z;
          } else if (t < q) {
            xv = xv - uc[q] * z;
          }
        }
      }
      if (t < nb) x[k0 + t] = xv;
    }
    __syncthreads();
    for (int r = t; r < k0; r += kT) {
      double uv[kSB];
#pragma unroll
      for (int q = 0; q < kSB; ++q) uv[q] = q < nb ? M[(k0 + q) * ld + r] : 0.0;
      double a = x[r];
#pragma unroll
      for (int q = 0; q < kSB; ++q)
        if (q < nb) a = a - uv[q] * x[k0 + q];
      x[r] = a;
    }
    __syncthreads();
  }
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
__device__ void integrate_w(const MechArgs& A, const MechLds& L, const Wide& W, double* J, double* M, int ld,
                            const OptsDev& o, double p, double dt, double& hio, int& nacc_o, int& nrej_o,
                            int& status_o) {
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
    const double g = 1.0 / (TB::gamma * hc);
    if (t < ld) {
      // eight independent loads in flight per thread
      for (int c0 = 0; c0 < n; c0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = c0 + q < n ? J[(c0 + q) * ld + t] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (c0 + q < n) M[(c0 + q) * ld + t] = (t == c0 + q ? g : 0.0) - v[q];
      }
    }
    __syncthreads();
    const int info = lu_w(M, n, ld, W);
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
}

template <int SCHEME, bool GEN>
__device__ void run_cell_w(const IntegrateArgs& a, const MechLds& L, const Wide& W, double* J, double* M,
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
  int nacc, nrej, st;
  integrate_w<SCHEME, GEN>(a.m, L, W, J, M, a.ld, a.o, p, a.dt, h, nacc, nrej, st);
  double* pout = a.phi_out + cell * w2;
  if (t < n) pout[t == 0 ? 0 : 1 + t] = W.y[t];
  if (t == 0) {
    pout[1] = p;
    if (a.h_io) a.h_io[cell] = h;
    if (a.accumulate) {
      if (a.n_acc) a.n_acc[cell] += nacc;
      if (a.n_rej) a.n_rej[cell] += nrej;
      if (a.status && a.status[cell] == 0) a.status[cell] = static_cast<signed char>(st);
    } else {
      if (a.n_acc) a.n_acc[cell] = nacc;
      if (a.n_rej) a.n_rej[cell] = nrej;
      if (a.status) a.status[cell] = static_cast<signed char>(st);
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
    const int info = lu_w(M, n, ld, W);
    for (long long e = t; e < nn; e += kT) {
      const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<long long>(i) * n);
      a.A[m * nn + e] = M[j * ld + i];
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
