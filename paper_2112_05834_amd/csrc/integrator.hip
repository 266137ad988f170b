// Per-cell stiff chemistry integration on CDNA4 (gfx950).
//
// One cell is owned by a group of G lanes of a 64-wide wavefront (G = 64: one
// cell per wave; G = 16: four cells per wave), with G >= n = Ns + 1. Lane i
// of the group owns state component i (0 = T, 1..Ns = Y_1..Y_Ns) and row i of
// the Rosenbrock matrix M = I/(gamma h) - J, kept in registers. The analytical
// Jacobian is assembled row-wise in the group's LDS area, from the mechanism
// image that every block stages in LDS; it stays there across rejected steps.
//
// Arithmetic per cell does not depend on G, on the cell's position in the
// grid or on the schedule: reductions follow one fixed pairing tree over 64
// virtual lanes, pivots are chosen by value then lowest position, and every
// other operation is per element in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace chemk {

namespace {

using namespace dev;

// LDS add whose result is not returned: nothing waits on it
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// lane-group primitives (one cell per group of G lanes, G in {16, 32, 64})
// ---------------------------------------------------------------------------
// (every pattern used here reads a lane inside the same row, so no lane is
// out of bounds; bound_ctrl lets the compiler skip initialising the
// destination's old value)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
constexpr int kXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141; // lane i <-> 7-i within 8
constexpr int kMirror = 0x140;     // lane i <-> 15-i within 16
constexpr int kRowBcast15 = 0x142; // lane 15 of each row into the next row
constexpr int kRowBcast31 = 0x143; // lane 31 into rows 2 and 3

// DPP move into the rows of ROWMASK only; the other rows keep old
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows_d(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_rows_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xf, false);
}

template <int G>
struct Grp {
  static_assert(G == 16 || G == 32 || G == 64, "group width");
  __device__ static __forceinline__ int lane() { return static_cast<int>(__lane_id()); }
  __device__ static __forceinline__ int gl() { return lane() & (G - 1); }
  __device__ static __forceinline__ int base() { return lane() & ~(G - 1); }

  // value of v in group lane src (src equal across the group)
  __device__ static __forceinline__ double bcast(double v, int src) {
    if constexpr (G == 64) {
      return readlane_d(v, __builtin_amdgcn_readfirstlane(src));
    } else {
      return __shfl(v, base() + src, 64);
    }
  }
  __device__ static __forceinline__ int bcast_i(int v, int src) {
    if constexpr (G == 64) {
      return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(src));
    } else {
      return __shfl(v, base() + src, 64);
    }
  }
  // Sum over the 64 virtual lanes of a cell (lanes beyond the group add +0)
  // with one pairing tree for every G: xor 1, xor 2, then the 8-lane and
  // 16-lane mirrors inside a DPP row, then rows (0+1) + (2+3). With one cell
  // per wave the rows are combined by DPP row broadcasts: row 3 ends with
  // (r3 + r2) + (r1 + r0), the same value as (r0 + r1) + (r2 + r3) in every
  // bit (IEEE addition commutes), read from lane 63.
  __device__ static __forceinline__ double sum(double x) {
    x = x + dpp_d<kXor1>(x);
    x = x + dpp_d<kXor2>(x);
    x = x + dpp_d<kHalfMirror>(x);
    x = x + dpp_d<kMirror>(x);
    if constexpr (G == 64) {
      x = x + dpp_rows_d<kRowBcast15, 0xA>(0.0, x);   // rows 1, 3: + row 0, row 2
      x = x + dpp_rows_d<kRowBcast31, 0xC>(0.0, x);   // rows 2, 3: + row 1
      return readlane_d(x, 63);
    } else if constexpr (G == 32) {
      return (x + __shfl_xor(x, 16, 64)) + (0.0 + 0.0);
    } else {
      return (x + 0.0) + (0.0 + 0.0);
    }
  }
  __device__ static __forceinline__ double max(double x) {
    x = fmax(x, dpp_d<kXor1>(x));
    x = fmax(x, dpp_d<kXor2>(x));
    x = fmax(x, dpp_d<kHalfMirror>(x));
    x = fmax(x, dpp_d<kMirror>(x));
    if constexpr (G == 64) {
      x = fmax(x, dpp_rows_d<kRowBcast15, 0xA>(x, x));
      x = fmax(x, dpp_rows_d<kRowBcast31, 0xC>(x, x));
      return readlane_d(x, 63);
    } else if constexpr (G == 32) {
      return fmax(x, __shfl_xor(x, 16, 64));
    } else {
      return x;
    }
  }
  __device__ static __forceinline__ int min_i(int x) {
    x = ::min(x, dpp_i<kXor1>(x));
    x = ::min(x, dpp_i<kXor2>(x));
    x = ::min(x, dpp_i<kHalfMirror>(x));
    x = ::min(x, dpp_i<kMirror>(x));
    if constexpr (G == 64) {
      x = ::min(x, dpp_rows_i<kRowBcast15, 0xA>(x, x));
      x = ::min(x, dpp_rows_i<kRowBcast31, 0xC>(x, x));
      return __builtin_amdgcn_readlane(x, 63);
    } else if constexpr (G == 32) {
      return ::min(x, __shfl_xor(x, 16, 64));
    } else {
      return x;
    }
  }
  // group-relative ballot
  __device__ static __forceinline__ unsigned long long ballot(bool p) {
    const unsigned long long b = __ballot(p);
    if constexpr (G == 64) {
      return b;
    } else {
      return (b >> base()) & ((1ull << G) - 1ull);
    }
  }
  __device__ static __forceinline__ bool any(bool p) { return ballot(p) != 0ull; }
  // the group lane where p holds (p true on exactly one lane)
  __device__ static __forceinline__ int first(bool p) {
    return __ffsll(static_cast<long long>(ballot(p))) - 1;
  }
};

// Per-cell LDS area layout (doubles): J [NN*NN] row-major, pivot-row buffer
// P [NN+1 rounded to even], a reaction/species buffer RB, then the
// per-species vectors C, gRT, hRT [NN-1 each; entries from ns on are zero,
// so column loops run to NN-1 without a bound check]. RB holds, for state
// sizes up to 32, the per-reaction rate of progress (and with the Jacobian
// kf*theta, kr*theta, q0*dtheta/d[M], dq/dT) read by the species pass
// [max(5*nr, 3*NN)]; above 32 only the species sums omega, d omega/dT and
// sum nu q0 dtheta/d[M] [3*NN] that the reaction lanes add into.
struct CellArea {
  double* J;
  double* P;
  double* RB;
  double* C;
  double* gRT;
  double* hRT;
};

__host__ __device__ constexpr int pbuf_doubles(int nn) { return (nn + 2) & ~1; }
// state sizes above 32 assemble rates and Jacobian reaction by reaction
__host__ __device__ constexpr bool reaction_major(int nn) { return nn > 32; }
__host__ __device__ constexpr int rbuf_doubles(int nn, int nr) {
  return reaction_major(nn) ? 3 * nn : (5 * nr > 3 * nn ? 5 * nr : 3 * nn);
}
__host__ __device__ constexpr int cell_doubles_c(int nn, int nr, int ns) {
  return ((nn * nn + 1) & ~1) + pbuf_doubles(nn) + rbuf_doubles(nn, nr) + 3 * (nn - 1);
}

template <int NN>
__device__ __forceinline__ CellArea cell_area(double* base, int nr, int ns) {
  CellArea c;
  c.J = base;
  c.P = base + ((NN * NN + 1) & ~1);
  c.RB = c.P + pbuf_doubles(NN);
  c.C = c.RB + rbuf_doubles(NN, nr);
  c.gRT = c.C + (NN - 1);
  c.hRT = c.gRT + (NN - 1);
  return c;
}

// Reaction-major assembly (state sizes above 32, one cell per wave): the
// lane of reaction rx adds nu_i q to om[i], and with the Jacobian nu_i dq/dT
// to wT[i] and nu_i q0 dtheta/d[M] to td[i], for every species i of the
// reaction (nu_i = -order on the reactant side, +order on the product side,
// so a species on both sides gets two adds). With the Jacobian it also forms
// the concentration partials once, dq/dC_j = kf theta dPf_j for reactants
// and -kr theta dPr_j for products, and adds nu_i dq/dC_j to J(1+i, 1+j) for
// every species i and j of the reaction, plus nu_i (alpha_k - 1) q0
// dtheta/d[M] for the listed third-body efficiencies. LDS adds that return
// nothing; the lane-to-reaction mapping is fixed, so the order of the adds
// into each element is fixed.
template <int NN, bool JAC>
__device__ __forceinline__ void rx_scatter(const MechLds& L, const double* C, const uint4 w, const RateOut& r,
                                           double* om, double* wT, double* td, double* J) {
  const int nre = (w.x >> 24) & 0xf, npr = (w.y >> 24) & 0xf;
  const int type = (w.x >> 28) & 3;
  double nu[6];
  int row[6];
  bool cv[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    cv[j] = j < nre;
    cv[3 + j] = j < npr;
    row[j] = cv[j] ? (w.x >> (8 * j)) & 0xff : 0;
    row[3 + j] = cv[3 + j] ? (w.y >> (8 * j)) & 0xff : 0;
    nu[j] = -static_cast<double>((w.z >> (4 * j)) & 0xf);
    nu[3 + j] = static_cast<double>((w.z >> (12 + 4 * j)) & 0xf);
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    if (!cv[a]) continue;
    lds_add(&om[row[a]], nu[a] * r.q);
    if (JAC) {
      lds_add(&wT[row[a]], nu[a] * r.dqdT);
      if (type >= 1) lds_add(&td[row[a]], nu[a] * r.q0b);
    }
  }
  if (!JAC) return;
  double Pf, Pr, dPf[3], dPr[3];
  int sf[3], sr[3];
  mass_action(C, w.x, w.z, nre, Pf, dPf, sf);
  mass_action(C, w.y, w.z >> 12, npr, Pr, dPr, sr);
  double dq[6];
  int col[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dq[j] = r.kfT * dPf[j];
    dq[3 + j] = -(r.krT * dPr[j]);
    col[j] = sf[j];
    col[3 + j] = sr[j];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    if (!cv[a]) continue;
    double* Jr = J + (1 + row[a]) * NN + 1;
#pragma unroll
    for (int b = 0; b < 6; ++b)
      if (cv[b]) lds_add(&Jr[col[b]], nu[a] * dq[b]);
  }
  if (type >= 1) {
    const int eoff = w.w & 0xffff, neff = (w.w >> 16) & 0xff;
    for (int e0 = 0; e0 < neff; e0 += kEffChunk) {
      int sp[kEffChunk];
      double am[kEffChunk];
#pragma unroll
      for (int q = 0; q < kEffChunk; ++q) {
        const int e = e0 + q < neff ? eoff + e0 + q : eoff;
        sp[q] = L.eff_sp[e];
        am[q] = L.eff_am1[e];
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        if (!cv[a]) continue;
        double* Jr = J + (1 + row[a]) * NN + 1;
        const double ab = nu[a] * r.q0b;
#pragma unroll
        for (int q = 0; q < kEffChunk; ++q)
          if (e0 + q < neff) lds_add(&Jr[sp[q]], ab * am[q]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// one cell
// ---------------------------------------------------------------------------
template <int NN, int G>
struct Cell {
  static_assert(G >= NN, "one state component per lane");
  using Gp = Grp<G>;
  // Reaction-major assembly of the production rates and the Jacobian for
  // state sizes above 32 (only 64-lane groups exist there); smaller sizes,
  // which also run several cells per wave, keep the species-major passes,
  // whose order of additions does not depend on the group width.
  static constexpr bool kScatter = reaction_major(NN);

  // f = dy/dt at y (this lane's component); with JAC also the analytical
  // Jacobian df/dy, written row-major into ca.J (complete on return).
  template <bool JAC>
  __device__ static __forceinline__ double rhs(const MechArgs& A, const MechLds& L, const CellArea& ca,
                                               double p, double y) {
    const int ns = A.ns, nr = A.nr;
    const int i = Gp::gl();                 // state component of this lane
    const bool sp = i >= 1 && i <= ns;      // lane holds species i-1
    const int s = sp ? i - 1 : 0;
    const double T = Gp::bcast(y, 0);
    const double rT = 1.0 / T;
    const double lnT = log(T);
    // mixture state
    const double Ys = sp ? y : 0.0;
    const double rWs = sp ? L.rW[s] : 0.0;
    const double invWbar = Gp::sum(Ys * rWs);
    const double Wbar = 1.0 / invWbar;
    const double rho = p * Wbar / (kR * T);
    const double Cs = rho * Ys * rWs;
    const bool pad = i > ns && i < NN;      // padding component of a padded state size
    if (sp) ca.C[s] = Cs;
    const double Ctot = Gp::sum(Cs);
    // species thermo (NASA-7, range by T < Tmid)
    double cpR = 0.0, hRT = 0.0, dcpR = 0.0;
    if (sp) {
      double gRT;
      nasa7<JAC>(A.nasa + 16 * s, T, rT, lnT, cpR, hRT, gRT, dcpR);
      ca.gRT[s] = gRT;
      ca.hRT[s] = hRT;
    } else if (pad) {
      ca.C[i - 1] = 0.0;
      ca.gRT[i - 1] = 0.0;
      ca.hRT[i - 1] = 0.0;
    }
    const double cp = Gp::sum(Ys * cpR * kR * rWs);
    double dcp = 0.0;
    if (JAC) {
      dcp = Gp::sum(Ys * dcpR * kR * rWs);
      if (i < NN) {
#pragma unroll
        for (int j = 0; j < NN; ++j) ca.J[i * NN + j] = 0.0;
      }
    }
    // species sums of the reaction-major assembly
    double* const som = ca.RB;
    double* const swT = ca.RB + NN;
    double* const std_ = ca.RB + 2 * NN;
    if (kScatter && i < NN) {
      som[i] = 0.0;
      if (JAC) {
        swT[i] = 0.0;
        std_[i] = 0.0;
      }
    }
    wsync();

    // ---- reactions: one lane per reaction ----
    const double lnRTp = log(kR * T / kPatm);
    if constexpr (kScatter) {
      // two blocks of reactions per pass, their rate evaluations interleaved
      // (independent work for the one wave on the SIMD); the adds follow in
      // block order
      int r0 = 0;
      for (; r0 + G < nr; r0 += 2 * G) {
        const int rxa = r0 + i;
        const int rxb = rxa + G;
        const bool vb = rxb < nr;
        const int rxb_c = vb ? rxb : rxa;
        const uint4 wa = L.rint[rxa];
        const uint4 wb = L.rint[rxb_c];
        const RateCore ka = rate_core<JAC>(L, wa, ca.C, ca.gRT, ca.hRT, rxa, rT, lnT, lnRTp);
        const RateCore kb = rate_core<JAC>(L, wb, ca.C, ca.gRT, ca.hRT, rxb_c, rT, lnT, lnRTp);
        const RateOut ra = rate_finish<JAC, false>(L, wa, ka, ca.C, ca.RB, nr, rxa, T, rT, lnT, Ctot);
        const RateOut rb = rate_finish<JAC, false>(L, wb, kb, ca.C, ca.RB, nr, rxb_c, T, rT, lnT, Ctot);
        rx_scatter<NN, JAC>(L, ca.C, wa, ra, som, swT, std_, ca.J);
        if (vb) rx_scatter<NN, JAC>(L, ca.C, wb, rb, som, swT, std_, ca.J);
      }
      if (r0 < nr && r0 + i < nr) {
        const int rx = r0 + i;
        const uint4 w = L.rint[rx];
        const RateOut r = reaction_rate<JAC, false>(L, w, ca.C, ca.gRT, ca.hRT, ca.RB, nr, rx, T, rT, lnT, lnRTp, Ctot);
        rx_scatter<NN, JAC>(L, ca.C, w, r, som, swT, std_, ca.J);
      }
    } else {
      for (int r0 = 0; r0 < nr; r0 += G) {
        const int rx = r0 + i;
        if (rx >= nr) break;
        reaction_rate<JAC>(L, ca.C, ca.gRT, ca.hRT, ca.RB, nr, rx, T, rT, lnT, lnRTp, Ctot);
      }
    }
    wsync();

    // ---- species: production rates (and sparse Jacobian rows d omega/dC) ----
    // Above 32 state components the sums were formed by the reaction lanes
    // and are read back. Otherwise each species lane walks its reactions'
    // records; the Jacobian row is accumulated with LDS adds that return
    // nothing (the lane owns its row, and one wave's LDS operations execute
    // in order, so the sum order is the program order), and the next
    // entry's records are fetched before the current one is processed.
    double om = 0.0, wT = 0.0, td = 0.0;
    if (kScatter) {
      if (sp) {
        om = som[s];
        if (JAC) {
          wT = swT[s];
          td = std_[s];
        }
      }
    } else if (sp) {
      const int e0 = L.sp_off[s], e1 = L.sp_off[s + 1];
      double* Jrow = ca.J + i * NN + 1;
      if (!JAC) {
#pragma unroll 4
        for (int e = e0; e < e1; ++e) {
          const unsigned ent = L.sp_ent[e];
          const double nu = static_cast<double>(static_cast<int>(ent >> 12) - 8);
          om = om + nu * ca.RB[ent & 0xfff];
        }
      } else {
        unsigned ent = e0 < e1 ? L.sp_ent[e0] : 0u;
        uint4 w = L.rint[ent & 0xfff];
        for (int e = e0; e < e1; ++e) {
          const int rx = ent & 0xfff;
          const double nu = static_cast<double>(static_cast<int>(ent >> 12) - 8);
          const uint4 wc = w;
          // prefetch the next entry
          const unsigned ent_n = e + 1 < e1 ? L.sp_ent[e + 1] : ent;
          double qr = ca.RB[rx], kfT = ca.RB[nr + rx], krT = ca.RB[2 * nr + rx];
          double q0b = ca.RB[3 * nr + rx], dqdT = ca.RB[4 * nr + rx];
          asm volatile("" : "+v"(qr), "+v"(kfT), "+v"(krT), "+v"(q0b), "+v"(dqdT));
          const int nre = (wc.x >> 24) & 0xf, npr = (wc.y >> 24) & 0xf;
          double Pf, Pr, dPf[3], dPr[3];
          int sf[3], sr[3];
          mass_action(ca.C, wc.x, wc.z, nre, Pf, dPf, sf);
          mass_action(ca.C, wc.y, wc.z >> 12, npr, Pr, dPr, sr);
          w = L.rint[ent_n & 0xfff];
          ent = ent_n;
          om = om + nu * qr;
          wT = wT + nu * dqdT;
          const double af = nu * kfT, ar = nu * krT;
#pragma unroll
          for (int j = 0; j < 3; ++j) lds_add(j < nre ? &Jrow[sf[j]] : ca.P, af * dPf[j]);
#pragma unroll
          for (int j = 0; j < 3; ++j) lds_add(j < npr ? &Jrow[sr[j]] : ca.P, -(ar * dPr[j]));
          const int type = (wc.x >> 28) & 3;
          if (type >= 1) {
            const double ab = nu * q0b;
            td = td + ab;
            const int eoff = wc.w & 0xffff, neff = (wc.w >> 16) & 0xff;
            for (int q = 0; q < neff; ++q) lds_add(&Jrow[L.eff_sp[eoff + q]], ab * L.eff_am1[eoff + q]);
          }
        }
      }
    }
    const double fY = sp ? A.W[s] * om / rho : 0.0;
    const double Q = Gp::sum(hRT * kR * T * om);
    const double rcp = rho * cp;
    const double fT = -Q / rcp;
    const double f = (i == 0) ? fT : fY;
    if (!JAC) return f;

    // ---- Jacobian: chain rule from d(omega)/dC, d(omega)/dT to y = (T, Y) ----
    wsync();
    double sv = 0.0;
    if (sp) {
      const double* Jrow = ca.J + i * NN + 1;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      // columns from ns on are zero in J and in C
#pragma unroll
      for (int k = 0; k < NN - 1; k += 4) {
        a0 = fma(Jrow[k], ca.C[k], a0);
        if (k + 1 < NN - 1) a1 = fma(Jrow[k + 1], ca.C[k + 1], a1);
        if (k + 2 < NN - 1) a2 = fma(Jrow[k + 2], ca.C[k + 2], a2);
        if (k + 3 < NN - 1) a3 = fma(Jrow[k + 3], ca.C[k + 3], a3);
      }
      sv = ((a0 + a1) + (a2 + a3)) + td * Ctot;
    }
    const double HS = Gp::sum(hRT * sv);
    const double HT = Gp::sum(hRT * td);
    const double dQdT = Gp::sum(sp ? cpR * kR * om + hRT * kR * T * (wT - sv / T) : 0.0);
    // T-row entry of column i (species i-1): lane i sums column i of D
    double JT = 0.0;
    if (sp) {
      double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
      // rows beyond species ns - 1 are zero in J and in hRT
#pragma unroll
      for (int q = 0; q < NN - 1; q += 4) {
        c0 = fma(ca.hRT[q], ca.J[(1 + q) * NN + i], c0);
        if (q + 1 < NN - 1) c1 = fma(ca.hRT[q + 1], ca.J[(2 + q) * NN + i], c1);
        if (q + 2 < NN - 1) c2 = fma(ca.hRT[q + 2], ca.J[(3 + q) * NN + i], c2);
        if (q + 3 < NN - 1) c3 = fma(ca.hRT[q + 3], ca.J[(4 + q) * NN + i], c3);
      }
      const double cs = (c0 + c1) + (c2 + c3);
      const double dQdY = kR * T * ((rho * rWs) * (cs + HT) - (Wbar * rWs) * HS);
      const double drcp = rho * cpR * kR * rWs - rcp * Wbar * rWs;
      JT = -(dQdY + fT * drcp) / rcp;
    }
    wsync();
    if (sp) {
      double* Jrow = ca.J + i * NN;
      const double Wi_rho = A.W[s] / rho;
      // rW is zero from ns on (up to 64 entries), which keeps the padding
      // columns of J zero
#pragma unroll
      for (int k = 0; k < NN - 1; ++k) {
        const double rWk = L.rW[k];
        const double D = Jrow[1 + k] + td;
        const double dw = (rho * rWk) * D - (Wbar * rWk) * sv;
        Jrow[1 + k] = Wi_rho * dw + fY * Wbar * rWk;
      }
      Jrow[0] = Wi_rho * (wT - sv / T) + fY / T;
      ca.J[i] = JT;
    } else if (i == 0) {
      const double drcp = -rcp / T + rho * dcp;
      ca.J[0] = -(dQdT + fT * drcp) / rcp;
    }
    wsync();
    return f;
  }

  // Without the bath gas (the last species, lane ns) its mass fraction is
  // 1 - the sum of the other species: this lane's value, with lane ns
  // replaced by that.
  __device__ static __forceinline__ double with_bath(int ns, double v) {
    const int i = Gp::gl();
    const double s = Gp::sum((i >= 1 && i < ns) ? v : 0.0);
    return i == ns ? 1.0 - s : v;
  }

  // The Jacobian of the state without the bath gas, from the full one in
  // ca.J: by the chain rule through Y_bath = 1 - sum_j Y_j every species
  // column loses the bath column. The bath's row and column are cleared, so
  // that its row of M is g e_ns, decoupled from the others.
  __device__ static __forceinline__ void reduce_bath(const CellArea& ca, int ns) {
    const int i = Gp::gl();
    wsync();
    if (i < ns) {
      double* Jr = ca.J + i * NN;
      const double jb = Jr[ns];
#pragma unroll
      for (int j = 1; j < NN; ++j)
        if (j < ns) Jr[j] = Jr[j] - jb;
      Jr[ns] = 0.0;
    } else if (i == ns) {
#pragma unroll
      for (int j = 0; j < NN; ++j) ca.J[i * NN + j] = 0.0;
    }
    wsync();
  }

  // Jacobian by forward differences, written row-major into ca.J: one more
  // right-hand side per integrated component (f0 = f(y) given). Every lane
  // holds its component of the perturbed state; lane j adds the increment.
  // Without the bath gas the perturbed state's bath lane is derived again,
  // so the columns are those of the reduced system, and the bath's row stays
  // zero.
  __device__ static void fd_jacobian(const MechArgs& A, const MechLds& L, const CellArea& ca, double p, double y,
                                     double f0, bool nb) {
    const int ns = A.ns;
    const int n = nb ? ns : ns + 1;
    const int i = Gp::gl();
    if (i < NN) {
#pragma unroll
      for (int j = 0; j < NN; ++j) ca.J[i * NN + j] = 0.0;
    }
#pragma nounroll
    for (int j = 0; j < n; ++j) {
      const double yj = Gp::bcast(y, j);
      const double yp = yj + fd_increment(yj);
      const double d = yp - yj;
      double ypert = i == j ? yp : y;
      if (nb) ypert = with_bath(ns, ypert);
      const double fj = rhs<false>(A, L, ca, p, ypert);
      if (i < NN && !(nb && i == ns)) ca.J[i * NN + j] = (fj - f0) / d;
    }
    wsync();
  }

  // -------------------------------------------------------------------------
  // LU with partial pivoting of the rows in registers (row = lane). Rows are
  // not moved during the elimination: pos tracks each row's LAPACK position,
  // so the pivot of column k is the largest |a| among rows at positions >= k,
  // ties to the lowest position, exactly as a row-swapping getrf. The pivot
  // row reaches the other lanes through the LDS buffer P. At the end every
  // row is sent to the lane of its position (one ds_permute per dword), so on
  // return lane k holds row k of the packed factors (L left of the diagonal,
  // unit diagonal implied; U from the diagonal on) and rdiag = 1/U_kk; pos
  // keeps the position this lane's original row went to (used to permute
  // right-hand sides). Returns the first singular column + 1.
  // -------------------------------------------------------------------------
  __device__ static __forceinline__ int lu(double (&M)[NN], int& pos, double& rdiag, double* P, int* pivk) {
    int info = 0;
    const int i = Gp::gl();
    pos = i < NN ? i : kBig;
    rdiag = 0.0;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const double a = M[k];
      const bool cand = pos >= k && pos < NN;
      const double key = cand ? fabs(a) : -1.0;
      const double amax = Gp::max(key);
      const bool tie = key == amax;
      const unsigned long long bal = Gp::ballot(tie);
      int owner;
      if (__popcll(bal) == 1) {
        owner = __ffsll(static_cast<long long>(bal)) - 1;
      } else {
        const int pmin = Gp::min_i(tie ? pos : kBig);
        owner = Gp::first(tie && pos == pmin);
      }
      const int ppos = Gp::bcast_i(pos, owner);
      const bool is_owner = i == owner;
      if (is_owner) {
        pos = k;
      } else if (pos == k) {
        pos = ppos;
      }
      if (pivk) pivk[k] = ppos;
      const double akk = Gp::bcast(a, owner);
      double rp;
      if (amax == 0.0) {
        if (info == 0) info = k + 1;
        rp = 0.0;
      } else {
        // hardware reciprocal refined by two Newton steps (a shorter
        // dependent chain than a correctly rounded division)
        rp = __builtin_amdgcn_rcp(akk);
        rp = fma(rp, fma(-akk, rp, 1.0), rp);
        rp = fma(rp, fma(-akk, rp, 1.0), rp);
      }
      if (is_owner) rdiag = rp;
      const bool below = pos > k && pos < NN;
      const double l = below ? a * rp : 0.0;
      if (below) M[k] = l;
#pragma unroll
      for (int j = k + 1; j < NN; ++j) M[j] = fma(-l, Gp::bcast(M[j], owner), M[j]);
    }
    // rows to the lanes of their positions
    const int dst = 4 * (Gp::base() + (pos < NN ? pos : i));
#pragma unroll
    for (int j = 0; j < NN; ++j) M[j] = permute_d(M[j], dst);
    rdiag = permute_d(rdiag, dst);
    return info;
  }

  // lane gl() receives the value of the lane whose byte address it is sent to
  __device__ static __forceinline__ double permute_d(double v, int dst_addr) {
    const int lo = __builtin_amdgcn_ds_permute(dst_addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_permute(dst_addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
  }

  // Solve M x = b with the factors of lu(); b is this lane's equation (row
  // gl() of M), the return value is solution component gl(). The right-hand
  // side is first sent to position order; both substitutions then broadcast
  // from fixed lanes.
  __device__ static __forceinline__ double solve(const double (&M)[NN], int pos, double rdiag, double b) {
    const int i = Gp::gl();
    b = permute_d(b, 4 * (Gp::base() + (pos < NN ? pos : i)));
    // the multipliers are masked rather than the update, which keeps the
    // selects off the chain of dependent broadcasts (a zero multiplier
    // leaves b unchanged for finite z)
#pragma unroll
    for (int j = 0; j < NN - 1; ++j) {
      const double lm = i > j ? M[j] : 0.0;
      const double z = Gp::bcast(b, j);
      b = fma(-lm, z, b);
    }
#pragma unroll
    for (int j = NN - 1; j > 0; --j) {
      const double um = i < j ? M[j] : 0.0;
      const double z = Gp::bcast(b * rdiag, j);
      b = fma(-um, z, b);
    }
    return b * rdiag;
  }

  // -------------------------------------------------------------------------
  // adaptive Rosenbrock integration (scheme SCHEME) over [0, dt] for one cell
  // (y: this lane's component)
  // -------------------------------------------------------------------------
  // GEN: honour the forward-difference Jacobian and the state without the
  // bath gas (run-time options); without it both are compiled out, so that
  // the kernels of the default options carry none of their code.
  template <int SCHEME, bool GEN>
  __device__ static __forceinline__ void integrate(const MechArgs& A, const MechLds& L, const CellArea& ca,
                                                   const OptsDev& o, double p, double dt, double& y,
                                                   double& hio, int& nacc_o, int& nrej_o, int& status_o,
                                                   int& njac_o, int& nfev_o) {
    using TB = Tab<SCHEME>;
    const int ns = A.ns;
    const bool nb = GEN && o.no_bath != 0;   // bath gas (lane ns) derived, not integrated
    const int n = nb ? ns : ns + 1;       // integrated components
    const int i = Gp::gl();
    const bool valid = i < n;
    if (nb) y = with_bath(ns, y);
    double M[NN];
    int pos;
    double rdiag;
    int status = 0;
    // a non-finite state, or a pressure that is not a positive number
    if (Gp::any((valid && !isfinite(y)) || !isfinite(p) || !(p > 0.0))) status = 3;
    double h = hio > 0.0 ? hio : dt;
    double hnext = h, t = 0.0;
    int nacc = 0, nrej = 0, att = 0, consec = 0;
    int njac = 0, nfev = 0;     // evaluations of J and of f (a difference Jacobian's included)
    bool need = true;
    double f0 = 0.0;
    while (status == 0 && t < dt) {
      if (att >= o.max_steps) {
        status = 1;
        break;
      }
      if (need) {
        if (GEN && o.jac_fd) {
          f0 = rhs<false>(A, L, ca, p, y);
          fd_jacobian(A, L, ca, p, y, f0, nb);
        } else {
          f0 = rhs<true>(A, L, ca, p, y);
          if (nb) reduce_bath(ca, ns);
        }
        need = false;
        ++njac;
        nfev += (GEN && o.jac_fd) ? 1 + n : 1;
      }
      const double rem = dt - t;
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
      if (i < NN) {
#pragma unroll
        for (int j = 0; j < NN; ++j) M[j] = (i == j ? g : 0.0) - ca.J[i * NN + j];
      } else {
#pragma unroll
        for (int j = 0; j < NN; ++j) M[j] = 0.0;
      }
      const int info = lu(M, pos, rdiag, ca.P, nullptr);
      ++att;
      if (info) {
        status = 4;
        break;
      }
      // stages: one right-hand side and one solve call site for all four;
      // every sum runs over j < st in ascending order with the scheme's
      // coefficients, zeros included, as the oracle forms it
      double u1 = 0.0, u2 = 0.0, u3 = 0.0, u4 = 0.0;
      double fs = f0;
#pragma nounroll
      for (int st = 0; st < 4; ++st) {
        const int src = tab_fsrc<SCHEME>(st);
        if (src == kFnew) {
          double ys = y;
          if (st > 0) ys = ys + tab_a<SCHEME>(st, 0) * u1;
          if (st > 1) ys = ys + tab_a<SCHEME>(st, 1) * u2;
          if (st > 2) ys = ys + tab_a<SCHEME>(st, 2) * u3;
          if (nb) ys = with_bath(ns, ys);
          fs = rhs<false>(A, L, ca, p, ys);
          ++nfev;
        } else if (src == kFy) {
          fs = f0;
        }
        double v = fs;
        if (st > 0) v = v + (tab_c<SCHEME>(st, 0) / hc) * u1;
        if (st > 1) v = v + (tab_c<SCHEME>(st, 1) / hc) * u2;
        if (st > 2) v = v + (tab_c<SCHEME>(st, 2) / hc) * u3;
        if (nb && i == ns) v = 0.0;         // the bath lane takes no step of its own
        const double x = solve(M, pos, rdiag, v);
        if (st == 0) u1 = x;
        else if (st == 1) u2 = x;
        else if (st == 2) u3 = x;
        else u4 = x;
      }
      // new solution and error estimate
      double yn = y + TB::m[0] * u1;
      yn = yn + TB::m[1] * u2;
      yn = yn + TB::m[2] * u3;
      yn = yn + TB::m[3] * u4;
      if (nb) yn = with_bath(ns, yn);
      double ev = 0.0 + TB::e[0] * u1;
      ev = ev + TB::e[1] * u2;
      ev = ev + TB::e[2] * u3;
      ev = ev + TB::e[3] * u4;
      const double sc = o.atol + o.rtol * fmax(fabs(y), fabs(yn));
      const double q = ev / sc;
      const double acc = Gp::sum(valid ? q * q : 0.0);
      double err = sqrt(acc / n);
      double hnew;
      if (Gp::any(valid && !isfinite(yn)) || !isfinite(err)) {
        err = INFINITY;
        hnew = hc * kFacRej;
      } else {
        double fac = step_factor<SCHEME>(err);
        fac = fmin(kFacMax, fmax(kFacMin, fac));
        hnew = hc * fac;
      }
      if (err <= 1.0) {
        if (consec > 0) hnew = fmin(hnew, hc);
        const double Tn = Gp::bcast(yn, 0);
        if (!(Tn >= kTMin && Tn <= kTMax)) {
          status = 5;
          break;
        }
        y = yn;
        ++nacc;
        t = clipped ? dt : t + hc;
        hnext = clipped ? fmax(hnew, h) : hnew;
        h = hnew;
        consec = 0;
        need = true;
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
};

// features for the learned cost model: (T-1500)/700, ln(p/1e5),
// mean log10 max(Y, 1e-30) / 10, log10(dt/1e-6)
template <int G>
__device__ __forceinline__ void cell_features(int ns, double y, double p, double dt, float (&ft)[4]) {
  const int i = Grp<G>::gl();
  const double lv = (i >= 1 && i <= ns) ? log10(fmax(y, 1e-30)) : 0.0;
  const double ell = Grp<G>::sum(lv) / ns;
  const double T = Grp<G>::bcast(y, 0);
  ft[0] = static_cast<float>((T - 1500.0) / 700.0);
  ft[1] = static_cast<float>(log(p / 1e5));
  ft[2] = static_cast<float>(ell / 10.0);
  ft[3] = static_cast<float>(log10(dt / 1e-6));
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <int NN, int G, int SCHEME, bool GEN>
__device__ __forceinline__ void run_cell(const IntegrateArgs& a, const MechLds& L, const CellArea& ca,
                                         long long cell) {
  using C = Cell<NN, G>;
  const int ns = a.m.ns;
  const int w2 = ns + 2;
  const int i = Grp<G>::gl();
  const double* pin = a.phi_in + cell * w2;
  const double p = pin[1];
  double y = i == 0 ? pin[0] : (i <= ns ? pin[1 + i] : 0.0);
  float ft[4];
  if (a.log.cap > 0) cell_features<G>(ns, y, p, a.dt, ft);
  double h = a.h_io ? a.h_io[cell] : 0.0;
  int nacc, nrej, st, njac, nfev;
  C::template integrate<SCHEME, GEN>(a.m, L, ca, a.o, p, a.dt, y, h, nacc, nrej, st, njac, nfev);
  double* pout = a.phi_out + cell * w2;
  if (i == 0) {
    pout[0] = y;
    pout[1] = p;
  } else if (i <= ns) {
    pout[1 + i] = y;
  }
  if (i == 0) {
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
      a.log.feats[4 * k + 0] = ft[0];
      a.log.feats[4 * k + 1] = ft[1];
      a.log.feats[4 * k + 2] = ft[2];
      a.log.feats[4 * k + 3] = ft[3];
      a.log.target[k] = logf(static_cast<float>(nacc + nrej > 0 ? nacc + nrej : 1));
    }
  }
}

// Large state sizes run one wave per SIMD (the per-cell LDS area allows no
// more), so let the register allocator use the whole 512-entry budget.
template <int NN>
constexpr int max_waves_per_eu() { return NN >= 32 ? 1 : 2; }

template <int NN, int G, bool PERSIST, int SCHEME, bool GEN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, max_waves_per_eu<NN>())))
k_integrate(IntegrateArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_mech(smem, a.m);
  const MechLds L = mech_views(smem, a.m);
  constexpr int CPW = 64 / G;
  const int wave = threadIdx.x / 64;
  const int grp = (threadIdx.x % 64) / G;
  double* base = reinterpret_cast<double*>(smem + a.m.lds_bytes) +
                 static_cast<long long>(wave * CPW + grp) * a.cell_doubles;
  const CellArea ca = cell_area<NN>(base, a.m.nr, a.m.ns);
  if (!PERSIST) {
    const long long cell = (static_cast<long long>(blockIdx.x) * a.wpb + wave) * CPW + grp;
    if (cell < a.n) run_cell<NN, G, SCHEME, GEN>(a, L, ca, cell);
  } else {
    for (;;) {
      unsigned long long idx = 0;
      if (Grp<G>::gl() == 0) idx = atomicAdd(a.head, static_cast<unsigned long long>(a.chunk));
      idx = static_cast<unsigned long long>(__shfl(static_cast<long long>(idx), Grp<G>::base(), 64));
      if (idx >= static_cast<unsigned long long>(a.n)) break;
      const long long end = min(static_cast<long long>(idx) + a.chunk, a.n);
      for (long long q = static_cast<long long>(idx); q < end; ++q) {
        const long long cell = a.perm ? static_cast<long long>(a.perm[q]) : q;
        run_cell<NN, G, SCHEME, GEN>(a, L, ca, cell);
      }
    }
  }
}

template <int NN, int G>
__global__ void __launch_bounds__(256) k_eval(EvalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  stage_mech(smem, a.m);
  const MechLds L = mech_views(smem, a.m);
  using C = Cell<NN, G>;
  constexpr int CPW = 64 / G;
  const int wave = threadIdx.x / 64;
  const int grp = (threadIdx.x % 64) / G;
  double* base = reinterpret_cast<double*>(smem + a.m.lds_bytes) +
                 static_cast<long long>(wave * CPW + grp) * a.cell_doubles;
  const CellArea ca = cell_area<NN>(base, a.m.nr, a.m.ns);
  const long long cell = (static_cast<long long>(blockIdx.x) * a.wpb + wave) * CPW + grp;
  if (cell >= a.n) return;
  const int ns = a.m.ns, n = ns + 1;
  const int i = Grp<G>::gl();
  const double* pin = a.phi + cell * (ns + 2);
  const double p = pin[1];
  const double y = i == 0 ? pin[0] : (i <= ns ? pin[1 + i] : 0.0);
  const double f = a.J ? C::template rhs<true>(a.m, L, ca, p, y) : C::template rhs<false>(a.m, L, ca, p, y);
  if (i < n) {
    a.f[cell * n + i] = f;
    if (a.J)
      for (int j = 0; j < n; ++j) a.J[(cell * n + i) * n + j] = ca.J[i * NN + j];
  }
}

template <int NN, int G>
__global__ void __launch_bounds__(256) k_lu(LuArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using C = Cell<NN, G>;
  constexpr int CPW = 64 / G;
  const int wave = threadIdx.x / 64;
  const int grp = (threadIdx.x % 64) / G;
  double* P = reinterpret_cast<double*>(smem) + (wave * CPW + grp) * pbuf_doubles(NN);
  const long long m = (static_cast<long long>(blockIdx.x) * a.wpb + wave) * CPW + grp;
  if (m >= a.batch) return;
  const int n = a.n;
  const int i = Grp<G>::gl();
  double M[NN];
#pragma unroll
  for (int j = 0; j < NN; ++j)
    M[j] = (i < n && j < n) ? a.A[(m * n + i) * n + j] : (i == j && i < NN ? 1.0 : 0.0);
  int pivk[NN];
  int pos;
  double rdiag;
  const int info = C::lu(M, pos, rdiag, P, pivk);
  if (i < n) {
#pragma unroll
    for (int j = 0; j < NN; ++j)
      if (j < n) a.A[(m * n + i) * n + j] = M[j];
  }
  if (i == 0) {
#pragma unroll
    for (int k = 0; k < NN; ++k)
      if (k < n) a.piv[m * n + k] = pivk[k];
    a.info[m] = info;
  }
  if (a.b) {
    const double b = i < n ? a.b[m * n + i] : 0.0;
    const double x = C::solve(M, pos, rdiag, b);
    if (i < n) a.b[m * n + i] = x;
  }
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_copy_f64(double* dst, const double* src, long long n) {
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define CHEM_VARIANTS(X) \
  X(10, 16)              \
  X(10, 64)              \
  X(16, 16)              \
  X(32, 32)              \
  X(55, 64)              \
  X(64, 64)

int variants_for(int n, Variant* out, int max_out) {
  // exact sizes first, then the smallest padded size
  static const Variant all[] = {
#define V(a, b) {a, b},
      CHEM_VARIANTS(V)
#undef V
  };
  int cnt = 0, best_nn = 1 << 30;
  for (const Variant& v : all)
    if (v.nn >= n && v.nn < best_nn) best_nn = v.nn;
  for (const Variant& v : all)
    if (v.nn == best_nn && cnt < max_out) out[cnt++] = v;
  return cnt;
}

int cell_doubles(int nn, int nr, int ns) { return cell_doubles_c(nn, nr, ns); }

template <int NN, int G, bool P>
static void* integrate_fn(int scheme, bool gen) {
  if (gen)
    return scheme == dev::kRos4 ? reinterpret_cast<void*>(&k_integrate<NN, G, P, dev::kRos4, true>)
                                : reinterpret_cast<void*>(&k_integrate<NN, G, P, dev::kRodas3, true>);
  return scheme == dev::kRos4 ? reinterpret_cast<void*>(&k_integrate<NN, G, P, dev::kRos4, false>)
                              : reinterpret_cast<void*>(&k_integrate<NN, G, P, dev::kRodas3, false>);
}

static void* find_integrate(const Variant& v, bool persistent, int scheme, bool gen) {
  if (scheme != dev::kRodas3 && scheme != dev::kRos4) return nullptr;
#define V(a, b)                                                                                        \
  if (v.nn == a && v.g == b)                                                                           \
    return persistent ? integrate_fn<a, b, true>(scheme, gen) : integrate_fn<a, b, false>(scheme, gen);
  CHEM_VARIANTS(V)
#undef V
  return nullptr;
}

hipError_t launch_integrate(const Variant& v, bool persistent, int grid, const IntegrateArgs& a,
                            size_t lds_bytes, hipStream_t st) {
  void* fn = find_integrate(v, persistent, a.o.scheme, a.o.jac_fd || a.o.no_bath);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  if (e != hipSuccess) return e;
  dim3 block(64 * a.wpb);
  IntegrateArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), block, args, lds_bytes, st);
}

int integrate_blocks_per_cu(const Variant& v, bool persistent, int wpb, size_t lds_bytes) {
  void* fn = find_integrate(v, persistent, dev::kRodas3, false);
  if (!fn) return 0;
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * wpb, lds_bytes) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_eval(const Variant& v, int grid, const EvalArgs& a, size_t lds_bytes, hipStream_t st) {
  void* fn = nullptr;
#define V(x, y) \
  if (v.nn == x && v.g == y) fn = reinterpret_cast<void*>(&k_eval<x, y>);
  CHEM_VARIANTS(V)
#undef V
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
  if (e != hipSuccess) return e;
  EvalArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(64 * a.wpb), args, lds_bytes, st);
}

hipError_t launch_lu(const Variant& v, int grid, const LuArgs& a, hipStream_t st) {
  void* fn = nullptr;
#define V(x, y) \
  if (v.nn == x && v.g == y) fn = reinterpret_cast<void*>(&k_lu<x, y>);
  CHEM_VARIANTS(V)
#undef V
  if (!fn) return hipErrorInvalidValue;
  LuArgs copy = a;
  void* args[] = {&copy};
  const size_t lds = sizeof(double) * pbuf_doubles(v.nn) * a.wpb * (64 / v.g);
  return hipLaunchKernel(fn, dim3(grid), dim3(64 * a.wpb), args, lds, st);
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_copy_f64(double* dst, const double* src, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy_f64, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace chemk
