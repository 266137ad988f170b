// Device code shared by the per-wave integrator (n <= 64) and the
// per-workgroup integrator (larger mechanisms): physical and method
// constants, the mechanism image in LDS, NASA-7 thermo, and the rate of
// progress of one reaction with the pieces its Jacobian needs.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace chemk {
namespace dev {

constexpr double kR = 8.314462618;     // J mol^-1 K^-1
constexpr double kPatm = 101325.0;     // Pa
constexpr double kLn10 = 2.302585092994045684;
constexpr int kBig = 1 << 20;

// Forward-difference Jacobian (the conventional alternative to the
// analytical one): column j is (f(y + d_j e_j) - f(y)) / d_j with
// d_j = (y_j + s_j) - y_j, the step actually taken, and
// s_j = sqrt(u max(1e-5, |y_j|)), u = 2^-53 (the increment rule of Hairer and
// Wanner's Rosenbrock codes).
constexpr double kFdUround = 1.1102230246251565e-16;
__device__ __forceinline__ double fd_increment(double yj) { return sqrt(kFdUround * fmax(1e-5, fabs(yj))); }

// step-size controller
constexpr double kFacMin = 0.2, kFacMax = 6.0, kFacSafe = 0.9, kFacRej = 0.1;
constexpr double kHMin = 1e-20, kTMin = 200.0, kTMax = 6000.0;

// Four-stage Rosenbrock schemes in the transformed form (unknowns u_i,
// matrix M = I/(gamma h) - J):
//   u_s = M^-1 ( f(y + sum_{j<s} a_sj u_j) + sum_{j<s} (c_sj / h) u_j ),
//   y_new = y + sum_j m_j u_j,  error estimate sum_j e_j u_j.
// fsrc[s] says where stage s takes f from: kFy = f(y) (a zero a-row), kFprev =
// the previous stage's f (the same a-row, so the same argument), kFnew = a new
// evaluation. Sums run over every j in ascending order, zero coefficients
// included, so that the operations match the oracle's. est_order is the order
// of the embedded solution (the step factor goes as err^(-1/(est_order+1))).
constexpr int kFy = 0, kFprev = 1, kFnew = 2;
constexpr int kRodas3 = 0, kRos4 = 1;

template <int SCHEME>
struct Tab;

// Rodas3 (Sandu et al. 1997): order 3(2), L-stable, stiffly accurate.
template <>
struct Tab<kRodas3> {
  static constexpr double gamma = 0.5;
  static constexpr double a[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {2, 0, 0, 0}, {2, 0, 1, 0}};
  static constexpr double c[4][4] = {{0, 0, 0, 0}, {4, 0, 0, 0}, {1, -1, 0, 0}, {1, -1, -8.0 / 3.0, 0}};
  static constexpr double m[4] = {2, 0, 1, 1};
  static constexpr double e[4] = {0, 0, 0, 1};
  static constexpr int fsrc[4] = {kFy, kFy, kFnew, kFnew};
  static constexpr int est_order = 2;
};

// ROS4 of Shampine (1982): order 4(3), gamma = 1/2, A-stable.
template <>
struct Tab<kRos4> {
  static constexpr double gamma = 0.5;
  static constexpr double a[4][4] = {
      {0, 0, 0, 0}, {2, 0, 0, 0}, {48.0 / 25.0, 6.0 / 25.0, 0, 0}, {48.0 / 25.0, 6.0 / 25.0, 0, 0}};
  static constexpr double c[4][4] = {{0, 0, 0, 0},
                                     {-8, 0, 0, 0},
                                     {372.0 / 25.0, 12.0 / 5.0, 0, 0},
                                     {-112.0 / 125.0, -54.0 / 125.0, -2.0 / 5.0, 0}};
  static constexpr double m[4] = {19.0 / 9.0, 1.0 / 2.0, 25.0 / 108.0, 125.0 / 108.0};
  static constexpr double e[4] = {17.0 / 54.0, 7.0 / 36.0, 0, 125.0 / 108.0};
  static constexpr int fsrc[4] = {kFy, kFnew, kFnew, kFprev};
  static constexpr int est_order = 3;
};

// Coefficient (s, j) of a stage index s known only at run time (s is
// uniform over the cell's lanes): a select over the four compile-time rows.
template <int SCHEME>
__device__ __forceinline__ double tab_a(int s, int j) {
  using T = Tab<SCHEME>;
  return s == 1 ? T::a[1][j] : (s == 2 ? T::a[2][j] : (s == 3 ? T::a[3][j] : T::a[0][j]));
}
template <int SCHEME>
__device__ __forceinline__ double tab_c(int s, int j) {
  using T = Tab<SCHEME>;
  return s == 1 ? T::c[1][j] : (s == 2 ? T::c[2][j] : (s == 3 ? T::c[3][j] : T::c[0][j]));
}
template <int SCHEME>
__device__ __forceinline__ int tab_fsrc(int s) {
  using T = Tab<SCHEME>;
  return s == 1 ? T::fsrc[1] : (s == 2 ? T::fsrc[2] : (s == 3 ? T::fsrc[3] : T::fsrc[0]));
}

// Step factor from the error norm (before the [kFacMin, kFacMax] clamp):
// kFacSafe err^(-1/(q+1)), the fourth root as two correctly rounded square
// roots.
template <int SCHEME>
__device__ __forceinline__ double step_factor(double err) {
  const double ef = fmax(err, 1e-10);
  if constexpr (Tab<SCHEME>::est_order == 3) {
    return kFacSafe / sqrt(sqrt(ef));
  } else {
    return kFacSafe / cbrt(ef);
  }
}

// ---------------------------------------------------------------------------
// mechanism in LDS
// ---------------------------------------------------------------------------
struct MechLds {
  const double *lnA, *b, *EaR, *troe, *eff_am1, *rW;
  const uint4* rint;
  const uint16_t *eff_sp, *sp_off, *sp_ent;
};

__device__ __forceinline__ MechLds mech_views(const unsigned char* s, const MechArgs& m) {
  MechLds L;
  const unsigned char* g = reinterpret_cast<const unsigned char*>(m.blob);
  L.lnA = reinterpret_cast<const double*>(g + m.off_lnA);
  L.b = reinterpret_cast<const double*>(g + m.off_b);
  L.EaR = reinterpret_cast<const double*>(g + m.off_EaR);
  L.troe = reinterpret_cast<const double*>(g + m.off_troe);
  L.rint = reinterpret_cast<const uint4*>(s + m.off_rint);
  L.eff_am1 = reinterpret_cast<const double*>(s + m.off_eff_am1);
  L.eff_sp = reinterpret_cast<const uint16_t*>(s + m.off_eff_sp);
  L.sp_off = reinterpret_cast<const uint16_t*>(s + m.off_sp_off);
  L.sp_ent = reinterpret_cast<const uint16_t*>(s + m.off_sp_ent);
  L.rW = reinterpret_cast<const double*>(s + m.off_rW);
  return L;
}

__device__ __forceinline__ void stage_mech(unsigned char* smem, const MechArgs& m) {
  uint4* d = reinterpret_cast<uint4*>(smem);
  const int n16 = m.lds_bytes / 16;
  for (int i = threadIdx.x; i < n16; i += blockDim.x) d[i] = m.blob[i];
  __syncthreads();
}

// Order one wave's LDS accesses at a point where other lanes' writes must
// be visible (the compiler may not move them across).
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// NASA-7 polynomials of one species at T (low range iff T < Tmid):
// cp/R, h/(RT), g/(RT) and, with JAC, d(cp/R)/dT.
template <bool JAC>
__device__ __forceinline__ void nasa7(const double* a, double T, double rT, double lnT, double& cpR, double& hRT,
                                      double& gRT, double& dcpR) {
  if (!(T < a[7])) a += 8;
  const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], a4 = a[4], a5 = a[5], a6 = a[6];
  cpR = fma(T, fma(T, fma(T, fma(T, a4, a3), a2), a1), a0);
  hRT = fma(T, fma(T, fma(T, fma(T, a4 * 0.2, a3 * 0.25), a2 * (1.0 / 3.0)), a1 * 0.5), a0) + a5 * rT;
  const double sR = fma(a0, lnT, fma(T, fma(T, fma(T, a4 * 0.25, a3 * (1.0 / 3.0)), a2 * 0.5), a1) * T) + a6;
  dcpR = JAC ? fma(T, fma(T, 4.0 * a4, 3.0 * a3), 2.0 * a2) * T + a1 : 0.0;
  gRT = hRT - sR;
}

// Mass-action product of one reaction side (up to 3 distinct species with
// orders 1..3) and its partial derivative by each species, without division
// by a concentration; branch-free (absent slots read species 0 and count as
// order 0). sg accumulates sign * order * g/RT of the side's species.
__device__ __forceinline__ void mass_action(const double* C, unsigned spw, unsigned ordw, int k,
                                            double& P, double (&dP)[3], int (&sp)[3]) {
  double pw[3], dp[3], cc[3];
  int oo[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const bool on = j < k;
    sp[j] = on ? (spw >> (8 * j)) & 0xff : 0;
    oo[j] = on ? (ordw >> (4 * j)) & 0xf : 0;
    cc[j] = C[sp[j]];
  }
  // keep the three loads together (one LDS round trip) rather than sunk
  // into per-slot branches
  asm volatile("" : "+v"(cc[0]), "+v"(cc[1]), "+v"(cc[2]));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int o = oo[j];
    const double c = cc[j];
    const double c2 = c * c;
    pw[j] = o == 0 ? 1.0 : (o == 1 ? c : (o == 2 ? c2 : c2 * c));
    dp[j] = o == 0 ? 0.0 : (o == 1 ? 1.0 : (o == 2 ? 2.0 * c : 3.0 * c2));
  }
  P = pw[0] * pw[1] * pw[2];
  dP[0] = dp[0] * pw[1] * pw[2];
  dP[1] = pw[0] * dp[1] * pw[2];
  dP[2] = pw[0] * pw[1] * dp[2];
}

// Efficiency lists are read in chunks of kEffChunk entries whose loads are
// all issued together (one LDS round trip per chunk rather than two per
// entry); entries past the end read the list's first entry and are not used.
constexpr int kEffChunk = 8;

// Third-body concentration [M] = Ctot + sum_e (alpha_e - 1) C[sp_e], summed
// in list order.
__device__ __forceinline__ double third_body(const MechLds& L, const double* C, double Ctot, int eoff, int neff) {
  double M = Ctot;
  for (int e0 = 0; e0 < neff; e0 += kEffChunk) {
    int sp[kEffChunk];
    double am[kEffChunk], c[kEffChunk];
#pragma unroll
    for (int q = 0; q < kEffChunk; ++q) {
      const int e = e0 + q < neff ? eoff + e0 + q : eoff;
      sp[q] = L.eff_sp[e];
      am[q] = L.eff_am1[e];
    }
#pragma unroll
    for (int q = 0; q < kEffChunk; ++q) c[q] = C[sp[q]];
#pragma unroll
    for (int q = 0; q < kEffChunk; ++q)
      if (e0 + q < neff) M = M + am[q] * c[q];
  }
  return M;
}

// Rate of progress of reaction rx from the cell's concentrations C and
// species g/RT, h/RT: q = theta q0 with q0 = kf prod C^nu' - kr prod C^nu''
// (kr = kf/Kc, Kc = exp(-sum nu g/RT) (p_atm/RT)^sum nu), theta = 1, [M] or
// the Troe falloff factor. With JAC also kf theta, kr theta, q0 dtheta/d[M]
// (times k0/kinf for falloff) and dq/dT at fixed C. Returned in RateOut and,
// when stored, written to RB[rx], RB[nr+rx], RB[2nr+rx], RB[3nr+rx] and
// RB[4nr+rx].
struct RateOut {
  double q, kfT, krT, q0b, dqdT;
};

// Rate evaluation in two parts, so that a caller can interleave two
// reactions: rate_core forms kf, kr and the mass-action products (w is the
// reaction's packed word L.rint[rx]); rate_finish applies the third-body or
// falloff factor and forms the outputs (with STORE also written to RB).
struct RateCore {
  double kf, kr, Pf, Pr, q0, dlnkf, sumh;
};

template <bool JAC>
__device__ __forceinline__ RateCore rate_core(const MechLds& L, const uint4 w, const double* C, const double* gRT,
                                              const double* hRT, int rx, double rT, double lnT, double lnRTp) {
  const bool rev = (w.x >> 30) & 1;
  const int nre = (w.x >> 24) & 0xf, npr = (w.y >> 24) & 0xf;
  const int dnu = static_cast<int>((w.z >> 24) & 0x7f) - 64;
  const double bb = L.b[rx], ear = L.EaR[rx];
  const double lnkf = L.lnA[rx] + bb * lnT - ear * rT;
  const double kf = exp(lnkf);
  double Pf, Pr, sumg = 0.0, sumh = 0.0;
  {
    double pw[3], pr[3], cf[3], cr[3], gf[3], gr[3], hf[3], hr[3];
    int of[3], orr[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const bool onf = j < nre, onr = j < npr;
      const int qf = onf ? (w.x >> (8 * j)) & 0xff : 0;
      const int qr = onr ? (w.y >> (8 * j)) & 0xff : 0;
      of[j] = onf ? (w.z >> (4 * j)) & 0xf : 0;
      orr[j] = onr ? (w.z >> (12 + 4 * j)) & 0xf : 0;
      cf[j] = C[qf];
      cr[j] = C[qr];
      gf[j] = gRT[qf];
      gr[j] = gRT[qr];
      hf[j] = JAC ? hRT[qf] : 0.0;
      hr[j] = JAC ? hRT[qr] : 0.0;
    }
    // one LDS round trip for all species data of the reaction
    asm volatile("" : "+v"(cf[0]), "+v"(cf[1]), "+v"(cf[2]), "+v"(cr[0]), "+v"(cr[1]), "+v"(cr[2]));
    asm volatile("" : "+v"(gf[0]), "+v"(gf[1]), "+v"(gf[2]), "+v"(gr[0]), "+v"(gr[1]), "+v"(gr[2]));
    if (JAC) asm volatile("" : "+v"(hf[0]), "+v"(hf[1]), "+v"(hf[2]), "+v"(hr[0]), "+v"(hr[1]), "+v"(hr[2]));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double cf2 = cf[j] * cf[j], cr2 = cr[j] * cr[j];
      pw[j] = of[j] == 0 ? 1.0 : (of[j] == 1 ? cf[j] : (of[j] == 2 ? cf2 : cf2 * cf[j]));
      pr[j] = orr[j] == 0 ? 1.0 : (orr[j] == 1 ? cr[j] : (orr[j] == 2 ? cr2 : cr2 * cr[j]));
      sumg = sumg - of[j] * gf[j];
      sumg = sumg + orr[j] * gr[j];
      if (JAC) {
        sumh = sumh - of[j] * hf[j];
        sumh = sumh + orr[j] * hr[j];
      }
    }
    Pf = pw[0] * pw[1] * pw[2];
    Pr = pr[0] * pr[1] * pr[2];
  }
  // kr = kf / Kc with Kc = exp(-sum nu g/RT) (p_atm/RT)^(sum nu)
  const double kr = rev ? exp(lnkf + sumg + dnu * lnRTp) : 0.0;
  const double q0 = kf * Pf - kr * Pr;
  const double dlnkf = (bb + ear * rT) * rT;
  return RateCore{kf, kr, Pf, Pr, q0, dlnkf, sumh};
}

template <bool JAC, bool STORE = true>
__device__ __forceinline__ RateOut rate_finish(const MechLds& L, const uint4 w, const RateCore& rc, const double* C,
                                               double* RB, int nr, int rx, double T, double rT, double lnT,
                                               double Ctot) {
  const int type = (w.x >> 28) & 3;
  const bool rev = (w.x >> 30) & 1;
  const int dnu = static_cast<int>((w.z >> 24) & 0x7f) - 64;
  const double kf = rc.kf, kr = rc.kr, Pf = rc.Pf, Pr = rc.Pr, q0 = rc.q0, dlnkf = rc.dlnkf, sumh = rc.sumh;
  double theta = 1.0, beta = 0.0, dthdT = 0.0;
  if (type >= 1) {
    double M = Ctot;
    const int eoff = w.w & 0xffff, neff = (w.w >> 16) & 0xff;
    M = third_body(L, C, M, eoff, neff);
    if (type == 1) {
      theta = M;
      beta = 1.0;
    } else {
      const double* tr = L.troe + 8 * ((w.w >> 24) & 0xff);
      const double k0 = exp(tr[0] + tr[1] * lnT - tr[2] * rT);
      const double dlnk0 = (tr[1] + tr[2] * rT) * rT;
      double Prd = k0 * M / kf;
      if (Prd < 1e-300) Prd = 1e-300;
      const double ta = tr[3];
      const double e3 = exp(-T * tr[4]), e1 = exp(-T * tr[5]);
      double Fc = (1.0 - ta) * e3 + ta * e1;
      double dFc = -(1.0 - ta) * tr[4] * e3 - ta * tr[5] * e1;
      if (tr[7] != 0.0) {
        const double e2 = exp(-tr[6] * rT);
        Fc = Fc + e2;
        dFc = dFc + tr[6] * rT * rT * e2;
      }
      if (Fc < 1e-300) Fc = 1e-300;
      const double Lc = log10(Fc);
      const double c = -0.4 - 0.67 * Lc;
      const double N = 0.75 - 1.27 * Lc;
      const double X = log10(Prd) + c;
      const double den = N - 0.14 * X;
      const double f1 = X / den;
      const double opf = 1.0 + f1 * f1;
      const double lgF = Lc / opf;
      const double F = exp(lgF * kLn10);
      const double lind = Prd / (1.0 + Prd);
      theta = lind * F;
      if (JAC) {
        const double dlogF_dX = -Lc * 2.0 * f1 / (opf * opf) * (N / (den * den));
        const double dlogF_dPr = dlogF_dX / (Prd * kLn10);
        const double dPhi = F / ((1.0 + Prd) * (1.0 + Prd)) + lind * F * kLn10 * dlogF_dPr;
        beta = dPhi * k0 / kf;
        const double dPr_dT = Prd * (dlnk0 - dlnkf);
        const double dL_dT = dFc / (Fc * kLn10);
        const double df1_dL = (-0.67 * den - X * (-1.27 + 0.14 * 0.67)) / (den * den);
        const double dlogF_dL = 1.0 / opf - Lc * 2.0 * f1 * df1_dL / (opf * opf);
        dthdT = dPhi * dPr_dT + lind * (F * kLn10 * dlogF_dL * dL_dT);
      }
    }
  }
  RateOut o{theta * q0, 0.0, 0.0, 0.0, 0.0};
  if (JAC) {
    const double dlnkr = rev ? dlnkf - (sumh * rT - dnu * rT) : 0.0;
    o.kfT = kf * theta;
    o.krT = kr * theta;
    o.q0b = q0 * beta;
    o.dqdT = theta * (kf * dlnkf * Pf - kr * dlnkr * Pr) + q0 * dthdT;
  }
  if (STORE) {
    RB[rx] = o.q;
    if (JAC) {
      RB[nr + rx] = o.kfT;
      RB[2 * nr + rx] = o.krT;
      RB[3 * nr + rx] = o.q0b;
      RB[4 * nr + rx] = o.dqdT;
    }
  }
  return o;
}

template <bool JAC, bool STORE = true>
__device__ __forceinline__ RateOut reaction_rate(const MechLds& L, const uint4 w, const double* C, const double* gRT,
                                                 const double* hRT, double* RB, int nr, int rx, double T, double rT,
                                                 double lnT, double lnRTp, double Ctot) {
  const RateCore rc = rate_core<JAC>(L, w, C, gRT, hRT, rx, rT, lnT, lnRTp);
  return rate_finish<JAC, STORE>(L, w, rc, C, RB, nr, rx, T, rT, lnT, Ctot);
}

template <bool JAC, bool STORE = true>
__device__ __forceinline__ RateOut reaction_rate(const MechLds& L, const double* C, const double* gRT,
                                                 const double* hRT, double* RB, int nr, int rx, double T, double rT,
                                                 double lnT, double lnRTp, double Ctot) {
  return reaction_rate<JAC, STORE>(L, L.rint[rx], C, gRT, hRT, RB, nr, rx, T, rT, lnT, lnRTp, Ctot);
}

}  // namespace dev
}  // namespace chemk
