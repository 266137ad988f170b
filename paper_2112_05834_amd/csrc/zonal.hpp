// Zonal reference mapping around the integrator (paper: Methodology, the
// DLBFoam paragraph): every cell is either integrated or takes the solution
// of a reference cell of similar Bilger mixture fraction Z.
#pragma once

#include <hip/hip_runtime.h>

namespace chemz {

constexpr int kMaxBands = 64;       // Z bands of one zone, each with its own reference

struct ZoneArgs {
  long long n;                 // cells
  int ns;                      // species; a cell's row holds ns + 2 doubles
  const double* phi_in;
  double* phi_out;
  const double* coef;          // [ns] Bilger coefficient b_i of each species
  const double* streams;       // [2] beta of the fuel and of the oxidiser stream
  double z_max, t_tol;
  double dz;                   // band width (0: the whole zone is one band)
  int nb;                      // bands: 1, or floor(z_max / dz) + 1 <= kMaxBands
  signed char* flag;           // [n] band + 1 of a zone cell, then band + 1 if mapped, 0 if integrated
  int* order;                  // [n] queue order; integrated cells fill its tail
  unsigned long long* ctl;     // [b] reference cell of band b (~0 = none), [kMaxBands] integrated cells
  unsigned long long* head;    // queue head of the persistent integration kernel
  double* stash;               // [kMaxBands][ns + 2] each band's reference input row
  int* n_acc;                  // the caller's counters and status (NULL allowed)
  int* n_rej;
  signed char* status;
  int* n_jac;                  // the solver's evaluation counters (NULL allowed)
  int* n_fev;
};

// coef[i] = (sum_e coupling[e] counts[i][e]) / W[i]; streams = (beta(y_fuel),
// beta(y_ox)). Sums in natural index order, one fused multiply-add per term.
hipError_t launch_zone_setup(int ns, int ne, const double* coupling, const int* counts, const double* W,
                             const double* y_fuel, const double* y_ox, double* coef, double* streams,
                             hipStream_t st);
// z[c] = (beta(Y_c) - beta_ox) / (beta_fuel - beta_ox) for n cells.
hipError_t launch_mixture_fraction(long long n, int ns, const double* phi, const double* coef,
                                   const double* streams, double* z, hipStream_t st);
// Resets ctl, marks each zone cell (Z <= z_max) with its band in flag and
// finds each band's reference (its cell of lowest index).
hipError_t launch_zone_classify(const ZoneArgs& a, hipStream_t st);
// Final mapped flags; the integrated cells go to the tail of order, the queue
// head is set to the first of them and the reference's input row is kept.
hipError_t launch_zone_select(const ZoneArgs& a, hipStream_t st);
// Mapped cells: the reference's change of state over the step.
hipError_t launch_zone_apply(const ZoneArgs& a, hipStream_t st);

}  // namespace chemz
