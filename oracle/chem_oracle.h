/* Plain serial FP64 CPU oracle for per-cell stiff chemistry integration.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the reference against which the
 * GPU library is checked. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the GPU product path never
 * calls it and shares no code with it.
 *
 * What it computes (paper: "Introduction" and "Analytical Jacobian and
 * improved ODE solution"): every cell holds a composition vector
 * phi = (T, p, species) that evolves under the stiff kinetics ODE
 * f = d(phi)/dt over one CFD time step; an implicit integrator needs the
 * Jacobian J_ij = df_i/dphi_j, here analytical, and LU factorisation with
 * back substitution of the integrator's matrix.
 *
 * The paper leaves the ODE scheme, rate laws, thermodynamics and controller
 * unnamed. This oracle reads them as: constant-pressure adiabatic reactor with
 * state y = (T, Y_1..Y_Ns) (p held fixed, n = Ns+1); NASA-7 thermo; modified
 * Arrhenius rates, third-body and Troe falloff; reverse rates from the
 * equilibrium constant; Rodas3 (4-stage, order 3(2), L-stable Rosenbrock
 * method, Sandu et al. 1997) with matrix M = I/(gamma h) - J factored by
 * Doolittle LU with partial pivoting (LAPACK getrf semantics).
 *
 * Layouts: phi is cell-major [n_cells][2+Ns] = (T [K], p [Pa], Y_1..Y_Ns);
 * y is [T, Y_1..Y_Ns]; matrices are row-major. All pointers are host
 * pointers owned by the caller.
 */
#ifndef CHEM_ORACLE_H
#define CHEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_mech orc_mech;

typedef struct {
  double rtol;      /* relative tolerance */
  double atol;      /* absolute tolerance, same for T and every Y */
  int max_steps;    /* attempted steps per cell per call */
  int scheme;       /* ORC_RODAS3 (0) or ORC_ROS4 (1) */
  int jacobian;     /* ORC_JAC_ANALYTICAL (0) or ORC_JAC_FD (1) */
  int state;        /* ORC_STATE_FULL (0) or ORC_STATE_NO_BATH (1) */
} orc_opts;

/* The integrated state: all species (n = Ns + 1), or, as pyJac does, without
 * the bath gas, the mechanism's last species, whose mass fraction is then
 * 1 - the sum of the others (n = Ns; needs Ns >= 2). */
enum { ORC_STATE_FULL = 0, ORC_STATE_NO_BATH = 1 };

/* Right-hand side and analytical Jacobian of the integrated state (n = Ns + 1
 * or Ns entries, row-major n x n). Return 0, or -1 on a bad argument. */
int orc_state_rhs(const orc_mech* m, int state, double p, const double* y, double* f);
int orc_state_jac(const orc_mech* m, int state, double p, const double* y, double* J);

/* How the integrator obtains J: analytically, or by forward differences
 * (the conventional way the paper's analytical Jacobian replaces). */
enum { ORC_JAC_ANALYTICAL = 0, ORC_JAC_FD = 1 };

/* Rosenbrock schemes (the paper leaves the scheme unnamed). */
enum { ORC_RODAS3 = 0, ORC_ROS4 = 1 };

/* Per-cell status codes. */
enum { ORC_OK = 0, ORC_MAX_STEPS = 1, ORC_H_UNDERFLOW = 2, ORC_NONFINITE = 3,
       ORC_SINGULAR = 4, ORC_T_RANGE = 5 };

/* Parse a mechanism file; returns 0 or -2 on a parse error (message in
 * orc_last_error()). */
int orc_mech_load(const char* path, orc_mech** out);
void orc_mech_free(orc_mech* m);
int orc_mech_dims(const orc_mech* m, int* n_species, int* n_reactions);
const char* orc_last_error(void);

/* NASA-7 per species at T: cp/R, h/(RT), s/R and d(cp/R)/dT. */
void orc_thermo(const orc_mech* m, double T, double* cp_R, double* h_RT, double* s_R,
                double* dcpR_dT);
/* Rate constants and rates of progress at (T, p, Y): kf, kr (infinite-pressure
 * values for falloff reactions) and q (third-body / falloff factor included). */
void orc_rates(const orc_mech* m, double T, double p, const double* Y, double* kf, double* kr,
               double* q);
/* Molar production rates omega_i [mol m^-3 s^-1] at (T, p, Y). */
void orc_omega(const orc_mech* m, double T, double p, const double* Y, double* omega);
/* Right-hand side f(y) = dy/dt at pressure p. */
void orc_rhs(const orc_mech* m, double p, const double* y, double* f);
/* Analytical Jacobian df/dy, row-major n x n. */
void orc_jac(const orc_mech* m, double p, const double* y, double* J);
/* Forward-difference Jacobian, row-major n x n, from f0 = f(y): column j is
 * (f(y + d_j e_j) - f0) / d_j with d_j = (y_j + s_j) - y_j and
 * s_j = sqrt(u max(1e-5, |y_j|)), u = 2^-53. */
void orc_jac_fd(const orc_mech* m, double p, const double* y, const double* f0, double* J);

/* In-place LU with partial pivoting of a row-major n x n matrix. piv[k] is the
 * row swapped with row k at step k (0-based). Returns 0, or k+1 if the pivot of
 * column k is exactly zero. */
int orc_lu(int n, double* A, int* piv);
/* Solve with the factors of orc_lu; b is overwritten with x. */
void orc_lu_solve(int n, const double* LU, const int* piv, double* b);

/* Coefficients of a scheme in the transformed form: gamma, strictly lower
 * a[4][4] and c[4][4] (row-major, row = stage), solution weights m[4], error
 * weights e[4]. Returns the number of stages, or -1 for an unknown scheme. */
int orc_tableau(int scheme, double* gamma, double* a, double* c, double* m, double* e);
void orc_rodas3_tableau(double* gamma, double* a, double* c, double* m, double* e);
/* One step of size h from y: y_new and the embedded error vector. Returns
 * the LU status (0 or k+1), or -1 for an unknown scheme. */
int orc_step(const orc_mech* m, int scheme, double p, const double* y, double h, double* y_new,
             double* err_vec);
int orc_rodas3_step(const orc_mech* m, double p, const double* y, double h, double* y_new,
                    double* err_vec);

/* Adaptive integration of every cell over [0, dt]. phi_out may alias phi_in.
 * h_io (may be NULL): in, the first substep (<= 0 means dt); out, the
 * controller's next proposal. n_acc, n_rej, status may be NULL. Cells are
 * spread over n_threads host threads with a shared atomic cell counter.
 * Returns 0, or -1 on a bad argument. */
int orc_integrate(const orc_mech* m, long n_cells, double dt, const orc_opts* o,
                  const double* phi_in, double* phi_out, double* h_io, int* n_acc, int* n_rej,
                  signed char* status, int n_threads);

/* The same, also counting for every cell the evaluations of the Jacobian
 * (n_jac: analytical, or one forward-difference Jacobian) and of the
 * right-hand side f (n_fev: every call of f, including the n calls a
 * forward-difference Jacobian makes), counted where they are made. Either
 * may be NULL. */
int orc_integrate_counts(const orc_mech* m, long n_cells, double dt, const orc_opts* o,
                         const double* phi_in, double* phi_out, double* h_io, int* n_acc, int* n_rej,
                         int* n_jac, int* n_fev, signed char* status, int n_threads);

/* Zonal reference mapping (paper: Methodology, the DLBFoam paragraph): a cell
 * is either integrated or takes the solution of a reference cell with a
 * similar Bilger mixture fraction Z.
 *
 * orc_mech_elements: number of elements and, if counts is not NULL, the atom
 * counts [ns][ne] of every species. Returns 0, or -1 for a NULL mechanism.
 *
 * orc_mixture_fraction: Z of n cells phi [n][2+Ns] into z [n]. coupling [ne]
 * weighs the moles of each element per kg of mixture (Bilger: 2 for C, 1/2
 * for H, -1 for O); y_fuel and y_ox [Ns] are the two stream compositions
 * (Z = 1 and Z = 0). Returns 0, or -1 on a bad argument or if the streams have
 * the same coupling value. */
int orc_mech_elements(const orc_mech* m, int* n_elements, int* counts);
int orc_mixture_fraction(const orc_mech* m, const double* coupling, const double* y_fuel,
                         const double* y_ox, long n, const double* phi, double* z);

#ifdef __cplusplus
}
#endif
#endif
