/* chem.h -- C ABI of the MI355X stiff-chemistry integrator (libchem.so).
 *
 * The operation (paper: "Introduction"; "Analytical Jacobian and improved ODE
 * solution"): each CFD cell carries a composition vector phi = (T, p, species)
 * that is advanced over one CFD time step dt by integrating the stiff
 * kinetics ODE f = d(phi)/dt with an implicit integrator that uses the
 * analytical Jacobian J_ij = df_i/dphi_j and an LU factorisation with back
 * substitution. Cells are independent; the paper balances their uneven cost
 * across MPI ranks ("DLBFoam: Dynamic load balancing"), which this library
 * turns into balancing across the waves of one GPU (persistent kernel with an
 * atomic work queue, optionally ordered by a learned cost model).
 *
 * Model used (the paper leaves it unnamed): constant-pressure adiabatic
 * reactor per cell with state y = (T, Y_1..Y_Ns) and p fixed; NASA-7 thermo;
 * modified Arrhenius, third-body and Troe falloff rates; reverse rates from
 * equilibrium constants; Rodas3 (4 stages, order 3 with embedded order 2,
 * L-stable) with M = I/(gamma h) - J factored by LU with partial pivoting.
 *
 * Conventions for every int-returning call: 0 = CHEM_OK, < 0 = error code
 * below; chem_last_error() then returns a message (thread-local, valid until
 * the next failing call on the same thread). No call aborts the process.
 *
 * Device pointers: every array argument named *_dev or documented as device
 * memory must be a device allocation on the solver's HIP device, contiguous,
 * with the stated element type and layout. The caller owns those arrays.
 * Calls that take a stream only enqueue work on it (no host synchronisation)
 * unless stated; pass the hipStream_t as void* (NULL = the null stream).
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define CHEM_OK 0
#define CHEM_EINVAL (-1)       /* bad argument (null pointer, size, layout)   */
#define CHEM_EMECH (-2)        /* mechanism file cannot be parsed / invalid   */
#define CHEM_EHIP (-3)         /* HIP runtime error                           */
#define CHEM_ENOMEM (-4)       /* device or host allocation failed            */
#define CHEM_ESTATE (-5)       /* call not valid in this state               */
#define CHEM_EUNSUPPORTED (-6) /* size not supported by the compiled kernels  */

/* Per-cell status codes (status array of chem_integrate). A failed cell keeps
 * its last accepted state in phi_out; the call itself still returns CHEM_OK. */
#define CHEM_CELL_OK 0
#define CHEM_CELL_MAX_STEPS 1   /* attempted steps reached opts.max_steps     */
#define CHEM_CELL_H_UNDERFLOW 2 /* step size fell below 1e-20 s               */
#define CHEM_CELL_NONFINITE 3   /* non-finite input (T, p or a Y), or p <= 0  */
#define CHEM_CELL_SINGULAR 4    /* exact zero pivot in the LU of M            */
#define CHEM_CELL_T_RANGE 5     /* an accepted step left T in [200, 6000] K   */

/* Rosenbrock schemes (the paper leaves the scheme unnamed), both in the
 * transformed form with M = I/(gamma h) - J: Rodas3 (Sandu et al. 1997, order
 * 3 with embedded order 2, L-stable) and ROS4 (Shampine 1982, order 4 with
 * embedded order 3, A-stable). Both take two new right-hand sides per
 * attempted step; the step factor goes as err^(-1/3) and err^(-1/4). */
#define CHEM_RODAS3 0
#define CHEM_ROS4 1

/* How J is obtained (paper: Introduction and Methodology, the Analytical
 * Jacobian paragraph; Fig. 2): analytically, or by forward differences as
 * conventional ODE codes do, one more right-hand side per state component
 * (column j from the step d_j = (y_j + s_j) - y_j, s_j = sqrt(2^-53
 * max(1e-5, |y_j|))). */
#define CHEM_JAC_ANALYTICAL 0
#define CHEM_JAC_FD 1

/* The integrated state (paper: Methodology, the Analytical Jacobian paragraph;
 * pyJac's state vector omits the bath gas). CHEM_STATE_FULL: T and every Y,
 * n = Ns + 1. CHEM_STATE_NO_BATH: the mechanism's last species is the bath
 * gas; it is not integrated and its mass fraction is 1 - the sum of the
 * others, n = Ns (needs Ns >= 2). The input's last mass fraction is then not
 * read, and phi_out carries 1 - the sum of the others in it. */
#define CHEM_STATE_FULL 0
#define CHEM_STATE_NO_BATH 1

/* Schedules. */
#define CHEM_PLAIN 0              /* one launch per chemistry step, static cell-to-wave map */
#define CHEM_PERSISTENT 1         /* resident waves pull cells from an atomic queue          */
#define CHEM_PERSISTENT_BINNED 2  /* as 1, queue ordered by predicted cost, longest first    */

typedef struct chem_mech chem_mech;     /* opaque, library owned, host side     */
typedef struct chem_solver chem_solver; /* opaque, library owned, one HIP device */

typedef struct {
  double rtol;              /* relative tolerance (default 1e-6)                         */
  double atol;              /* absolute tolerance, T and every Y (default 1e-10)         */
  int32_t max_steps;        /* attempted steps per cell per chemistry step (100000)      */
  int32_t schedule;         /* CHEM_PLAIN / CHEM_PERSISTENT / CHEM_PERSISTENT_BINNED     */
  int32_t cells_per_wave;   /* cells integrated by one 64-lane wave; 0 = autotuned/auto  */
  int32_t queue_chunk;      /* cells taken per atomic queue pull; 0 = auto               */
  int32_t blocks;           /* persistent grid size in blocks; 0 = fill the device       */
  int32_t waves_per_block;  /* 0 = auto                                                  */
  int64_t hbm_budget_bytes; /* workspace budget for in-flight cells; 0 = 50% of free     */
  int32_t scheme;           /* CHEM_RODAS3 (default) or CHEM_ROS4                        */
  int32_t jacobian;         /* CHEM_JAC_ANALYTICAL (default) or CHEM_JAC_FD              */
  int32_t state;            /* CHEM_STATE_FULL (default) or CHEM_STATE_NO_BATH           */
} chem_opts;

/* Fill o with the defaults above. Paper: Results and discussion (the Spray A
 * run's tolerances, atol 1e-10 and rtol 1e-6, are the defaults). */
void chem_opts_default(chem_opts* o);

/* ---- mechanism ---------------------------------------------------------- */

/* Paper: Introduction (the kinetics ODE f of a given mechanism) and
 * Methodology, Analytical Jacobian paragraph (rates and Jacobian generated
 * for a given chemical kinetics mechanism).
 * Parse the text mechanism at path (format: species with W and NASA-7
 * coefficients, reactions with Arrhenius A [SI], b, Ea [J/mol], optional
 * third-body efficiencies and Troe parameters). Host only. *out is owned by
 * the caller and released with chem_mech_free. Errors: CHEM_EINVAL,
 * CHEM_EMECH (message names the offending token). */
int chem_mech_load(const char* path, chem_mech** out);
/* Species and reaction counts (n = Ns + 1 state components). Paper: Results
 * and discussion (the 54-species, 269-reaction mechanism). */
int chem_mech_dims(const chem_mech* m, int32_t* n_species, int32_t* n_reactions);
/* Paper: Methodology, Analytical Jacobian paragraph and Fig. 2 (the cost of
 * right-hand side and Jacobian evaluations per cell).
 * Algorithmic work per evaluation, counted from the mechanism's structure:
 * flops of one right-hand side and of one analytical Jacobian (beyond the
 * right-hand side it also yields), with each exp/log/pow counted as one
 * transcendental (reported separately, not in the flop figures). Any output
 * pointer may be NULL. */
int chem_mech_work(const chem_mech* m, double* flops_rhs, double* flops_jac,
                   double* trans_rhs, double* trans_jac);
void chem_mech_free(chem_mech* m); /* NULL-safe */

/* ---- solver ------------------------------------------------------------- */

/* Paper: Methodology, Analytical Jacobian paragraph (the per-cell stiff ODE
 * solver, its tolerances and its linear algebra).
 * Bind a mechanism to HIP device hip_device: uploads the mechanism image
 * (the part staged in LDS by every block plus thermo tables) and allocates the
 * queue and scratch. The mechanism may be freed afterwards. Errors:
 * CHEM_EINVAL, CHEM_EHIP, CHEM_ENOMEM, CHEM_EUNSUPPORTED (state size n = Ns+1
 * beyond the compiled kernels). */
int chem_solver_create(const chem_mech* m, const chem_opts* o, int32_t hip_device,
                       chem_solver** out);
void chem_solver_free(chem_solver* s); /* NULL-safe; synchronises the device */
/* Replace or read the solver's options (same validation as create). Paper:
 * Methodology, Analytical Jacobian paragraph and Fig. 2 (solver tolerances). */
int chem_solver_set_opts(chem_solver* s, const chem_opts* o);
int chem_solver_get_opts(const chem_solver* s, chem_opts* o);

/* Paper: Introduction (phi = (p, T, species) advanced by f = dphi/dt) and
 * Methodology, Analytical Jacobian paragraph (implicit integration with the
 * analytical J, LU decomposition and back substitution); the schedules serve
 * Methodology, DLBFoam paragraph (balancing the uneven per-cell cost).
 * Integrate every cell over [0, dt] (one chemistry step).
 *   phi_in, phi_out : device, [n_cells][2+Ns] float64 = (T [K], p [Pa], Y_1..Y_Ns);
 *                     phi_out may alias phi_in exactly (not partially).
 *   h_io   : device [n_cells] float64 or NULL. In: first substep (<= 0 means
 *            dt). Out: the controller's next proposal (for chained steps).
 *   n_acc, n_rej : device [n_cells] int32 or NULL: accepted / rejected
 *            attempts of this call.
 *   status : device [n_cells] int8 or NULL: CHEM_CELL_* per cell.
 *   stream : hipStream_t; work is enqueued only.
 * Results do not depend on the schedule, cells_per_wave, queue_chunk or
 * blocks: every cell's arithmetic is identical (bit for bit) under all of
 * them. n_cells = 0 is a no-op. Errors: CHEM_EINVAL (n_cells < 0, dt <= 0 or
 * not finite, null phi, partial aliasing), CHEM_ESTATE (binned schedule
 * without a usable model is not an error: it falls back to queue order),
 * CHEM_EHIP. */
int chem_integrate(chem_solver* s, int64_t n_cells, double dt, const double* phi_in,
                   double* phi_out, double* h_io, int32_t* n_acc, int32_t* n_rej,
                   int8_t* status, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * chemistry step as chem_integrate on the persistent queue in index order
 * (learned binning is not applied, no cost-model log record and no kernel
 * timing event is made), that allocates and frees nothing. Its queue head,
 * and for state sizes above 64 the J and M workspace slots of the
 * workgroup kernel, live in a static device array of
 * CHEM_NOALLOC_SCRATCH_BYTES (128 MiB) that every GPU the library runs on
 * holds until the process ends; its address is looked up once per device
 * when the first solver on that device is created. The workgroup kernel
 * gets min(resident workgroups, (128 MiB - 256 B) / (2 n ld 8 B)) slots
 * (289 for n = 161, against 512 in chem_integrate's default budget); a
 * state size whose one slot would not fit is rejected with
 * CHEM_EUNSUPPORTED (none up to n = 256 is). The queue head is reset by a
 * kernel at the start of every call. All calls on one GPU share that GPU's
 * array, so two calls that overlap in time on one GPU (on different streams
 * or from different solvers) race and give wrong results: serialise them.
 * Arrays, results (bit-identical to chem_integrate under any schedule) and
 * errors as chem_integrate. */
#define CHEM_NOALLOC_SCRATCH_BYTES (128ll << 20)
int chem_integrate_noalloc(chem_solver* s, int64_t n_cells, double dt, const double* phi_in,
                           double* phi_out, double* h_io, int32_t* n_acc, int32_t* n_rej,
                           int8_t* status, void* stream);

/* Paper: Results and discussion (chemistry is solved in every CFD iteration;
 * the Spray A run times 100 of them).
 * n_steps chained chemistry steps of the same dt, each feeding the next (h_io
 * carried between them), captured once into a HIP graph and replayed; phi_out
 * holds the final state, n_acc / n_rej accumulate over the steps and status is
 * the first non-zero status of the steps. phi_in is not modified; the library
 * ping-pongs through an internal buffer. The graph is cached per (pointers,
 * sizes, options) and rebuilt when they change. If the caller is capturing the
 * stream already, the steps go straight into the caller's graph and the
 * solver's own graph is left alone; call once outside the capture first, so
 * that the internal buffers exist. Errors as chem_integrate. */
int chem_integrate_steps(chem_solver* s, int32_t n_steps, int64_t n_cells, double dt,
                         const double* phi_in, double* phi_out, double* h_io, int32_t* n_acc,
                         int32_t* n_rej, int8_t* status, void* stream);

/* Paper: Methodology (the ODE solver's cost per cell is what the load
 * balancing distributes; Fig. 2 separates the Jacobian's share of it).
 * Per-cell counts of evaluations, written by every later integration call of
 * this solver (chem_integrate, chem_integrate_noalloc, chem_integrate_steps
 * and chem_integrate_zonal) next to n_acc and n_rej:
 *   n_jac : device [n_cells] int32 or NULL: Jacobian evaluations (analytical,
 *           or one forward-difference Jacobian), one per step start: once at
 *           the start and after every accepted step that the integration
 *           continues from;
 *   n_fev : device [n_cells] int32 or NULL: evaluations of the right-hand
 *           side f: one per step start, the n more that a forward-difference
 *           Jacobian makes, and the stages of every attempt whose LU
 *           succeeded that need f at a new point (two per attempt for Rodas3
 *           and for ROS4).
 * Both arrays hold capacity entries (int32), must stay valid while calls use
 * them, and are overwritten per call (chem_integrate_steps adds over its
 * steps; cells that chem_integrate_zonal maps get 0); a later call with more
 * than capacity cells fails with CHEM_EINVAL before any work is enqueued.
 * Pass NULL for both to stop (capacity is then ignored). The pointers are
 * kept, not owned; a cached graph of chained steps is dropped so that the
 * next chem_integrate_steps captures them. Errors: CHEM_EINVAL (s NULL,
 * capacity < 0, or capacity 0 with a counter array). */
int chem_eval_counters(chem_solver* s, int32_t* n_jac, int32_t* n_fev, int64_t capacity);

/* ---- kernel-level entry points (tests and roofline measurements) -------- */

/* Paper: Methodology, Analytical Jacobian paragraph: the right-hand side
 * (reaction rate evaluations) and J_ij = df_i/dphi_j.
 * Right-hand side f(y) and analytical Jacobian at every cell's state.
 *   phi : device [n_cells][2+Ns]; f : device [n_cells][n] (n = Ns+1, order
 *   T, Y_1..Y_Ns); J : device [n_cells][n][n] row-major (df_i/dy_j) or NULL. */
int chem_eval_rhs_jac(chem_solver* s, int64_t n_cells, const double* phi, double* f, double* J,
                      void* stream);
/* Paper: Methodology, Analytical Jacobian paragraph: the LU decomposition and
 * back substitution of the integrator (LAPACK routines in the paper).
 * Batched LU with partial pivoting (LAPACK getrf semantics: piv[k] is the row
 * swapped with row k at step k, 0-based; ties go to the lowest row) of
 * row-major n x n matrices A[batch][n][n], in place; info[b] = 0 or k+1 for
 * the first exactly-zero pivot. Then, if b is not NULL, solves A x = b for
 * b[batch][n] in place. n must equal the solver's state size. */
int chem_lu_batch(chem_solver* s, int64_t batch, double* A, int32_t* piv, int32_t* info,
                  double* b, void* stream);
/* Paper: Methodology, the Analytical Jacobian paragraph (LAPACK's LU and back
 * substitution) and Fig. 2. The vendor routine for comparison with the
 * library's own LU, not used by any integration: rocSOLVER's
 * dgetrf_strided_batched, then, if b is not NULL, dgetrs_strided_batched for
 * one right-hand side, on batch column-major n x n matrices A (device,
 * [batch][n][n] with element (i, j) at j n + i) in place. piv: device int32
 * [batch][n], LAPACK's 1-based interchanges; info: device int32 [batch];
 * b: device [batch][n] or NULL. Enqueued on stream, on the current HIP
 * device. rocSOLVER and rocBLAS are loaded at the first call (dlopen) and a
 * rocBLAS handle is kept per device. Errors: CHEM_EINVAL, CHEM_EUNSUPPORTED
 * (the libraries cannot be loaded), CHEM_EHIP. */
int chem_lu_batch_rocsolver(int32_t n, int64_t batch, double* A, int32_t* piv, int32_t* info,
                            double* b, void* stream);

/* ---- learned cost model (changes scheduling only, never results) ------- */
/* Paper for every call of this block: Methodology, DLBFoam paragraph (a
 * cell's cost depends on its local thermochemical state; problems move from
 * busy to idle workers). Here a model predicts the cost so that the queue
 * hands out the costliest cells first. */

/* Keep a device log of (features[4], ln substeps) per integrated cell, up to
 * capacity records (ring; later records overwrite). capacity 0 disables. */
int chem_log_enable(chem_solver* s, int64_t capacity);
/* Copy the log into caller buffers (device, feats [cap][4] float32, target
 * [cap] float32) and write the number of valid records to *n_out (host).
 * Synchronises the stream. */
int chem_log_fetch(chem_solver* s, float* feats_dev, float* target_dev, int64_t* n_out,
                   void* stream);
/* Features of every cell (device [n][4] float32), as the predictor sees them. */
int chem_features(chem_solver* s, int64_t n_cells, double dt, const double* phi, float* feats,
                  void* stream);

typedef struct {
  int32_t epochs;  /* passes over the samples (default 10)          */
  int32_t batch;   /* minibatch size (default 4096)                 */
  float lr, beta1, beta2, eps;  /* Adam (1e-3, 0.9, 0.999, 1e-8)   */
  uint64_t seed;   /* weight init and shuffling                     */
} chem_train_opts;
void chem_train_opts_default(chem_train_opts* t);

/* Train the 4->64->64->1 ReLU MLP (BF16 weights and activations as matmul
 * operands, FP32 accumulation, FP32 master weights, Adam) to predict ln
 * substeps from the 4 features, on n samples (device float32). Fits the
 * feature standardisation and the 8 bin edges (octiles of the training
 * predictions). Synchronises the stream. */
int chem_model_train(chem_solver* s, int64_t n, const float* feats_dev, const float* target_dev,
                     const chem_train_opts* t, void* stream);
/* Predicted ln substeps for n cells' features (device float32 in / out). */
int chem_model_predict(chem_solver* s, int64_t n, const float* feats_dev, float* pred_dev,
                       void* stream);
/* Use given per-cell costs (device float32 [n_cells], same unit as the
 * prediction: ln substeps) instead of the model's prediction for binned
 * calls on exactly n_cells cells, binned with the model's edges (for
 * comparison against bins sorted by true cost); NULL clears. The buffer must
 * stay valid while set. Without model edges the queue order is used. */
int chem_set_cost_override(chem_solver* s, int64_t n_cells, const float* cost_dev);
/* Model state as a file: weights (FP32 master), normalisation, bin edges. */
int chem_model_save(const chem_solver* s, const char* path);
int chem_model_load(chem_solver* s, const char* path);
/* Whether the last binned launch used the model or an override (1) or fell
 * back to queue order (0: no model, or a non-finite cost, detected on the
 * device). Reads a device flag: synchronises with the device. */
int chem_last_binning_used(const chem_solver* s, int32_t* used);

/* Model weights in host memory: params [4545] float32 in the order
 * W1 [64][4], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 (row = output
 * unit); norm [8] = feature means [4] then standard deviations [4]; edges [7]
 * ascending bin edges. get: any pointer may be NULL; CHEM_ESTATE without
 * weights (or without edges when edges is requested). set: norm NULL means
 * means 0 and deviations 1; edges NULL leaves the model without edges. */
int chem_model_get(const chem_solver* s, float* params, float* norm, float* edges);
int chem_model_set(chem_solver* s, const float* params, const float* norm, const float* edges);
/* Mean squared error and its gradient (float32 [4545], device) of the
 * current weights over n samples taken as one minibatch (features and
 * targets as for chem_model_train); loss_dev: one float (device). */
int chem_model_grad(chem_solver* s, int64_t n, const float* feats_dev, const float* target_dev,
                    float* grad_dev, float* loss_dev, void* stream);
/* The seven octile edges of n finite costs (device float32): the values at
 * ascending sorted positions floor(k n / 8), k = 1..7, written to host
 * edges[7]. Synchronises the stream. */
int chem_bin_edges(chem_solver* s, int64_t n, const float* cost_dev, float* edges, void* stream);
/* Queue order for n costs (device float32): cells of bin 7 (cost >= edges[6])
 * first down to bin 0, cell index ascending within a bin; identity when any
 * cost is not finite. edges: host [7], NULL = the model's. perm_dev: device
 * int32 [n], caller-owned. */
int chem_bin_order(chem_solver* s, int64_t n, const float* cost_dev, const float* edges, int32_t* perm_dev,
                   void* stream);

/* ---- autotuning --------------------------------------------------------- */

/* Time the candidate launch shapes on n_sample cells (device
 * [n_sample][2+Ns]) for the solver's current schedule and keep the fastest in
 * the solver's options. Candidates: every compiled cells-per-wave variant,
 * 1, 2 or 4 waves per block (as far as the LDS allows), and queue chunks 1,
 * 2, 4, ..., 64 for the persistent schedules. Blocks per compute unit follow
 * from the LDS footprint and are not searched. Synchronises. Results are
 * unaffected (the arithmetic per cell is the same for all shapes). The load
 * balancing this serves is the paper's (Methodology: load balancing of the
 * chemistry problems); the search is this library's. */
int chem_autotune(chem_solver* s, int64_t n_sample, const double* phi_sample_dev, double dt,
                  void* stream);

/* chem_autotune through a cache file (host path, JSON lines, one object per
 * tuned configuration:
 *   {"key": "...", "cells_per_wave": c, "waves_per_block": w,
 *    "queue_chunk": q, "ms": t}).
 * The key names the mechanism (FNV-1a 64 of its packed image), the state
 * size, the schedule, n_sample, dt, the device architecture and its
 * compute-unit count. If a line with this key holds a shape the solver can
 * run, the last such line sets the solver's options with nothing timed and
 * *from_cache = 1. Otherwise the shapes are timed as by chem_autotune, the
 * fastest is kept and appended to the file (created if missing), and
 * *from_cache = 0. Lines that do not parse are skipped. Errors: CHEM_EINVAL
 * for bad arguments or a file that cannot be written. */
int chem_autotune_cached(chem_solver* s, const char* cache_path, int64_t n_sample, const double* phi_sample_dev,
                         double dt, void* stream, int32_t* from_cache);

/* Paper: Methodology, Analytical Jacobian paragraph (the dense Jacobian and
 * its LU, here kept in HBM for large mechanisms).
 * Workspace of the workgroup-per-cell path (state sizes above 64): number of
 * HBM slots (cells in flight; one per resident workgroup, at most
 * hbm_budget_bytes in total, default half the free device memory) and bytes
 * per slot (J and M, 2 n ld doubles with ld = n rounded up to 16). Allocates
 * the slots if needed. Both are 0 for smaller state sizes, whose cells need
 * no HBM workspace. */
int chem_workspace_info(chem_solver* s, int32_t* slots, int64_t* bytes_per_slot);

/* ---- zonal reference mapping ---------------------------------------- */
/* Paper: Methodology, the DLBFoam paragraph. A cell is either integrated or
 * takes the solution of a reference cell with a similar Bilger mixture
 * fraction Z. Read here as:
 *   beta(Y) = sum_i Y_i / W_i * sum_e coupling[e] a_{e,i}  (a = atom counts),
 *   Z = (beta(Y) - beta(y_ox)) / (beta(y_fuel) - beta(y_ox));
 * the zone is every cell with Z <= z_max, split into Z bands of width dz
 * (chem_zone_bands; one band by default), and each band's reference is its
 * zone cell of lowest index. A zone cell whose |T - T_ref| <= t_tol for its
 * band's reference is mapped: it takes that reference's change of T and of
 * every Y over the step (p kept). Every call of this block cites this
 * passage. */

/* Number of elements of the mechanism and, if counts is not NULL, the atom
 * counts of every species: host int32 [Ns][n_elements], row-major. */
int chem_mech_elements(const chem_mech* m, int32_t* n_elements, int32_t* counts);

/* Set the mixture-fraction definition and the mapping thresholds of a solver.
 * coupling: host [n_elements], the weight of each element's moles per kg of
 * mixture (Bilger: 2 for carbon, 1/2 for hydrogen, -1 for oxygen, 0 for the
 * rest). y_fuel, y_ox: host [Ns], the stream compositions (Z = 1 and 0).
 * z_max and t_tol [K] are compared with <=. Allocates the solver's zone
 * buffers on first use and synchronises the device. Errors: CHEM_EINVAL (NULL
 * or non-finite argument, t_tol < 0, or streams with the same beta),
 * CHEM_EHIP; after an error the solver has no zone definition until the
 * next successful call. Do not call while a zonal integration of this solver
 * is in flight. */
int chem_zone_config(chem_solver* s, const double* coupling, const double* y_fuel, const double* y_ox,
                     double z_max, double t_tol);

/* Split the zone into bands of Z: band b = floor(max(Z, 0) / dz), each with
 * its own reference (its cell of lowest index), so that a cell is mapped only
 * from a reference of similar Z. dz = 0 (the default) keeps the whole zone
 * as one band. At most 64 bands (floor(z_max / dz) + 1). Errors: CHEM_EINVAL
 * (dz < 0, non-finite, or too many bands for the configured z_max). */
int chem_zone_bands(chem_solver* s, double dz);

/* Z of n cells: phi device [n][2+Ns] in, z device [n] FP64 out; enqueued on
 * stream. Errors: CHEM_EINVAL, CHEM_ESTATE (no chem_zone_config yet). */
int chem_mixture_fraction(chem_solver* s, int64_t n_cells, const double* phi, double* z, void* stream);

/* chem_integrate with zonal reference mapping: same arrays and semantics as
 * chem_integrate for the integrated cells. A mapped cell gets
 * phi_out = phi_in + (reference's phi_out - phi_in) for T and Y, its p
 * unchanged, n_acc = n_rej = 0, the reference's status, and its h_io left as
 * it was. mapped: device int8 [n] out (band + 1 of a mapped cell, so 1 with
 * one band; 0 for an integrated cell), or NULL.
 * The integrated cells always go through the persistent queue (learned
 * binning is not applied to them). Enqueue only, no host synchronisation,
 * except that a call with more cells than any earlier one first synchronises
 * the stream and allocates the solver's flag and order buffers (int8 and
 * int32 per cell), so capture such a call only after one of at least its
 * size. The solver's zone buffers are shared by its calls: do not overlap two
 * zonal calls of one solver on different streams. n_cells at most
 * 2^31 - 1. Errors: as chem_integrate, plus CHEM_ESTATE (no
 * chem_zone_config yet). */
int chem_integrate_zonal(chem_solver* s, int64_t n_cells, double dt, const double* phi_in, double* phi_out,
                         double* h_io, int32_t* n_acc, int32_t* n_rej, int8_t* status, int8_t* mapped,
                         void* stream);

/* ---- kernel timing ---------------------------------------------------- */
/* Paper: Fig. 2 and Results and discussion (evaluation and CPU times of the
 * chemistry solution), measured here per integration launch. */

/* enable != 0: from now on record a pair of HIP events on the caller's
 * stream around every integration-kernel launch made outside graph capture
 * (clears earlier records); enable == 0: stop recording and free them. */
int chem_kernel_timing(chem_solver* s, int32_t enable);
/* Wait for the recorded launches and write their durations in milliseconds
 * (launch order, at most cap) to host ms_out; *n_out = number written. The
 * records are cleared. */
int chem_kernel_times(chem_solver* s, float* ms_out, int32_t cap, int32_t* n_out);

/* Message of the last failing call on this thread (utility; no paper
 * passage). */
const char* chem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
