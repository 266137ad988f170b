// Kernel launch interface shared by the C ABI and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chemk {

// Mechanism as seen by a kernel: sizes, offsets of the LDS image sections,
// and global tables.
struct MechArgs {
  int ns, nr;
  int off_lnA, off_b, off_EaR, off_rint, off_troe, off_eff_sp, off_eff_am1, off_sp_off, off_sp_ent,
      off_rW;
  int blob_bytes;          // multiple of 16
  int lds_bytes;           // leading part of the blob staged in LDS (multiple of 16)
  const uint4* blob;       // global copy of the image
  const double* nasa;      // [ns][16]
  const double* W;         // [ns]
};

struct OptsDev {
  double rtol, atol;
  int max_steps;
  int scheme;                   // 0 Rodas3, 1 ROS4
  int jac_fd;                   // 1: Jacobian by forward differences (n extra right-hand sides)
  int no_bath;                  // 1: the last species (bath gas) is not integrated: Y = 1 - sum of the others
};

// Learned-cost logging (records written by the integration kernel).
struct LogArgs {
  float* feats;                 // [cap][4]
  float* target;                // [cap]
  unsigned long long* head;     // record counter
  long long cap;                // 0 = off
};

struct IntegrateArgs {
  MechArgs m;
  OptsDev o;
  double dt;
  long long n;
  const double* phi_in;
  double* phi_out;
  double* h_io;
  int* n_acc;
  int* n_rej;
  signed char* status;
  int* n_jac;                   // evaluations of J per cell, or NULL
  int* n_fev;                   // evaluations of f per cell, or NULL
  int accumulate;               // add counters / keep first failure status
  int cell_doubles;             // per-cell LDS area (doubles)
  int wpb;                      // waves per block
  const int* perm;              // queue order (persistent) or NULL
  unsigned long long* head;     // queue head (persistent)
  int chunk;                    // cells per queue pull
  LogArgs log;
  // workgroup-per-cell kernel: per-slot workspace in HBM (J and M, n x ld
  // column-major each), one slot per resident workgroup
  double* ws;
  long long ws_stride;          // doubles per slot
  int ld;                       // leading dimension of J and M
};

struct EvalArgs {
  MechArgs m;
  long long n;
  const double* phi;
  double* f;
  double* J;
  int cell_doubles;
  int wpb;
  double* ws;
  long long ws_stride;
  int ld;
};

struct LuArgs {
  long long batch;
  int n;
  double* A;
  int* piv;
  int* info;
  double* b;
  int wpb;
  double* ws;
  long long ws_stride;
  int ld;
};

// Kernel variant: state size NN (compiled), lanes per cell G. The
// workgroup-per-cell kernel for larger mechanisms is {kWideNN, 256}.
struct Variant {
  int nn;
  int g;
};
constexpr int kWideNN = 256;          // largest n of the workgroup kernel
constexpr int kWideThreads = 256;     // threads per cell
constexpr int kWidePanel = 12;        // LU panel width
inline int wide_ld(int n) { return (n + 15) & ~15; }
// LDS bytes of the workgroup kernel's per-cell area (after the mechanism prefix)
int wide_cell_bytes(int ns, int nr, int ld);
hipError_t launch_integrate_wide(bool persistent, int grid, const IntegrateArgs& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_eval_wide(int grid, const EvalArgs& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_lu_wide(int grid, const LuArgs& a, size_t lds_bytes, hipStream_t st);
int integrate_wide_blocks_per_cu(bool persistent, size_t lds_bytes);

// Which compiled variants exist for a state size n (returns count, fills out).
int variants_for(int n, Variant* out, int max_out);
// Per-cell LDS doubles for a variant and mechanism.
int cell_doubles(int nn, int nr, int ns);

hipError_t launch_integrate(const Variant& v, bool persistent, int grid, const IntegrateArgs& a,
                            size_t lds_bytes, hipStream_t st);
hipError_t launch_eval(const Variant& v, int grid, const EvalArgs& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_lu(const Variant& v, int grid, const LuArgs& a, hipStream_t st);
// Occupancy (blocks per CU) of the integrate kernel for a block size and LDS size.
int integrate_blocks_per_cu(const Variant& v, bool persistent, int wpb, size_t lds_bytes);

// Small helper kernels.
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, hipStream_t st);
hipError_t launch_copy_f64(double* dst, const double* src, long long n, hipStream_t st);

}  // namespace chemk
