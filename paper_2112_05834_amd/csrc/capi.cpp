// C ABI of the stiff-chemistry integrator: argument checking, launch shape
// selection, the persistent work queue, chained steps in a HIP graph, and
// the learned cost model driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/chem.h"
#include "kernels.hpp"
#include "mech.hpp"
#include "model.hpp"
#include "zonal.hpp"

struct chem_mech {
  chem::MechHost host;
  chem::Packed packed;
  chem::Work work;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return CHEM_EHIP;
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t _e = (expr);                 \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hipGetDevice(&prev);
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    hipGetDevice(&cur);
    if (prev >= 0 && cur != prev) hipSetDevice(prev);
  }
};

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

// ---------------------------------------------------------------------------
// Static device scratch of the allocation-free entry point
// (chem_integrate_noalloc): control words first (the persistent queue head),
// then the workgroup kernel's J and M workspace slots. Every GPU the library
// runs on holds its own copy until the process ends. In host code the name
// `scratch` stands for the array only as a symbol: kernels and copies get the
// device address looked up for the current device, never the name itself.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = CHEM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");
constexpr size_t kScratchCtl = 256;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_addr;   // per device

// The address of `scratch` on device dev, which must be current. Looked up
// once per device; later calls return the kept address.
int scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr.size() <= static_cast<size_t>(dev)) g_scratch_addr.resize(dev + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(CHEM_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_addr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_addr[dev];
  return CHEM_OK;
}
}  // namespace

struct chem_solver {
  int dev = 0;
  int cus = 0;
  std::string arch;                  // device architecture name
  unsigned long long mech_fp = 0;    // FNV-1a 64 of the packed mechanism image
  chem_opts opts{};
  int ns = 0, nr = 0, n = 0;
  chemk::MechArgs margs{};
  void* d_blob = nullptr;
  double* d_nasa = nullptr;
  double* d_W = nullptr;
  unsigned long long* d_head = nullptr;   // [0] queue head, [1] log head
  int32_t* d_njac = nullptr;              // caller's per-cell evaluation counters (chem_eval_counters)
  int32_t* d_nfev = nullptr;
  int64_t counters_cap = 0;               // entries they hold
  unsigned char* scratch = nullptr;       // this device's address of the static scratch array
  chemk::Variant variants[8];
  int nvariants = 0;
  chem::Work work{};
  // chained steps
  double* d_ping = nullptr;
  size_t ping_cells = 0;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_src = nullptr;
  hipStream_t capture_stream = nullptr;   // graphs are captured here, launched on the caller's stream
  struct {
    int32_t n_steps = 0;
    int64_t n_cells = 0;
    double dt = 0;
    const void *in = nullptr, *out = nullptr, *h = nullptr, *a = nullptr, *r = nullptr, *s = nullptr;
    hipStream_t st = nullptr;
    chem_opts o{};
  } gkey;
  // learned cost model and binning
  chem_model::Model model;
  int last_binning_used = 0;
  const float* cost_override = nullptr;
  int64_t cost_override_n = 0;
  // workgroup-per-cell kernel (state sizes above one wave): per-slot HBM
  // workspace for J and M, one slot per resident workgroup
  bool wide = false;
  int ld = 0;
  size_t wide_lds = 0;
  int wide_slots = 0;
  int64_t wide_budget = -1;      // budget the slots were sized for
  double* d_ws = nullptr;
  long long ws_stride = 0;       // doubles per slot
  // kernel timing: event pairs around integration launches
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
  // logging
  float* log_feats = nullptr;
  float* log_target = nullptr;
  int64_t log_cap = 0;
  // zonal reference mapping
  int ne = 0;
  std::vector<int> elem;              // [ns][ne] atom counts
  bool zone_ready = false;
  double z_max = 0, t_tol = 0;
  double dz = 0;                      // Z band width (0: one band)
  double* d_zone = nullptr;           // coef [ns], streams [2], reference rows [kMaxBands][ns+2]
  unsigned long long* d_zctl = nullptr;
  signed char* d_zflag = nullptr;
  int* d_zorder = nullptr;
  int64_t zone_cap = 0;
};

constexpr unsigned long long kFnvBasis = 0xcbf29ce484222325ull;
unsigned long long fnv1a(const void* p, size_t n, unsigned long long h) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

namespace chem {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace chem

extern "C" {

const char* chem_last_error(void) { return g_err.c_str(); }

void chem_opts_default(chem_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-6;
  o->atol = 1e-10;
  o->max_steps = 100000;
  o->schedule = CHEM_PLAIN;
}

int chem_mech_load(const char* path, chem_mech** out) {
  if (!path || !out) return fail(CHEM_EINVAL, "chem_mech_load: null argument");
  *out = nullptr;
  auto m = std::make_unique<chem_mech>();
  std::string err;
  if (!chem::parse_mechanism(path, m->host, err)) return fail(CHEM_EMECH, err);
  m->packed = chem::pack(m->host);
  m->work = chem::count_work(m->host);
  *out = m.release();
  return CHEM_OK;
}

int chem_mech_dims(const chem_mech* m, int32_t* ns, int32_t* nr) {
  if (!m) return fail(CHEM_EINVAL, "chem_mech_dims: null mechanism");
  if (ns) *ns = m->host.ns;
  if (nr) *nr = m->host.nr;
  return CHEM_OK;
}

int chem_mech_work(const chem_mech* m, double* f_rhs, double* f_jac, double* t_rhs, double* t_jac) {
  if (!m) return fail(CHEM_EINVAL, "chem_mech_work: null mechanism");
  if (f_rhs) *f_rhs = m->work.f_rhs;
  if (f_jac) *f_jac = m->work.f_jac;
  if (t_rhs) *t_rhs = m->work.t_rhs;
  if (t_jac) *t_jac = m->work.t_jac;
  return CHEM_OK;
}

void chem_mech_free(chem_mech* m) { delete m; }

static int check_opts(const chem_opts* o) {
  if (!o) return fail(CHEM_EINVAL, "null options");
  if (!(o->rtol > 0) || !(o->atol > 0) || !std::isfinite(o->rtol) || !std::isfinite(o->atol))
    return fail(CHEM_EINVAL, "rtol and atol must be positive and finite");
  if (o->max_steps < 1) return fail(CHEM_EINVAL, "max_steps must be >= 1");
  if (o->schedule < CHEM_PLAIN || o->schedule > CHEM_PERSISTENT_BINNED)
    return fail(CHEM_EINVAL, "unknown schedule");
  if (o->cells_per_wave < 0 || o->cells_per_wave > 8 || (o->cells_per_wave & (o->cells_per_wave - 1)))
    return fail(CHEM_EINVAL, "cells_per_wave must be 0, 1, 2, 4 or 8");
  if (o->queue_chunk < 0 || o->blocks < 0 || o->waves_per_block < 0 || o->waves_per_block > 4 ||
      o->hbm_budget_bytes < 0)
    return fail(CHEM_EINVAL, "negative launch option or waves_per_block > 4");
  if (o->scheme != CHEM_RODAS3 && o->scheme != CHEM_ROS4) return fail(CHEM_EINVAL, "unknown scheme");
  if (o->jacobian != CHEM_JAC_ANALYTICAL && o->jacobian != CHEM_JAC_FD)
    return fail(CHEM_EINVAL, "unknown jacobian mode");
  if (o->state != CHEM_STATE_FULL && o->state != CHEM_STATE_NO_BATH) return fail(CHEM_EINVAL, "unknown state");
  return CHEM_OK;
}

int chem_solver_create(const chem_mech* m, const chem_opts* o, int32_t dev, chem_solver** out) {
  if (!m || !out) return fail(CHEM_EINVAL, "chem_solver_create: null argument");
  *out = nullptr;
  chem_opts def;
  chem_opts_default(&def);
  if (!o) o = &def;
  if (int rc = check_opts(o)) return rc;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (dev < 0 || dev >= ndev) return fail(CHEM_EINVAL, "hip_device out of range");
  // handed to the caller on success; on any error below, freed together with
  // the device memory allocated so far
  std::unique_ptr<chem_solver, void (*)(chem_solver*)> s(new chem_solver(), chem_solver_free);
  s->dev = dev;
  s->opts = *o;
  s->ns = m->host.ns;
  s->nr = m->host.nr;
  s->n = s->ns + 1;
  s->work = m->work;
  s->ne = m->host.ne;
  s->elem = m->host.elem;
  s->nvariants = chemk::variants_for(s->n, s->variants, 8);
  if (s->nvariants == 0 && s->n <= chemk::kWideNN) {
    s->wide = true;
    s->variants[0] = chemk::Variant{chemk::kWideNN, chemk::kWideThreads};
    s->nvariants = 1;
    s->ld = chemk::wide_ld(s->n);
    s->ws_stride = 2LL * s->n * s->ld;
  }
  if (s->nvariants == 0)
    return fail(CHEM_EUNSUPPORTED, "no compiled kernel for state size " + std::to_string(s->n));
  DeviceGuard g(dev);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  s->cus = prop.multiProcessorCount;
  s->arch = prop.gcnArchName;
  const chem::Packed& P = m->packed;
  s->mech_fp = fnv1a(P.blob.data(), P.blob.size(), kFnvBasis);
  s->mech_fp = fnv1a(P.nasa.data(), P.nasa.size() * sizeof(double), s->mech_fp);
  s->mech_fp = fnv1a(P.W.data(), P.W.size() * sizeof(double), s->mech_fp);
  HIP_TRY(hipMalloc(&s->d_blob, P.blob.size()), "hipMalloc");
  HIP_TRY(hipMemcpy(s->d_blob, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMalloc(&s->d_nasa, P.nasa.size() * sizeof(double)), "hipMalloc");
  HIP_TRY(hipMemcpy(s->d_nasa, P.nasa.data(), P.nasa.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMalloc(&s->d_W, P.W.size() * sizeof(double)), "hipMalloc");
  HIP_TRY(hipMemcpy(s->d_W, P.W.data(), P.W.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  HIP_TRY(hipMalloc(&s->d_head, 4 * sizeof(unsigned long long)), "hipMalloc");
  HIP_TRY(hipMemset(s->d_head, 0, 4 * sizeof(unsigned long long)), "hipMemset");
  chemk::MechArgs& a = s->margs;
  a.ns = s->ns;
  a.nr = s->nr;
  a.off_lnA = P.off_lnA;
  a.off_b = P.off_b;
  a.off_EaR = P.off_EaR;
  a.off_rint = P.off_rint;
  a.off_troe = P.off_troe;
  a.off_eff_sp = P.off_eff_sp;
  a.off_eff_am1 = P.off_eff_am1;
  a.off_sp_off = P.off_sp_off;
  a.off_sp_ent = P.off_sp_ent;
  a.off_rW = P.off_rW;
  a.blob_bytes = static_cast<int>(P.blob.size());
  a.lds_bytes = P.lds_bytes;
  a.blob = static_cast<const uint4*>(s->d_blob);
  a.nasa = s->d_nasa;
  a.W = s->d_W;
  if (int rc = chem_model::init(s->model)) return fail(rc, chem_model::last_error());
  if (s->wide) {
    s->wide_lds = static_cast<size_t>(a.lds_bytes) + chemk::wide_cell_bytes(s->ns, s->nr, s->ld);
    if (s->wide_lds > kMaxLds)
      return fail(CHEM_EUNSUPPORTED, "mechanism and one cell's work area exceed the 160 KB LDS");
  }
  if (int rc = scratch_address(dev, &s->scratch)) return rc;
  HIP_TRY(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
  *out = s.release();
  return CHEM_OK;
}

static void clear_timing(chem_solver* s) {
  for (auto& e : s->tev) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  s->tev.clear();
}

static void drop_graph(chem_solver* s) {
  if (s->graph) hipGraphExecDestroy(s->graph);
  if (s->graph_src) hipGraphDestroy(s->graph_src);
  s->graph = nullptr;
  s->graph_src = nullptr;
  s->gkey.n_steps = 0;
}

void chem_solver_free(chem_solver* s) {
  if (!s) return;
  DeviceGuard g(s->dev);
  hipDeviceSynchronize();
  drop_graph(s);
  clear_timing(s);
  chem_model::release(s->model);
  hipFree(s->d_blob);
  hipFree(s->d_nasa);
  hipFree(s->d_W);
  hipFree(s->d_head);
  hipFree(s->d_ping);
  hipFree(s->d_ws);
  hipFree(s->log_feats);
  hipFree(s->log_target);
  hipFree(s->d_zone);
  hipFree(s->d_zctl);
  hipFree(s->d_zflag);
  hipFree(s->d_zorder);
  if (s->capture_stream) hipStreamDestroy(s->capture_stream);
  delete s;
}

int chem_solver_set_opts(chem_solver* s, const chem_opts* o) {
  if (!s) return fail(CHEM_EINVAL, "null solver");
  if (int rc = check_opts(o)) return rc;
  s->opts = *o;
  return CHEM_OK;
}

int chem_solver_get_opts(const chem_solver* s, chem_opts* o) {
  if (!s || !o) return fail(CHEM_EINVAL, "null argument");
  *o = s->opts;
  return CHEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch shape
// ---------------------------------------------------------------------------
namespace {

struct Shape {
  chemk::Variant v;
  int wpb = 4;
  int cpw = 1;
  size_t lds = 0;
};

int pick_shape(const chem_solver* s, const chem_opts& o, Shape& sh) {
  if (s->wide) {
    if (o.cells_per_wave > 1)
      return fail(CHEM_EUNSUPPORTED, "state size " + std::to_string(s->n) + " runs one cell per workgroup");
    sh.v = s->variants[0];
    sh.cpw = 1;
    sh.wpb = chemk::kWideThreads / 64;
    sh.lds = s->wide_lds;
    return CHEM_OK;
  }
  // variant by requested cells per wave, else the first compiled one
  int want_g = o.cells_per_wave > 0 ? 64 / o.cells_per_wave : 0;
  sh.v = s->variants[0];
  if (want_g) {
    bool found = false;
    for (int i = 0; i < s->nvariants; ++i)
      if (s->variants[i].g == want_g) {
        sh.v = s->variants[i];
        found = true;
      }
    if (!found)
      return fail(CHEM_EUNSUPPORTED, "cells_per_wave " + std::to_string(o.cells_per_wave) +
                                         " not compiled for state size " + std::to_string(s->n));
  }
  sh.cpw = 64 / sh.v.g;
  const size_t cell_bytes = sizeof(double) * chemk::cell_doubles(sh.v.nn, s->nr, s->ns);
  const size_t blob = s->margs.lds_bytes;
  int wpb = o.waves_per_block > 0 ? o.waves_per_block : 4;
  while (wpb > 1 && blob + wpb * sh.cpw * cell_bytes > kMaxLds) --wpb;
  sh.lds = blob + wpb * sh.cpw * cell_bytes;
  if (sh.lds > kMaxLds)
    return fail(CHEM_EUNSUPPORTED, "mechanism and one cell's work area exceed the 160 KB LDS");
  sh.wpb = wpb;
  return CHEM_OK;
}

int check_integrate_args(const chem_solver* s, int64_t n, double dt, const double* in, double* out) {
  if (!s) return fail(CHEM_EINVAL, "null solver");
  if (n < 0) return fail(CHEM_EINVAL, "n_cells < 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "dt must be positive and finite");
  if (n > 0 && (!in || !out)) return fail(CHEM_EINVAL, "null phi_in or phi_out");
  if ((s->d_njac || s->d_nfev) && n > s->counters_cap)
    return fail(CHEM_EINVAL, "more cells than the evaluation counters set by chem_eval_counters hold");
  if (n > 0 && in != out) {
    const char* a = reinterpret_cast<const char*>(in);
    const char* b = reinterpret_cast<const char*>(out);
    const size_t bytes = static_cast<size_t>(n) * (s->ns + 2) * sizeof(double);
    if (a < b + bytes && b < a + bytes) return fail(CHEM_EINVAL, "phi_in and phi_out overlap partially");
  }
  return CHEM_OK;
}

// Workspace slots of the workgroup kernel: one per resident workgroup, at
// most hbm_budget_bytes (default: half the free device memory) in total.
// Allocates; never called under stream capture.
int ensure_ws(chem_solver* s) {
  if (!s->wide) return CHEM_OK;
  const int64_t budget_opt = s->opts.hbm_budget_bytes;
  if (s->d_ws && s->wide_budget == budget_opt) return CHEM_OK;
  int bpc = chemk::integrate_wide_blocks_per_cu(true, s->wide_lds);
  if (bpc < 1) bpc = 1;
  const long long cap = static_cast<long long>(s->cus) * bpc;
  int64_t budget = budget_opt;
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    budget = static_cast<int64_t>(fr / 2) + (s->d_ws ? static_cast<int64_t>(s->wide_slots) * s->ws_stride * 8 : 0);
  }
  const long long slot_bytes = s->ws_stride * static_cast<long long>(sizeof(double));
  long long slots = budget / slot_bytes;
  if (slots > cap) slots = cap;
  if (slots < 1) return fail(CHEM_ENOMEM, "hbm_budget_bytes is below one cell's workspace");
  hipFree(s->d_ws);
  s->d_ws = nullptr;
  s->wide_slots = 0;
  drop_graph(s);
  HIP_TRY(hipMalloc(&s->d_ws, static_cast<size_t>(slots) * slot_bytes), "hipMalloc workspace");
  s->wide_slots = static_cast<int>(slots);
  s->wide_budget = budget_opt;
  return CHEM_OK;
}

// Queue head and workgroup workspace taken from the static scratch instead
// of the solver's own buffers (the allocation-free entry point).
struct StaticRes {
  unsigned long long* head = nullptr;
  double* ws = nullptr;
  long long slots = 0;
};

// One chemistry step with the solver's options on stream st. With res, the
// queue head and workspace come from there, and no log record or timing
// event is made.
int launch_step(chem_solver* s, const chem_opts& o, int64_t n, double dt, const double* in, double* out,
                double* h_io, int32_t* n_acc, int32_t* n_rej, int8_t* status, int accumulate,
                const int* perm, hipStream_t st, bool head_set = false, const StaticRes* res = nullptr) {
  Shape sh;
  if (int rc = pick_shape(s, o, sh)) return rc;
  chemk::IntegrateArgs a{};
  a.m = s->margs;
  a.o.rtol = o.rtol;
  a.o.atol = o.atol;
  a.o.max_steps = o.max_steps;
  a.o.scheme = o.scheme;
  a.o.jac_fd = o.jacobian == CHEM_JAC_FD;
  a.o.no_bath = o.state == CHEM_STATE_NO_BATH;
  if (a.o.no_bath && s->ns < 2) return fail(CHEM_EINVAL, "dropping the bath gas needs at least two species");
  a.dt = dt;
  a.n = n;
  a.phi_in = in;
  a.phi_out = out;
  a.h_io = h_io;
  a.n_acc = n_acc;
  a.n_rej = n_rej;
  a.status = reinterpret_cast<signed char*>(status);
  a.n_jac = s->d_njac;
  a.n_fev = s->d_nfev;
  a.accumulate = accumulate;
  a.cell_doubles = chemk::cell_doubles(sh.v.nn, s->nr, s->ns);
  a.wpb = sh.wpb;
  a.perm = perm;
  unsigned long long* const head = res ? res->head : s->d_head;
  a.head = head;
  a.chunk = o.queue_chunk > 0 ? o.queue_chunk : 1;
  if (!res) {
    a.log.cap = s->log_cap;
    a.log.feats = s->log_feats;
    a.log.target = s->log_target;
    a.log.head = s->d_head + 1;
  }
  const bool persistent = o.schedule != CHEM_PLAIN;
  const long long per_block = static_cast<long long>(sh.wpb) * sh.cpw;
  long long grid;
  if (s->wide) {
    double* const ws = res ? res->ws : s->d_ws;
    if (!ws) return fail(CHEM_ESTATE, "workspace not allocated");
    a.ws = ws;
    a.ws_stride = s->ws_stride;
    a.ld = s->ld;
    grid = res ? res->slots : s->wide_slots;
    if (o.blocks > 0 && o.blocks < grid) grid = o.blocks;
    if (grid > n) grid = n;
    if (persistent && !head_set) HIP_TRY(chemk::launch_fill_u64(head, 0ull, st), "queue reset");
  } else if (!persistent) {
    grid = (n + per_block - 1) / per_block;
  } else {
    int bpc = chemk::integrate_blocks_per_cu(sh.v, true, sh.wpb, sh.lds);
    if (bpc < 1) bpc = 1;
    grid = o.blocks > 0 ? o.blocks : static_cast<long long>(s->cus) * bpc;
    const long long need = (n + per_block - 1) / per_block;
    if (grid > need) grid = need;
    if (!head_set) HIP_TRY(chemk::launch_fill_u64(head, 0ull, st), "queue reset");
  }
  if (grid < 1) return CHEM_OK;
  if (grid > 0x7fffffffLL) return fail(CHEM_EINVAL, "too many cells for one launch");
  bool timed = false;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (s->timing && !res) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
    if (cs == hipStreamCaptureStatusNone) {
      HIP_TRY(hipEventCreate(&ev.first), "hipEventCreate");
      HIP_TRY(hipEventCreate(&ev.second), "hipEventCreate");
      s->tev.push_back(ev);
      HIP_TRY(hipEventRecord(ev.first, st), "hipEventRecord");
      timed = true;
    }
  }
  if (s->wide) {
    HIP_TRY(chemk::launch_integrate_wide(persistent, static_cast<int>(grid), a, sh.lds, st), "integrate launch");
  } else {
    HIP_TRY(chemk::launch_integrate(sh.v, persistent, static_cast<int>(grid), a, sh.lds, st), "integrate launch");
  }
  if (timed) HIP_TRY(hipEventRecord(ev.second, st), "hipEventRecord");
  return CHEM_OK;
}

int binned_perm(chem_solver* s, int64_t n, double dt, const double* in, hipStream_t st, const int** perm) {
  *perm = nullptr;
  int used = 0;
  const float* over = (s->cost_override && s->cost_override_n == n) ? s->cost_override : nullptr;
  int rc = chem_model::plan(s->model, s->margs, n, dt, in, over, st, perm, &used);
  if (rc) return fail(rc, chem_model::last_error());
  s->last_binning_used = used;
  return CHEM_OK;
}

// binning buffers for n cells (allocation happens here, never under capture)
int reserve_binning(chem_solver* s, int64_t n) {
  if (s->opts.schedule != CHEM_PERSISTENT_BINNED) return CHEM_OK;
  int rc = chem_model::reserve(s->model, n);
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

}  // namespace

extern "C" {

int chem_integrate(chem_solver* s, int64_t n, double dt, const double* in, double* out, double* h_io,
                   int32_t* n_acc, int32_t* n_rej, int8_t* status, void* stream) {
  if (int rc = check_integrate_args(s, n, dt, in, out)) return rc;
  if (n == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = ensure_ws(s)) return rc;
  const int* perm = nullptr;
  if (s->opts.schedule == CHEM_PERSISTENT_BINNED) {
    if (int rc = reserve_binning(s, n)) return rc;
    if (int rc = binned_perm(s, n, dt, in, st, &perm)) return rc;
  }
  return launch_step(s, s->opts, n, dt, in, out, h_io, n_acc, n_rej, status, 0, perm, st);
}

// chem_integrate on the persistent queue in index order, with the queue head
// and the workgroup kernel's workspace in the static scratch: nothing is
// allocated or freed here, and no allocating runtime call is made.
int chem_integrate_noalloc(chem_solver* s, int64_t n, double dt, const double* in, double* out, double* h_io,
                           int32_t* n_acc, int32_t* n_rej, int8_t* status, void* stream) {
  if (int rc = check_integrate_args(s, n, dt, in, out)) return rc;
  if (n == 0) return CHEM_OK;
  if (!s->scratch) return fail(CHEM_ESTATE, "chem_integrate_noalloc: no scratch address for this device");
  DeviceGuard g(s->dev);
  StaticRes res;
  res.head = reinterpret_cast<unsigned long long*>(s->scratch);
  if (s->wide) {
    const size_t slot = static_cast<size_t>(s->ws_stride) * sizeof(double);
    const size_t room = kScratchBytes - kScratchCtl;
    if (slot > room)
      return fail(CHEM_EUNSUPPORTED, "chem_integrate_noalloc: one cell's workspace (" + std::to_string(slot) +
                                         " bytes) exceeds the static scratch (" + std::to_string(room) + " bytes)");
    int bpc = chemk::integrate_wide_blocks_per_cu(true, s->wide_lds);
    if (bpc < 1) bpc = 1;
    const long long resident = static_cast<long long>(s->cus) * bpc;
    const long long fit = static_cast<long long>(room / slot);
    res.ws = reinterpret_cast<double*>(s->scratch + kScratchCtl);
    res.slots = resident < fit ? resident : fit;
  }
  chem_opts o = s->opts;
  o.schedule = CHEM_PERSISTENT;
  return launch_step(s, o, n, dt, in, out, h_io, n_acc, n_rej, status, 0, nullptr, static_cast<hipStream_t>(stream),
                     false, &res);
}

}  // extern "C"

// The steps enqueued one after the other on st (no graph of the solver's own):
// used when the caller is capturing st already.
static int enqueue_steps(chem_solver* s, int32_t n_steps, int64_t n, double dt, const double* in, double* out,
                         double* h_io, int32_t* n_acc, int32_t* n_rej, int8_t* status, hipStream_t st) {
  for (int32_t step = 0; step < n_steps; ++step) {
    const double* src = step == 0 ? in : ((n_steps - step) % 2 == 0 ? out : s->d_ping);
    double* dst = ((n_steps - 1 - step) % 2 == 0) ? out : s->d_ping;
    const int* perm = nullptr;
    if (s->opts.schedule == CHEM_PERSISTENT_BINNED)
      if (int rc = binned_perm(s, n, dt, src, st, &perm)) return rc;
    if (int rc = launch_step(s, s->opts, n, dt, src, dst, h_io, n_acc, n_rej, status, step > 0, perm, st)) return rc;
  }
  return CHEM_OK;
}

extern "C" {

int chem_integrate_steps(chem_solver* s, int32_t n_steps, int64_t n, double dt, const double* in, double* out,
                         double* h_io, int32_t* n_acc, int32_t* n_rej, int8_t* status, void* stream) {
  if (int rc = check_integrate_args(s, n, dt, in, out)) return rc;
  if (n_steps < 1) return fail(CHEM_EINVAL, "n_steps must be >= 1");
  if (n == 0) return CHEM_OK;
  if (in == out && n_steps > 1) return fail(CHEM_EINVAL, "chem_integrate_steps: phi_in must not alias phi_out");
  DeviceGuard g(s->dev);
  if (int rc = reserve_binning(s, n)) return rc;
  if (int rc = ensure_ws(s)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t w = static_cast<size_t>(s->ns) + 2;
  if (s->ping_cells < static_cast<size_t>(n) && n_steps > 1) {
    drop_graph(s);
    hipFree(s->d_ping);
    s->d_ping = nullptr;
    s->ping_cells = 0;
    HIP_TRY(hipMalloc(&s->d_ping, static_cast<size_t>(n) * w * sizeof(double)), "hipMalloc ping buffer");
    s->ping_cells = static_cast<size_t>(n);
  }
  // the caller is capturing already: enqueue the steps into its graph, and
  // leave the solver's own graph alone (no graph calls during the capture)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return enqueue_steps(s, n_steps, n, dt, in, out, h_io, n_acc, n_rej, status, st);
  auto& k = s->gkey;
  const bool same = s->graph && k.n_steps == n_steps && k.n_cells == n && k.dt == dt && k.in == in && k.out == out &&
                    k.h == h_io && k.a == n_acc && k.r == n_rej && k.s == status && k.st == st &&
                    std::memcmp(&k.o, &s->opts, sizeof(chem_opts)) == 0;
  if (!same) {
    drop_graph(s);
    // capture on the solver's own stream (the caller's may be the null
    // stream, which cannot be captured); the graph is launched on st
    hipStream_t cst = s->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    {
      int rc = CHEM_OK;
      // step k reads src and writes dst; the last step writes out
      for (int32_t step = 0; step < n_steps && rc == CHEM_OK; ++step) {
        const double* src = step == 0 ? in : ((n_steps - step) % 2 == 0 ? out : s->d_ping);
        double* dst = ((n_steps - 1 - step) % 2 == 0) ? out : s->d_ping;
        const int* perm = nullptr;
        if (s->opts.schedule == CHEM_PERSISTENT_BINNED) rc = binned_perm(s, n, dt, src, cst, &perm);
        if (rc == CHEM_OK)
          rc = launch_step(s, s->opts, n, dt, src, dst, h_io, n_acc, n_rej, status, step > 0, perm, cst);
      }
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(cst, &graph);
      if (rc != CHEM_OK) {
        if (graph) hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
      }
      s->graph = exec;
      s->graph_src = graph;
      k.n_steps = n_steps;
      k.n_cells = n;
      k.dt = dt;
      k.in = in;
      k.out = out;
      k.h = h_io;
      k.a = n_acc;
      k.r = n_rej;
      k.s = status;
      k.st = st;
      k.o = s->opts;
    }
  }
  HIP_TRY(hipGraphLaunch(s->graph, st), "hipGraphLaunch");
  return CHEM_OK;
}

int chem_eval_rhs_jac(chem_solver* s, int64_t n, const double* phi, double* f, double* J, void* stream) {
  if (!s || n < 0 || (n > 0 && (!phi || !f))) return fail(CHEM_EINVAL, "chem_eval_rhs_jac: bad argument");
  if (n == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  chem_opts o = s->opts;
  Shape sh;
  if (int rc = pick_shape(s, o, sh)) return rc;
  chemk::EvalArgs a{};
  a.m = s->margs;
  a.n = n;
  a.phi = phi;
  a.f = f;
  a.J = J;
  a.wpb = sh.wpb;
  if (s->wide) {
    if (int rc = ensure_ws(s)) return rc;
    a.ws = s->d_ws;
    a.ws_stride = s->ws_stride;
    a.ld = s->ld;
    const long long grid = n < s->wide_slots ? n : s->wide_slots;
    HIP_TRY(chemk::launch_eval_wide(static_cast<int>(grid), a, sh.lds, static_cast<hipStream_t>(stream)), "eval launch");
    return CHEM_OK;
  }
  a.cell_doubles = chemk::cell_doubles(sh.v.nn, s->nr, s->ns);
  const long long per_block = static_cast<long long>(sh.wpb) * sh.cpw;
  const long long grid = (n + per_block - 1) / per_block;
  HIP_TRY(chemk::launch_eval(sh.v, static_cast<int>(grid), a, sh.lds, static_cast<hipStream_t>(stream)), "eval launch");
  return CHEM_OK;
}

int chem_lu_batch(chem_solver* s, int64_t batch, double* A, int32_t* piv, int32_t* info, double* b, void* stream) {
  if (!s || batch < 0 || (batch > 0 && (!A || !piv || !info))) return fail(CHEM_EINVAL, "chem_lu_batch: bad argument");
  if (batch == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  Shape sh;
  if (int rc = pick_shape(s, s->opts, sh)) return rc;
  chemk::LuArgs a{};
  a.batch = batch;
  a.n = s->n;
  a.A = A;
  a.piv = piv;
  a.info = info;
  a.b = b;
  a.wpb = 4;
  if (s->wide) {
    if (int rc = ensure_ws(s)) return rc;
    a.ws = s->d_ws;
    a.ws_stride = s->ws_stride;
    a.ld = s->ld;
    const long long grid = batch < s->wide_slots ? batch : s->wide_slots;
    const size_t lds = chemk::wide_cell_bytes(0, 0, s->ld);
    HIP_TRY(chemk::launch_lu_wide(static_cast<int>(grid), a, lds, static_cast<hipStream_t>(stream)), "lu launch");
    return CHEM_OK;
  }
  const long long per_block = 4LL * sh.cpw;
  const long long grid = (batch + per_block - 1) / per_block;
  HIP_TRY(chemk::launch_lu(sh.v, static_cast<int>(grid), a, static_cast<hipStream_t>(stream)), "lu launch");
  return CHEM_OK;
}

// ---- learned cost model --------------------------------------------------

int chem_log_enable(chem_solver* s, int64_t cap) {
  if (!s || cap < 0) return fail(CHEM_EINVAL, "chem_log_enable: bad argument");
  DeviceGuard g(s->dev);
  hipFree(s->log_feats);
  hipFree(s->log_target);
  s->log_feats = nullptr;
  s->log_target = nullptr;
  s->log_cap = 0;
  drop_graph(s);
  if (cap == 0) return CHEM_OK;
  HIP_TRY(hipMalloc(&s->log_feats, static_cast<size_t>(cap) * 4 * sizeof(float)), "hipMalloc log");
  HIP_TRY(hipMalloc(&s->log_target, static_cast<size_t>(cap) * sizeof(float)), "hipMalloc log");
  HIP_TRY(hipMemset(s->d_head + 1, 0, sizeof(unsigned long long)), "hipMemset");
  s->log_cap = cap;
  return CHEM_OK;
}

int chem_log_fetch(chem_solver* s, float* feats, float* target, int64_t* n_out, void* stream) {
  if (!s || !n_out) return fail(CHEM_EINVAL, "chem_log_fetch: bad argument");
  DeviceGuard g(s->dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  unsigned long long cnt = 0;
  HIP_TRY(hipMemcpy(&cnt, s->d_head + 1, sizeof(cnt), hipMemcpyDeviceToHost), "hipMemcpy");
  const int64_t nv = s->log_cap == 0 ? 0 : static_cast<int64_t>(std::min<unsigned long long>(cnt, s->log_cap));
  if (nv > 0 && (!feats || !target)) return fail(CHEM_EINVAL, "chem_log_fetch: null output buffer");
  if (nv > 0) {
    HIP_TRY(hipMemcpy(feats, s->log_feats, nv * 4 * sizeof(float), hipMemcpyDeviceToDevice), "hipMemcpy");
    HIP_TRY(hipMemcpy(target, s->log_target, nv * sizeof(float), hipMemcpyDeviceToDevice), "hipMemcpy");
  }
  *n_out = nv;
  return CHEM_OK;
}

int chem_features(chem_solver* s, int64_t n, double dt, const double* phi, float* feats, void* stream) {
  if (!s || n < 0 || (n > 0 && (!phi || !feats)) || !(dt > 0)) return fail(CHEM_EINVAL, "chem_features: bad argument");
  if (n == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  int rc = chem_model::features(s->margs, n, dt, phi, feats, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

void chem_train_opts_default(chem_train_opts* t) {
  if (!t) return;
  t->epochs = 10;
  t->batch = 4096;
  t->lr = 1e-3f;
  t->beta1 = 0.9f;
  t->beta2 = 0.999f;
  t->eps = 1e-8f;
  t->seed = 1234;
}

int chem_model_train(chem_solver* s, int64_t n, const float* feats, const float* target, const chem_train_opts* t,
                     void* stream) {
  if (!s || n < 1 || !feats || !target) return fail(CHEM_EINVAL, "chem_model_train: bad argument");
  chem_train_opts def;
  chem_train_opts_default(&def);
  if (!t) t = &def;
  if (t->epochs < 1 || t->batch < 1 || !(t->lr > 0)) return fail(CHEM_EINVAL, "chem_model_train: bad options");
  DeviceGuard g(s->dev);
  drop_graph(s);
  int rc = chem_model::train(s->model, n, feats, target, *t, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_model_predict(chem_solver* s, int64_t n, const float* feats, float* pred, void* stream) {
  if (!s || n < 0 || (n > 0 && (!feats || !pred))) return fail(CHEM_EINVAL, "chem_model_predict: bad argument");
  if (n == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  int rc = chem_model::predict(s->model, n, feats, pred, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_set_cost_override(chem_solver* s, int64_t n, const float* cost) {
  if (!s || (cost && n < 1)) return fail(CHEM_EINVAL, "chem_set_cost_override: bad argument");
  s->cost_override = cost;
  s->cost_override_n = cost ? n : 0;
  drop_graph(s);
  return CHEM_OK;
}

int chem_model_save(const chem_solver* s, const char* path) {
  if (!s || !path) return fail(CHEM_EINVAL, "chem_model_save: bad argument");
  DeviceGuard g(s->dev);
  int rc = chem_model::save(s->model, path);
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_model_load(chem_solver* s, const char* path) {
  if (!s || !path) return fail(CHEM_EINVAL, "chem_model_load: bad argument");
  DeviceGuard g(s->dev);
  drop_graph(s);
  int rc = chem_model::load(s->model, path);
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_last_binning_used(const chem_solver* s, int32_t* used) {
  if (!s || !used) return fail(CHEM_EINVAL, "chem_last_binning_used: bad argument");
  *used = 0;
  if (!s->last_binning_used) return CHEM_OK;
  DeviceGuard g(s->dev);
  int fin = 0;
  if (int rc = chem_model::last_plan_finite(s->model, &fin)) return fail(rc, chem_model::last_error());
  *used = fin ? 1 : 0;
  return CHEM_OK;
}

int chem_model_get(const chem_solver* s, float* params, float* norm, float* edges) {
  if (!s) return fail(CHEM_EINVAL, "chem_model_get: bad argument");
  DeviceGuard g(s->dev);
  int rc = chem_model::get_params(s->model, params, norm, edges);
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_model_set(chem_solver* s, const float* params, const float* norm, const float* edges) {
  if (!s || !params) return fail(CHEM_EINVAL, "chem_model_set: bad argument");
  DeviceGuard g(s->dev);
  drop_graph(s);
  int rc = chem_model::set_params(s->model, params, norm, edges);
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_model_grad(chem_solver* s, int64_t n, const float* feats, const float* target, float* grad, float* loss,
                    void* stream) {
  if (!s || n < 1 || !feats || !target || !grad || !loss) return fail(CHEM_EINVAL, "chem_model_grad: bad argument");
  DeviceGuard g(s->dev);
  int rc = chem_model::grad(s->model, n, feats, target, grad, loss, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_bin_edges(chem_solver* s, int64_t n, const float* cost, float* edges, void* stream) {
  if (!s || n < 1 || !cost || !edges) return fail(CHEM_EINVAL, "chem_bin_edges: bad argument");
  DeviceGuard g(s->dev);
  int rc = chem_model::octiles(s->model, n, cost, edges, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

int chem_bin_order(chem_solver* s, int64_t n, const float* cost, const float* edges, int32_t* perm, void* stream) {
  if (!s || n < 1 || !cost || !perm) return fail(CHEM_EINVAL, "chem_bin_order: bad argument");
  DeviceGuard g(s->dev);
  int rc = chem_model::order(s->model, n, cost, edges, perm, static_cast<hipStream_t>(stream));
  return rc ? fail(rc, chem_model::last_error()) : CHEM_OK;
}

// ---- autotuning ------------------------------------------------------------

}  // extern "C"

// Time every launch shape (compiled cells-per-wave variants, 1/2/4 waves per
// block, queue chunks 1..64 for the persistent schedules) on n_sample cells
// and return the fastest in best.
static int tune(chem_solver* s, int64_t n_sample, const double* phi, double dt, hipStream_t st, chem_opts& best,
                float& best_ms) {
  if (int rc = ensure_ws(s)) return rc;
  const size_t w = static_cast<size_t>(s->ns) + 2;
  double* out = nullptr;
  double* h = nullptr;
  HIP_TRY(hipMalloc(&out, n_sample * w * sizeof(double)), "hipMalloc");
  if (hipMalloc(&h, n_sample * sizeof(double)) != hipSuccess) {
    hipFree(out);
    return fail(CHEM_ENOMEM, "hipMalloc");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    hipFree(out);
    hipFree(h);
    return fail(CHEM_EHIP, "autotune: hipEventCreate failed");
  }
  best = s->opts;
  best_ms = 1e30f;
  int rc = CHEM_OK;
  const int chunks[] = {1, 2, 4, 8, 16, 32, 64};
  const int nchunks = s->opts.schedule == CHEM_PLAIN ? 1 : 7;
  for (int vi = 0; vi < s->nvariants && rc == CHEM_OK; ++vi) {
    for (int wpb = 1; wpb <= 4 && rc == CHEM_OK; wpb *= 2) {
      for (int ci = 0; ci < nchunks && rc == CHEM_OK; ++ci) {
        chem_opts o = s->opts;
        o.cells_per_wave = 64 / s->variants[vi].g;
        o.waves_per_block = wpb;
        o.queue_chunk = chunks[ci];
        Shape sh;
        if (pick_shape(s, o, sh) != CHEM_OK || sh.wpb != wpb) continue;
        float ms = 0;
        for (int rep = 0; rep < 2; ++rep) {   // first repetition warms up
          if (hipMemsetAsync(h, 0, n_sample * sizeof(double), st) != hipSuccess ||
              hipEventRecord(e0, st) != hipSuccess) {
            rc = fail(CHEM_EHIP, "autotune: stream operation failed");
            break;
          }
          rc = launch_step(s, o, n_sample, dt, phi, out, h, nullptr, nullptr, nullptr, 0, nullptr, st);
          if (rc) break;
          if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(CHEM_EHIP, "autotune: launch failed");
            break;
          }
        }
        if (rc == CHEM_OK && ms < best_ms) {
          best_ms = ms;
          best = o;
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(out);
  hipFree(h);
  best.blocks = s->opts.blocks;
  return rc;
}

static std::string tune_key(const chem_solver* s, int64_t n_sample, double dt) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "mech=%016llx n=%d schedule=%d sample=%lld dt=%.17g arch=%s cus=%d", s->mech_fp,
                s->n, s->opts.schedule, static_cast<long long>(n_sample), dt, s->arch.c_str(), s->cus);
  return buf;
}

// Integer value of "name": in a JSON line, or false.
static bool json_int(const std::string& line, const char* name, long long& v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  const char* c = line.c_str() + p + pat.size();
  char* e = nullptr;
  v = std::strtoll(c, &e, 10);
  return e != c;
}

extern "C" {

int chem_autotune(chem_solver* s, int64_t n_sample, const double* phi, double dt, void* stream) {
  if (!s || n_sample < 1 || !phi || !(dt > 0)) return fail(CHEM_EINVAL, "chem_autotune: bad argument");
  DeviceGuard g(s->dev);
  chem_opts best;
  float ms = 0;
  if (int rc = tune(s, n_sample, phi, dt, static_cast<hipStream_t>(stream), best, ms)) return rc;
  s->opts = best;
  drop_graph(s);
  return CHEM_OK;
}

int chem_autotune_cached(chem_solver* s, const char* cache_path, int64_t n_sample, const double* phi, double dt,
                         void* stream, int32_t* from_cache) {
  if (!s || !cache_path || !from_cache || n_sample < 1 || !phi || !(dt > 0))
    return fail(CHEM_EINVAL, "chem_autotune_cached: bad argument");
  *from_cache = 0;
  DeviceGuard g(s->dev);
  const std::string key = tune_key(s, n_sample, dt);
  const std::string kfield = "\"key\": \"" + key + "\"";
  if (FILE* f = std::fopen(cache_path, "r")) {
    std::string line;
    char buf[1024];
    bool hit = false;
    chem_opts o = s->opts;
    while (std::fgets(buf, sizeof(buf), f)) {
      line = buf;
      if (line.find(kfield) == std::string::npos) continue;
      long long cpw, wpb, chunk;
      if (!json_int(line, "cells_per_wave", cpw) || !json_int(line, "waves_per_block", wpb) ||
          !json_int(line, "queue_chunk", chunk))
        continue;
      chem_opts t = s->opts;
      t.cells_per_wave = static_cast<int32_t>(cpw);
      t.waves_per_block = static_cast<int32_t>(wpb);
      t.queue_chunk = static_cast<int32_t>(chunk);
      Shape sh;
      if (chunk < 1 || chunk > 1 << 20 || pick_shape(s, t, sh) != CHEM_OK) continue;
      o = t;   // the last valid line for the key wins
      hit = true;
    }
    std::fclose(f);
    if (hit) {
      s->opts = o;
      drop_graph(s);
      *from_cache = 1;
      return CHEM_OK;
    }
  }
  chem_opts best;
  float ms = 0;
  if (int rc = tune(s, n_sample, phi, dt, static_cast<hipStream_t>(stream), best, ms)) return rc;
  s->opts = best;
  drop_graph(s);
  FILE* f = std::fopen(cache_path, "a");
  if (!f) return fail(CHEM_EINVAL, std::string("chem_autotune_cached: cannot append to ") + cache_path);
  std::fprintf(f, "{%s, \"cells_per_wave\": %d, \"waves_per_block\": %d, \"queue_chunk\": %d, \"ms\": %.4f}\n",
               kfield.c_str(), best.cells_per_wave, best.waves_per_block, best.queue_chunk, ms);
  const bool ok = std::fclose(f) == 0;
  if (!ok) return fail(CHEM_EINVAL, std::string("chem_autotune_cached: write to ") + cache_path + " failed");
  return CHEM_OK;
}

int chem_workspace_info(chem_solver* s, int32_t* slots, int64_t* bytes_per_slot) {
  if (!s || !slots || !bytes_per_slot) return fail(CHEM_EINVAL, "chem_workspace_info: bad argument");
  *slots = 0;
  *bytes_per_slot = 0;
  if (!s->wide) return CHEM_OK;
  DeviceGuard g(s->dev);
  if (int rc = ensure_ws(s)) return rc;
  *slots = s->wide_slots;
  *bytes_per_slot = s->ws_stride * static_cast<int64_t>(sizeof(double));
  return CHEM_OK;
}

// ---- kernel timing -----------------------------------------------------------

int chem_eval_counters(chem_solver* s, int32_t* n_jac, int32_t* n_fev, int64_t capacity) {
  if (!s || capacity < 0 || ((n_jac || n_fev) && capacity == 0))
    return fail(CHEM_EINVAL, "chem_eval_counters: bad argument");
  DeviceGuard g(s->dev);
  s->d_njac = n_jac;
  s->d_nfev = n_fev;
  s->counters_cap = (n_jac || n_fev) ? capacity : 0;
  drop_graph(s);   // a cached chain of steps holds the previous pointers
  return CHEM_OK;
}

int chem_kernel_timing(chem_solver* s, int32_t enable) {
  if (!s) return fail(CHEM_EINVAL, "chem_kernel_timing: bad argument");
  DeviceGuard g(s->dev);
  if (!s->tev.empty()) HIP_TRY(hipEventSynchronize(s->tev.back().second), "hipEventSynchronize");
  clear_timing(s);
  s->timing = enable != 0;
  return CHEM_OK;
}

int chem_kernel_times(chem_solver* s, float* ms, int32_t cap, int32_t* n_out) {
  if (!s || !n_out || cap < 0 || (cap > 0 && !ms)) return fail(CHEM_EINVAL, "chem_kernel_times: bad argument");
  DeviceGuard g(s->dev);
  int32_t k = 0;
  for (auto& e : s->tev) {
    HIP_TRY(hipEventSynchronize(e.second), "hipEventSynchronize");
    if (k < cap) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, e.first, e.second), "hipEventElapsedTime");
      ms[k++] = t;
    }
  }
  clear_timing(s);
  *n_out = k;
  return CHEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// zonal reference mapping
// ---------------------------------------------------------------------------
extern "C" {

int chem_mech_elements(const chem_mech* m, int32_t* ne, int32_t* counts) {
  if (!m || !ne) return fail(CHEM_EINVAL, "chem_mech_elements: null argument");
  *ne = m->host.ne;
  if (counts)
    for (size_t i = 0; i < m->host.elem.size(); ++i) counts[i] = m->host.elem[i];
  return CHEM_OK;
}

int chem_zone_config(chem_solver* s, const double* coupling, const double* y_fuel, const double* y_ox,
                     double z_max, double t_tol) {
  if (!s || !coupling || !y_fuel || !y_ox) return fail(CHEM_EINVAL, "chem_zone_config: null argument");
  if (!std::isfinite(z_max) || !std::isfinite(t_tol) || t_tol < 0)
    return fail(CHEM_EINVAL, "chem_zone_config: z_max and t_tol must be finite, t_tol >= 0");
  if (s->dz > 0 && z_max / s->dz >= chemz::kMaxBands)
    return fail(CHEM_EINVAL, "chem_zone_config: z_max / dz gives more than 64 bands");
  for (int e = 0; e < s->ne; ++e)
    if (!std::isfinite(coupling[e])) return fail(CHEM_EINVAL, "chem_zone_config: non-finite coupling");
  for (int i = 0; i < s->ns; ++i)
    if (!std::isfinite(y_fuel[i]) || !std::isfinite(y_ox[i]))
      return fail(CHEM_EINVAL, "chem_zone_config: non-finite stream composition");
  DeviceGuard g(s->dev);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  s->zone_ready = false;       // until the new definition is in place
  const int ns = s->ns, ne = s->ne;
  if (!s->d_zone || !s->d_zctl) {    // both, or (after a failed allocation) again
    hipFree(s->d_zone);
    hipFree(s->d_zctl);
    s->d_zone = nullptr;
    s->d_zctl = nullptr;
    HIP_TRY(hipMalloc(&s->d_zone, sizeof(double) * (ns + 2 + chemz::kMaxBands * (ns + 2))), "hipMalloc zone");
    HIP_TRY(hipMalloc(&s->d_zctl, (chemz::kMaxBands + 1) * sizeof(unsigned long long)), "hipMalloc zone");
  }
  // inputs staged in one temporary buffer: coupling, y_fuel, y_ox, counts
  std::vector<double> in(ne + 2 * ns);
  std::copy(coupling, coupling + ne, in.begin());
  std::copy(y_fuel, y_fuel + ns, in.begin() + ne);
  std::copy(y_ox, y_ox + ns, in.begin() + ne + ns);
  void* d_in = nullptr;
  const size_t in_bytes = sizeof(double) * in.size() + sizeof(int) * s->elem.size();
  HIP_TRY(hipMalloc(&d_in, in_bytes), "hipMalloc zone inputs");
  double* din = static_cast<double*>(d_in);
  int* dcounts = reinterpret_cast<int*>(din + in.size());
  hipError_t e = hipMemcpy(din, in.data(), sizeof(double) * in.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(dcounts, s->elem.data(), sizeof(int) * s->elem.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = chemz::launch_zone_setup(ns, ne, din, dcounts, s->d_W, din + ne, din + ne + ns, s->d_zone, s->d_zone + ns,
                                 nullptr);
  double streams[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(streams, s->d_zone + ns, sizeof(streams), hipMemcpyDeviceToHost);
  hipFree(d_in);
  if (e != hipSuccess) return hip_fail(e, "zone setup");
  if (!(streams[0] != streams[1]) || !std::isfinite(streams[0]) || !std::isfinite(streams[1])) {
    return fail(CHEM_EINVAL, "chem_zone_config: fuel and oxidiser streams have the same coupling value");
  }
  s->z_max = z_max;
  s->t_tol = t_tol;
  s->zone_ready = true;
  return CHEM_OK;
}

int chem_zone_bands(chem_solver* s, double dz) {
  if (!s) return fail(CHEM_EINVAL, "null solver");
  // a rejected band width leaves no zone definition behind (a zone left
  // live with its earlier width would map across the whole of Z <= z_max)
  if (!std::isfinite(dz) || dz < 0) {
    s->zone_ready = false;
    return fail(CHEM_EINVAL, "chem_zone_bands: dz must be finite and >= 0");
  }
  if (dz > 0 && s->zone_ready && s->z_max / dz >= chemz::kMaxBands) {
    s->zone_ready = false;
    return fail(CHEM_EINVAL, "chem_zone_bands: z_max / dz gives more than 64 bands");
  }
  s->dz = dz;
  return CHEM_OK;
}

int chem_mixture_fraction(chem_solver* s, int64_t n, const double* phi, double* z, void* stream) {
  if (!s) return fail(CHEM_EINVAL, "null solver");
  if (n < 0 || (n > 0 && (!phi || !z))) return fail(CHEM_EINVAL, "chem_mixture_fraction: bad argument");
  if (!s->zone_ready) return fail(CHEM_ESTATE, "chem_mixture_fraction: call chem_zone_config first");
  DeviceGuard g(s->dev);
  HIP_TRY(chemz::launch_mixture_fraction(n, s->ns, phi, s->d_zone, s->d_zone + s->ns, z,
                                         static_cast<hipStream_t>(stream)),
          "mixture fraction launch");
  return CHEM_OK;
}

int chem_integrate_zonal(chem_solver* s, int64_t n, double dt, const double* in, double* out, double* h_io,
                         int32_t* n_acc, int32_t* n_rej, int8_t* status, int8_t* mapped, void* stream) {
  if (int rc = check_integrate_args(s, n, dt, in, out)) return rc;
  if (!s->zone_ready) return fail(CHEM_ESTATE, "chem_integrate_zonal: call chem_zone_config first");
  if (n > 0x7fffffffLL) return fail(CHEM_EINVAL, "chem_integrate_zonal: more than 2^31 - 1 cells");
  if (n == 0) return CHEM_OK;
  DeviceGuard g(s->dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = ensure_ws(s)) return rc;
  if (s->zone_cap < n) {
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    hipFree(s->d_zflag);
    hipFree(s->d_zorder);
    s->d_zflag = nullptr;
    s->d_zorder = nullptr;
    s->zone_cap = 0;
    HIP_TRY(hipMalloc(&s->d_zflag, static_cast<size_t>(n)), "hipMalloc zone flags");
    HIP_TRY(hipMalloc(&s->d_zorder, sizeof(int) * static_cast<size_t>(n)), "hipMalloc zone order");
    s->zone_cap = n;
  }
  chemz::ZoneArgs z{};
  z.n = n;
  z.ns = s->ns;
  z.phi_in = in;
  z.phi_out = out;
  z.coef = s->d_zone;
  z.streams = s->d_zone + s->ns;
  z.stash = s->d_zone + s->ns + 2;
  z.z_max = s->z_max;
  z.t_tol = s->t_tol;
  z.dz = s->dz;
  z.nb = 1;
  if (s->dz > 0 && s->z_max >= 0) {
    const double nb = std::floor(s->z_max / s->dz) + 1.0;
    if (!(nb <= chemz::kMaxBands)) return fail(CHEM_EINVAL, "chem_integrate_zonal: more than 64 Z bands");
    z.nb = static_cast<int>(nb);
  }
  z.flag = mapped ? reinterpret_cast<signed char*>(mapped) : s->d_zflag;
  z.order = s->d_zorder;
  z.ctl = s->d_zctl;
  z.head = s->d_head;
  z.n_acc = n_acc;
  z.n_rej = n_rej;
  z.status = reinterpret_cast<signed char*>(status);
  z.n_jac = s->d_njac;
  z.n_fev = s->d_nfev;
  HIP_TRY(chemz::launch_zone_classify(z, st), "zone classify launch");
  HIP_TRY(chemz::launch_zone_select(z, st), "zone select launch");
  chem_opts o = s->opts;
  o.schedule = CHEM_PERSISTENT;
  if (int rc = launch_step(s, o, n, dt, in, out, h_io, n_acc, n_rej, status, 0, s->d_zorder, st, true)) return rc;
  HIP_TRY(chemz::launch_zone_apply(z, st), "zone apply launch");
  return CHEM_OK;
}

}  // extern "C"
