// Problem contexts shared by the C ABI entry points and the solve server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ibim.h"
#include "device_mem.h"
#include "ibim_internal.h"
#include "krylov.h"
#include "operator.h"
#include "symmetric.h"
#include "treecode.h"

namespace ibim {

// Sets the thread-local message returned by ibim_last_error and returns code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* where);

#define HIP_TRY(expr, where)                             \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return ibim::hip_fail(_e, where); \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return device_alloc((void**)p, n * sizeof(T));
}

template <class T>
hipError_t upload(T** p, const T* src, size_t n, hipStream_t s) {
  hipError_t e = dalloc(p, n);
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  return hipMemcpyAsync(*p, src, n * sizeof(T), hipMemcpyHostToDevice, s);
}

template <class T>
void dfree(T*& p) {
  if (p) device_free((void*)p);
  p = nullptr;
}

// Restores the caller's current device on scope exit.
struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace ibim

using ibim::DeviceProblem;
using ibim::DeviceScope;
using ibim::HostPlan;
using ibim::Krylov;
using ibim::PairPlan;
using ibim::SymPlan;
using ibim::dfree;

struct ibim_ctx {
  HostPlan plan;
  ibim_options opt{};
  double eps_in = 1, eps_out = 1, kappa = 0;
  std::vector<double> zq, q;  // charges (host)
  // device state
  DeviceProblem P;
  PairPlan pair;
  double* partial = nullptr;  // nsplit * 2M (one-directional kernels)
  // symmetric float64 pair sum (used when sym.enabled)
  SymPlan sym;
  int32_t* d_sym_items = nullptr;  // (rb, cb) pairs
  int n_sym_items = 0;
  uint32_t* d_careful = nullptr;   // T x T bits
  double* sym_scratch = nullptr;   // sym.scratch_doubles
  double pair_flops = 0.0;         // flops of one pair-sum launch (see ibim_pair_work)
  // treecode summation (used when opt.summation == IBIM_SUM_TREE)
  ibim::TreePlan tplan;
  ibim::TreeDevice tree;
  double* om11 = nullptr;
  double* om21 = nullptr;
  double* d_zq = nullptr;
  double* d_q = nullptr;
  double* d_psi = nullptr;
  Krylov kr;
  bool kr_ready = false;
  // pair-kernel timing (events bracket every pair launch while enabled)
  bool timing = false;
  std::vector<hipEvent_t> tev;  // 2 per launch
  size_t tcount = 0;            // launches recorded
  int applies = 0;              // operator applications of the current solve

  bool on_device() const { return opt.device >= 0 && device_ready; }
  bool device_ready = false;
  int nx = 0, ny = 0, nz = 0;  // grid dimensions (kept for the near list)
  // mixed direct form: an upper bound on the near-list entries (tube nodes in
  // the cube each row's near search scans), from ctx_create_host
  int64_t near_bound = 0;
  double node_span = 0;        // diagonal of the nodes' bounding box (largest pair distance)
  size_t device_bytes = 0;     // device memory held by the context
  size_t setup_peak_bytes = 0; // largest device memory during its setup (temporaries included)

  void release() {
    if (!on_device()) return;
    DeviceScope ds(opt.device);
    dfree(P.px); dfree(P.py); dfree(P.pz); dfree(P.nx); dfree(P.ny); dfree(P.nz); dfree(P.w);
    dfree(P.px32); dfree(P.py32); dfree(P.pz32); dfree(P.nx32); dfree(P.ny32); dfree(P.nz32);
    dfree(P.crow); dfree(P.ccol); dfree(P.blocks); dfree(P.nrow); dfree(P.ncol);
    dfree(P.xrow); dfree(P.xtile);
    dfree(d_sym_items); dfree(d_careful); dfree(sym_scratch);
    tree.release();
    dfree(partial); dfree(om11); dfree(om21); dfree(d_zq); dfree(d_q); dfree(d_psi);
    dfree(kr.V); dfree(kr.H); dfree(kr.cs); dfree(kr.sn); dfree(kr.g); dfree(kr.y);
    dfree(kr.hcol); dfree(kr.hcol2); dfree(kr.scal); dfree(kr.status); dfree(kr.partial);
    dfree(kr.tmp); dfree(kr.tmp2); dfree(kr.bsc);
    if (kr.host_status) (void)hipHostFree(kr.host_status);
    kr.host_status = nullptr;
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
    tev.clear();
  }
};


namespace ibim {

// Validates options (IBIM_EINVAL with a message for the first bad field).
int check_options(const ibim_options& o);
// Host part of ibim_setup: validates, builds the geometry and correction sets.
int ctx_create_host(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
                    double eps_tube, double eps_in, double eps_out, double kappa,
                    const double* charge_xyz, const double* charge_q, int n_charges,
                    const ibim_options& o, ibim_ctx** out);
// Device part: uploads, correction weights, mixed-precision data, scratch.
int ctx_setup_device(ibim_ctx* c, hipStream_t s);
// Device bytes a context will hold once set up with a Krylov basis, plus the
// peak of its setup temporaries: an upper bound (the near list of the mixed
// form is bounded by the tube nodes its search scans).
size_t ctx_footprint_estimate(const ibim_ctx* c);

int apply_impl(ibim_ctx* c, const double* u, double* out, hipStream_t s);
int ensure_krylov(ibim_ctx* c);
int rhs_impl(ibim_ctx* c, double* g, hipStream_t s);
// psi_rxn at every charge into c->d_psi (asynchronous).
int energy_launch(ibim_ctx* c, const double* x, hipStream_t s);
double energy_sum(const ibim_ctx* c, const double* psi_host);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_copy(const double* a, double* b, int64_t n, hipStream_t s);
// y = Lambda^-1 x (x == y allowed): the row scaling of IBIM_PRECOND_DIAG.
hipError_t launch_row_scaling(const ibim_ctx* c, const double* x, double* y, hipStream_t s);

}  // namespace ibim
