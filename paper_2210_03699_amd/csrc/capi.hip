// C ABI of the CTR-IBIM solver: problem contexts, device uploads, the GMRES
// driver (Section 2.5), the right-hand side (eq. PB-lambda-g) and the
// polarisation energy (eq. pol-energy).
#include <hip/hip_runtime.h>

#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ibim.h"
#include "context.h"
#include "ibim_internal.h"
#include "krylov.h"
#include "operator.h"
#include "weights.h"

using namespace ibim;

namespace ibim {

thread_local std::string g_last_error = "no error";

namespace {
thread_local DeviceArena* t_arena = nullptr;
std::mutex g_arena_mu;
std::map<uintptr_t, size_t> g_arenas;  // live blocks: base -> size
}  // namespace

hipError_t arena_create(DeviceArena* a, size_t bytes) {
  *a = DeviceArena{};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 1);
  if (e != hipSuccess) return e;
  a->base = (char*)p;
  a->size = bytes;
  std::lock_guard<std::mutex> lk(g_arena_mu);
  g_arenas[(uintptr_t)p] = bytes;
  return hipSuccess;
}

void arena_release(DeviceArena* a) {
  if (!a->base) return;
  {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    g_arenas.erase((uintptr_t)a->base);
  }
  (void)hipFree(a->base);
  *a = DeviceArena{};
}

hipError_t device_alloc(void** p, size_t bytes) {
  DeviceArena* a = t_arena;
  if (a && a->base) {
    const size_t off = (a->top + 255) & ~(size_t)255;
    if (off <= a->size && bytes <= a->size - off) {
      *p = a->base + off;
      a->top = off + bytes;
      return hipSuccess;
    }
    a->outside += bytes;
  }
  return hipMalloc(p, bytes);
}

void device_free(void* p) {
  {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    auto it = g_arenas.upper_bound((uintptr_t)p);
    if (it != g_arenas.begin()) {
      --it;
      if ((uintptr_t)p - it->first < it->second) return;  // freed with its block
    }
  }
  (void)hipFree(p);
}

ArenaScope::ArenaScope(DeviceArena* a) : prev(t_arena) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = prev; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? IBIM_ENOMEM : IBIM_EHIP,
              std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace ibim

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Partial sums of ibim_apply_noalloc.  Each GPU the library runs on holds its
// own copy for the life of the process; host code reaches it only through the
// device address from hipGetSymbolAddress (taken once per device, with that
// device current), never through the array's name.
constexpr size_t kNoAllocScratchDoubles = (size_t)IBIM_NOALLOC_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (the current device).
int noalloc_scratch(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return fail(IBIM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return IBIM_OK;
}

__global__ void rhs_kernel(const double* px, const double* py, const double* pz, const double* nx,
                           const double* ny, const double* nz, int32_t M, const double* zq,
                           const double* q, int nc, double inv_eps_in, double* g) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double x = px[k], y = py[k], z = pz[k];
  const double n0 = nx[k], n1 = ny[k], n2 = nz[k];
  double g1 = 0.0, g2 = 0.0;
  for (int j = 0; j < nc; ++j) {
    const double rx = x - zq[3 * j], ry = y - zq[3 * j + 1], rz = z - zq[3 * j + 2];
    const double R2 = rx * rx + ry * ry + rz * rz;
    const double iR = 1.0 / sqrt(R2);
    const double qj = q[j] * inv_eps_in;
    g1 += qj * iR;
    g2 -= qj * (rx * n0 + ry * n1 + rz * n2) * iR * iR * iR;
  }
  g[k] = g1 / (4.0 * kPiD);
  g[M + k] = g2 / (4.0 * kPiD);
}

// psi[j] = h^3 sum_m f_j(m) w_m for charge j (one workgroup per charge,
// fixed-order tree reduction).
__global__ __launch_bounds__(256) void psi_rxn_kernel(const double* px, const double* py,
                                                      const double* pz, const double* nx,
                                                      const double* ny, const double* nz,
                                                      const double* w, int32_t M, const double* x,
                                                      const double* zq, double ratio,
                                                      double kappa, double h3, double* psi) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const double zx = zq[3 * j], zy = zq[3 * j + 1], zz = zq[3 * j + 2];
  double acc = 0.0;
  for (int32_t m = threadIdx.x; m < M; m += blockDim.x) {
    const double rx = zx - px[m], ry = zy - py[m], rz = zz - pz[m];
    const double R2 = rx * rx + ry * ry + rz * rz;
    const double R = sqrt(R2);
    const double iR = 1.0 / R;
    const double kr = kappa * R;
    const double e = exp(-kr);
    const double rn = rx * nx[m] + ry * ny[m] + rz * nz[m];
    const double dG0 = rn * iR * iR * iR;          // 4 pi dG0/dn_y
    const double dGk = dG0 * (e + e * kr);          // 4 pi dGk/dn_y
    const double G0mGk = -expm1(-kr) * iR;          // 4 pi (G0 - Gk)
    acc += ((ratio * dGk - dG0) * x[m] + G0mGk * x[M + m]) * w[m];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) psi[j] = h3 * red[0] / (4.0 * kPiD);
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) x[r] = v;
}

// y = D^-1 x with D = Lambda: the psi rows divided by lambda1, the psi_n rows by lambda2.
__global__ void unscale_kernel(const double* x, double* y, int64_t M, double lam1, double lam2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) y[i] = x[i] / lam1;
  else if (i < 2 * M) y[i] = x[i] / lam2;
}

__global__ void copy_kernel(const double* a, double* b, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = a[r];
}

int check_ctx(const ibim_ctx* c) {
  if (!c) return fail(IBIM_EINVAL, "null context");
  return IBIM_OK;
}

int check_dev(const ibim_ctx* c) {
  int r = check_ctx(c);
  if (r) return r;
  if (!c->on_device()) return fail(IBIM_ENODEV, "host-only context (options.device < 0)");
  return IBIM_OK;
}

int fetch(ibim_ctx* c, const double* d, int n, hipStream_t s, double* out) {
  HIP_TRY(hipMemcpyAsync(c->kr.host_status, d, n * sizeof(double), hipMemcpyDeviceToHost, s),
          "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  for (int i = 0; i < n; ++i) out[i] = c->kr.host_status[i];
  return IBIM_OK;
}

}  // namespace

namespace ibim {

// out = A u with the pair sum's partial sums in sym_scratch (symmetric
// kernels, when sym_on) or in partial (one-directional kernels).
static int apply_core(ibim_ctx* c, const double* u, double* out, hipStream_t s, bool sym_on,
                      double* sym_scratch, double* partial, bool timed) {
  const int prec = c->opt.precision;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    if (2 * c->tcount + 2 > c->tev.size()) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "hipEventCreate");
        c->tev.push_back(e);
      }
    }
    e0 = c->tev[2 * c->tcount];
    e1 = c->tev[2 * c->tcount + 1];
    HIP_TRY(hipEventRecord(e0, s), "hipEventRecord");
  }
  const bool tree = c->opt.summation == IBIM_SUM_TREE;
  if (tree) {
    HIP_TRY(launch_tree_sum(c->tree, c->P, u, s), "treecode launch");
  } else if (sym_on) {
    const SymArgs sa = make_sym_args(c->P, c->sym, c->d_sym_items, c->d_careful, u, sym_scratch);
    if (prec == IBIM_MIXED)
      HIP_TRY(launch_pair_sym_mixed(sa, c->n_sym_items, s), "pair kernel launch");
    else
      HIP_TRY(launch_pair_sym(sa, c->n_sym_items, s), "pair kernel launch");
  } else if (prec == IBIM_MIXED)
    HIP_TRY(launch_pair_mixed(c->P, c->pair, u, partial, s), "pair kernel launch");
  else
    HIP_TRY(launch_pair(c->P, c->pair, prec, u, partial, s), "pair kernel launch");
  if (timed) {
    HIP_TRY(hipEventRecord(e1, s), "hipEventRecord");
    ++c->tcount;
  }
  if (tree)
    HIP_TRY(launch_tree_finish(c->tree, c->P, u, out, s), "finish kernel launch");
  else if (sym_on && prec == IBIM_MIXED)
    HIP_TRY(launch_finish_sym_mixed(c->P, c->sym, c->d_careful, u, sym_scratch, out, s),
            "finish kernel launch");
  else if (sym_on)
    HIP_TRY(launch_finish_sym(c->P, c->sym, u, sym_scratch, out, s), "finish kernel launch");
  else if (prec == IBIM_MIXED)
    HIP_TRY(launch_finish_mixed(c->P, c->pair, u, partial, out, s), "finish kernel launch");
  else
    HIP_TRY(launch_finish(c->P, c->pair, prec, u, partial, out, s), "finish kernel launch");
  return IBIM_OK;
}

int apply_impl(ibim_ctx* c, const double* u, double* out, hipStream_t s) {
  if (int r = apply_core(c, u, out, s, c->sym.enabled, c->sym_scratch, c->partial, c->timing))
    return r;
  ++c->applies;
  return IBIM_OK;
}

int ensure_krylov(ibim_ctx* c) {
  if (c->kr_ready) return IBIM_OK;
  Krylov& k = c->kr;
  k.m = c->opt.restart;
  k.n = 2 * (int64_t)c->P.M;
  const size_t m = (size_t)k.m;
  HIP_TRY(dalloc(&k.V, (m + 1) * (size_t)k.n), "GMRES basis allocation");
  HIP_TRY(dalloc(&k.H, (m + 1) * m), "alloc");
  HIP_TRY(dalloc(&k.cs, m), "alloc");
  HIP_TRY(dalloc(&k.sn, m), "alloc");
  HIP_TRY(dalloc(&k.g, m + 1), "alloc");
  HIP_TRY(dalloc(&k.y, m), "alloc");
  HIP_TRY(dalloc(&k.hcol, m + 1), "alloc");
  HIP_TRY(dalloc(&k.hcol2, m + 1), "alloc");
  HIP_TRY(dalloc(&k.scal, 4), "alloc");
  HIP_TRY(dalloc(&k.status, 2), "alloc");
  HIP_TRY(dalloc(&k.partial, (m + 1) * 1024), "alloc");
  HIP_TRY(dalloc(&k.tmp, (size_t)k.n), "alloc");
  HIP_TRY(dalloc(&k.tmp2, (size_t)k.n), "alloc");
  HIP_TRY(dalloc(&k.bsc, (size_t)k.n), "alloc");
  HIP_TRY(hipHostMalloc((void**)&k.host_status, 4 * sizeof(double), hipHostMallocDefault),
          "pinned allocation");
  c->device_bytes += ((m + 4) * (size_t)k.n + (m + 1) * (m + 1030) + 8 * m) * sizeof(double);
  c->kr_ready = true;
  return IBIM_OK;
}

// Partial-sum bytes the symmetric pair kernel may use under these options.
static size_t sym_scratch_cap(const ibim_options& o) {
  return o.pair_scratch_max > 0 ? (size_t)o.pair_scratch_max : kSymScratchMax;
}

// The symmetric plan of a context: none for the treecode, none past the
// scratch cap, and none in float64 when kappa times the largest pair
// distance exceeds what the kernel's table exponential accepts.
static SymPlan sym_plan_for(const ibim_ctx* c) {
  const ibim_options& o = c->opt;
  SymPlan sp = make_sym_plan(c->plan.M, o.summation == IBIM_SUM_TREE ? 0 : sym_scratch_cap(o));
  if (o.precision == IBIM_FP64 && c->kappa * c->node_span > kSymMaxKappaR) sp.enabled = false;
  return sp;
}

// Checks the options shared by ibim_setup and the solve server.
int check_options(const ibim_options& o) {
  if (o.precision != IBIM_FP64 && o.precision != IBIM_MIXED)
    return fail(IBIM_EINVAL, "unknown precision mode");
  if (!(o.r_near >= 0.0) || !std::isfinite(o.r_near))
    return fail(IBIM_EINVAL, "r_near must be >= 0");
  if (o.restart < 1 || o.restart > 1000 || o.max_iter < 1)
    return fail(IBIM_EINVAL, "restart must be in [1, 1000] and max_iter >= 1");
  if (o.hybrid != IBIM_CTR2 && o.hybrid != IBIM_HYB && o.hybrid != IBIM_KREG)
    return fail(IBIM_EINVAL, "unknown hybrid mode");
  if (o.precond != IBIM_PRECOND_NONE && o.precond != IBIM_PRECOND_DIAG)
    return fail(IBIM_EINVAL, "unknown preconditioning mode");
  if (o.summation != IBIM_SUM_DIRECT && o.summation != IBIM_SUM_TREE)
    return fail(IBIM_EINVAL, "unknown summation mode");
  if (o.tree_min_nodes < 0) return fail(IBIM_EINVAL, "tree_min_nodes must be >= 0");
  if (o.pair_scratch_max < 0) return fail(IBIM_EINVAL, "pair_scratch_max must be >= 0");
  if (o.summation == IBIM_SUM_TREE) {
    if (o.tree_order < 2 || o.tree_order > ibim::kTreeMaxOrder)
      return fail(IBIM_EINVAL, "tree_order must be in [2, 12]");
    if (!(o.tree_theta > 0.0 && o.tree_theta <= 1.0))
      return fail(IBIM_EINVAL, "tree_theta must be in (0, 1]");
  }
  return IBIM_OK;
}

// Near radius of the mixed form (default 2h: the smallest measured radius
// whose surface-potential error stays near the larger radii's, with G_pol
// about 100 times inside the 1e-6 bar at every radius from h to 4h).
static double near_radius(const ibim_options& o, double h) {
  return o.r_near > 0.0 ? o.r_near : 2.0 * h;
}

// Upper bound on the mixed near list: for every row, the tube nodes in the
// cube of half-width ceil((r_near + 2 eps)/h) cells around its grid node
// (clipped to the grid) that build_near_list scans, counted with 3-D prefix
// sums of the tube indicator.
static int64_t near_list_bound(const HostPlan& pl, int nx, int ny, int nz, double r_near) {
  const int64_t sx = (int64_t)(ny + 1) * (nz + 1), sy = nz + 1;
  std::vector<int32_t> S((size_t)(nx + 1) * sx, 0);
  for (int64_t m = 0; m < pl.M; ++m) {
    const int64_t q = pl.grid_index[m];
    const int i = (int)(q / ((int64_t)ny * nz)), j = (int)((q / nz) % ny), k = (int)(q % nz);
    S[(i + 1) * sx + (j + 1) * sy + (k + 1)] = 1;
  }
  for (int i = 1; i <= nx; ++i)
    for (int j = 1; j <= ny; ++j)
      for (int k = 1; k <= nz; ++k) {
        const int64_t c = i * sx + j * sy + k;
        S[c] += S[c - sx] + S[c - sy] + S[c - 1] - S[c - sx - sy] - S[c - sx - 1] - S[c - sy - 1] +
                S[c - sx - sy - 1];
      }
  const double reach = std::ceil((r_near + 2.0 * pl.eps) / pl.h);
  const double diag = std::ceil(std::sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz));
  const int W = (int)std::min(reach, diag);
  int64_t total = 0;
  for (int64_t m = 0; m < pl.M; ++m) {
    const int64_t q = pl.grid_index[m];
    const int i = (int)(q / ((int64_t)ny * nz)), j = (int)((q / nz) % ny), k = (int)(q % nz);
    const int64_t i0 = std::max(i - W, 0), i1 = std::min(i + W, nx - 1) + 1;
    const int64_t j0 = std::max(j - W, 0), j1 = std::min(j + W, ny - 1) + 1;
    const int64_t k0 = std::max(k - W, 0), k1 = std::min(k + W, nz - 1) + 1;
    auto at = [&](int64_t a, int64_t b, int64_t c) { return (int64_t)S[a * sx + b * sy + c]; };
    total += at(i1, j1, k1) - at(i0, j1, k1) - at(i1, j0, k1) - at(i1, j1, k0) + at(i0, j0, k1) +
             at(i0, j1, k0) + at(i1, j0, k0) - at(i0, j0, k0);
  }
  return total;
}

// Host part of ibim_setup: the geometry, the correction sets and, for the
// treecode, its plan; IBIM_SUM_TREE is resolved here for the problem's size.
int ctx_create_host(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
                    double eps_tube, double eps_in, double eps_out, double kappa,
                    const double* charge_xyz, const double* charge_q, int n_charges,
                    const ibim_options& o, ibim_ctx** out) {
  *out = nullptr;
  if (!(eps_in > 0) || !(eps_out > 0) || !(kappa >= 0) || !std::isfinite(kappa))
    return fail(IBIM_EINVAL, "eps_in, eps_out must be > 0 and kappa >= 0");
  if (n_charges < 0 || (n_charges > 0 && (!charge_xyz || !charge_q)))
    return fail(IBIM_EINVAL, "bad charge arrays");
  if (int r = check_options(o)) return r;
  ibim_ctx* c = new (std::nothrow) ibim_ctx();
  if (!c) return fail(IBIM_ENOMEM, "host allocation failed");
  c->opt = o;
  c->eps_in = eps_in;
  c->eps_out = eps_out;
  c->kappa = kappa;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  if (n_charges > 0) {
    c->zq.assign(charge_xyz, charge_xyz + 3 * (size_t)n_charges);
    c->q.assign(charge_q, charge_q + (size_t)n_charges);
  }
  std::string err;
  int r = build_host_plan(sdf, nx, ny, nz, origin, h, eps_tube, o.hybrid, &c->plan, &err);
  if (!r && o.summation == IBIM_SUM_TREE) {
    // the treecode serves problems of at least tree_min_nodes nodes
    if ((int64_t)c->plan.M < o.tree_min_nodes) c->opt.summation = IBIM_SUM_DIRECT;
  }
  if (!r && c->opt.summation == IBIM_SUM_TREE) {
    TreeParams prm;
    prm.order = o.tree_order;
    prm.theta = o.tree_theta;
    prm.proxy_cost = o.precision == IBIM_MIXED ? kTreeProxyCost32 : kTreeProxyCost64;
    prm.two_way = true;
    const HostPlan& pl = c->plan;
    r = build_tree_plan(prm, pl.M, pl.px.data(), pl.py.data(), pl.pz.data(), pl.crow.data(),
                        pl.ccol.data(), h, &c->tplan, &err);
  }
  if (r) {
    delete c;
    return fail(r, err);
  }
  if (c->opt.precision == IBIM_MIXED && c->opt.summation == IBIM_SUM_DIRECT)
    c->near_bound = near_list_bound(c->plan, nx, ny, nz, near_radius(c->opt, h));
  {
    const HostPlan& pl = c->plan;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int32_t m = 0; m < pl.M; ++m) {
      const double p[3] = {pl.px[m], pl.py[m], pl.pz[m]};
      for (int d = 0; d < 3; ++d) {
        lo[d] = m == 0 ? p[d] : std::min(lo[d], p[d]);
        hi[d] = m == 0 ? p[d] : std::max(hi[d], p[d]);
      }
    }
    c->node_span = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                             (hi[2] - lo[2]) * (hi[2] - lo[2]));
  }
  *out = c;
  return IBIM_OK;
}

size_t ctx_footprint_estimate(const ibim_ctx* c) {
  const HostPlan& pl = c->plan;
  const size_t M = (size_t)pl.M, nnz = (size_t)pl.crow[pl.M];
  const PairPlan pp = make_pair_plan((int32_t)M, c->opt.precision);
  const size_t ntile = (size_t)pp.ntile;
  const size_t m = (size_t)c->opt.restart, n = 2 * M, nc = c->q.size();
  // geometry and weights, corrections (ccol, om11, om21, 2x2 blocks), exclusion
  // tiles (at most one entry per corrected pair), split partial sums
  size_t b = 7 * M * 8 + (M + 1) * 4 + nnz * (4 + 6 * 8);
  b += (ntile + 1) * 4 + std::min(nnz, ntile * ntile) * 4;
  b += (4 * nc + (nc > 0 ? nc : 1)) * 8;
  const SymPlan sp = sym_plan_for(c);
  if (c->opt.summation == IBIM_SUM_TREE)
    b += tree_device_bytes(c->tplan);
  else if (sp.enabled)
    b += sp.scratch_doubles * 8 + ((size_t)sp.nRB * sp.nCB * 2 + 2) * 4 +
         (((size_t)sp.T * sp.T + 31) / 32) * 4;
  else
    b += (size_t)pp.nsplit * n * 8;
  // Krylov basis and GMRES scratch (as allocated by ensure_krylov)
  b += ((m + 4) * n + (m + 1) * (m + 1030) + 8 * m) * 8;
  // temporaries of the device setup (freed before it returns, but held at
  // its peak): the weights' per-entry inputs, then (mixed direct form) the
  // grid-to-node map, node grid indices and the near-list row counts
  size_t tmp = nnz * (4 + 1 + 3 * 8) + 8 * M * 8;
  if (c->opt.precision == IBIM_MIXED && c->opt.summation == IBIM_SUM_DIRECT) {
    const size_t grid = (size_t)c->nx * c->ny * c->nz;
    tmp = std::max(tmp, grid * 4 + M * 8 + M * 4);
    // float32 geometry, near-list rows and (bounded) entries
    b += 6 * M * 4 + (M + 1) * 8 + (size_t)c->near_bound * 4;
  }
  return b + tmp;
}

int ctx_setup_device(ibim_ctx* c, hipStream_t s) {
  const ibim_options& o = c->opt;
  DeviceScope ds(o.device);
  if (!ds.ok) return fail(IBIM_EHIP, "hipSetDevice failed");
  const HostPlan& pl = c->plan;
  const int32_t M = (int32_t)pl.M;
  const int64_t nnz = pl.crow[M];
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const double h = pl.h, eps_tube = pl.eps;
  const int n_charges = (int)c->q.size();
  DeviceProblem& P = c->P;
  P.M = M;
  P.nnz = nnz;
  P.eps_in = c->eps_in;
  P.eps_out = c->eps_out;
  P.kappa = c->kappa;
  P.h = h;
  P.lam1 = 0.5 * (1.0 + c->eps_out / c->eps_in);
  P.lam2 = 0.5 * (1.0 + c->eps_in / c->eps_out);
  c->device_ready = true;  // release() frees whatever is allocated below
  size_t bytes = 0;
  std::vector<int32_t> crow32(M + 1);
  for (int32_t k = 0; k <= M; ++k) crow32[k] = (int32_t)pl.crow[k];

  auto bad = [&](hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? IBIM_ENOMEM : IBIM_EHIP,
                std::string(what) + ": " + hipGetErrorString(e));
  };
#define UP(dst, vec)                                                   \
  do {                                                                 \
    hipError_t _e = upload(&(dst), (vec).data(), (vec).size(), s);     \
    if (_e != hipSuccess) return bad(_e, "upload");                    \
    bytes += (vec).size() * sizeof((vec)[0]);                          \
  } while (0)
  UP(P.px, pl.px); UP(P.py, pl.py); UP(P.pz, pl.pz);
  UP(P.nx, pl.nx); UP(P.ny, pl.ny); UP(P.nz, pl.nz);
  UP(P.w, pl.w);
  UP(P.crow, crow32);
  UP(P.ccol, pl.ccol);
  std::vector<int32_t> xrow, xtile;
  exclusion_tiles(M, pl.crow.data(), pl.ccol.data(), &xrow, &xtile);
  UP(P.xrow, xrow);
  UP(P.xtile, xtile);
  if (n_charges > 0) {
    UP(c->d_zq, c->zq);
    UP(c->d_q, c->q);
  }
  // correction weights, built on the device from temporary per-entry data
  int32_t* d_rowid = nullptr;
  int8_t* d_axis = nullptr;
  double *d_alpha = nullptr, *d_beta = nullptr, *d_eta = nullptr, *d_tau = nullptr;
  double *d_k1 = nullptr, *d_k2 = nullptr;
  // the weights' per-entry inputs and outputs are alive beside everything
  // uploaded so far
  size_t peak = bytes + (size_t)nnz * (4 + 1 + 3 * 8) + 8 * (size_t)M * 8 + 6 * (size_t)nnz * 8;
  hipError_t e = upload(&d_rowid, pl.crowid.data(), pl.crowid.size(), s);
  if (e == hipSuccess) e = upload(&d_axis, pl.caxis.data(), pl.caxis.size(), s);
  if (e == hipSuccess) e = upload(&d_alpha, pl.calpha.data(), pl.calpha.size(), s);
  if (e == hipSuccess) e = upload(&d_beta, pl.cbeta.data(), pl.cbeta.size(), s);
  if (e == hipSuccess) e = upload(&d_eta, pl.ceta.data(), pl.ceta.size(), s);
  if (e == hipSuccess) e = upload(&d_tau, pl.tau.data(), pl.tau.size(), s);
  if (e == hipSuccess) e = upload(&d_k1, pl.kap1.data(), pl.kap1.size(), s);
  if (e == hipSuccess) e = upload(&d_k2, pl.kap2.data(), pl.kap2.size(), s);
  if (e == hipSuccess) e = dalloc(&c->om11, (size_t)nnz);
  if (e == hipSuccess) e = dalloc(&c->om21, (size_t)nnz);
  if (e == hipSuccess) e = dalloc(&P.blocks, 4 * (size_t)nnz);
  bytes += 6 * (size_t)nnz * 8;
  if (e == hipSuccess) {
    WeightArgs wa;
    wa.nnz = nnz;
    wa.rowid = d_rowid;
    wa.col = P.ccol;
    wa.axis = d_axis;
    wa.alpha = d_alpha;
    wa.beta = d_beta;
    wa.eta = d_eta;
    wa.tau = d_tau;
    wa.kap1 = d_k1;
    wa.kap2 = d_k2;
    wa.w = P.w;
    wa.eps_in = c->eps_in;
    wa.eps_out = c->eps_out;
    wa.kappa = c->kappa;
    wa.h = h;
    wa.c12 = kreg_constant(c->kappa, pl.ktau);
    wa.om11 = c->om11;
    wa.om21 = c->om21;
    wa.blocks = P.blocks;
    e = launch_weights(wa, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(d_rowid); dfree(d_axis); dfree(d_alpha); dfree(d_beta); dfree(d_eta); dfree(d_tau);
  dfree(d_k1); dfree(d_k2);
  if (e != hipSuccess) return bad(e, "correction weights");
  if (o.precision == IBIM_MIXED && o.summation == IBIM_SUM_DIRECT) {
    // float32 geometry relative to the centroid, and the near list (direct sum)
    double cen[3] = {0, 0, 0};
    for (int32_t m = 0; m < M; ++m) {
      cen[0] += pl.px[m];
      cen[1] += pl.py[m];
      cen[2] += pl.pz[m];
    }
    for (int a = 0; a < 3; ++a) P.centre[a] = cen[a] / M;
    std::vector<float> f(M);
    auto up32 = [&](float** dst, const std::vector<double>& v, double shift) {
      for (int32_t m = 0; m < M; ++m) f[m] = (float)(v[m] - shift);
      hipError_t e2 = upload(dst, f.data(), f.size(), s);
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);  // f is reused
      return e2;
    };
    e = up32(&P.px32, pl.px, P.centre[0]);
    if (e == hipSuccess) e = up32(&P.py32, pl.py, P.centre[1]);
    if (e == hipSuccess) e = up32(&P.pz32, pl.pz, P.centre[2]);
    if (e == hipSuccess) e = up32(&P.nx32, pl.nx, 0.0);
    if (e == hipSuccess) e = up32(&P.ny32, pl.ny, 0.0);
    if (e == hipSuccess) e = up32(&P.nz32, pl.nz, 0.0);
    bytes += 6 * (size_t)M * 4;
    int32_t* d_node_of = nullptr;
    int64_t* d_gidx = nullptr;
    if (e == hipSuccess) {
      std::vector<int32_t> node_of((size_t)nx * ny * nz, -1);
      for (int32_t m = 0; m < M; ++m) node_of[pl.grid_index[m]] = m;
      e = upload(&d_node_of, node_of.data(), node_of.size(), s);
      if (e == hipSuccess) e = upload(&d_gidx, pl.grid_index.data(), pl.grid_index.size(), s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    const double r_near = near_radius(o, h);
    if (e == hipSuccess)
      e = build_near_list(P, d_node_of, d_gidx, nx, ny, nz, r_near, eps_tube, s);
    dfree(d_node_of);
    dfree(d_gidx);
    if (e != hipSuccess) return bad(e, "mixed-precision setup");
    // grid-to-node map and node indices beside the near list (or its counts)
    peak = std::max(peak, bytes + (size_t)nx * ny * nz * 4 + (size_t)M * 8 +
                              std::max((size_t)M * 4, ((size_t)M + 1) * 8 + (size_t)P.nnear * 4));
    bytes += ((size_t)M + 1) * 8 + (size_t)P.nnear * 4;
  }
  c->pair = make_pair_plan(M, o.precision);
  c->sym = sym_plan_for(c);
  if (o.summation == IBIM_SUM_TREE) {
    // the plan was built with the geometry (ctx_create_host)
    e = tree_upload(c->tplan, P, pl.px.data(), pl.py.data(), pl.pz.data(), pl.nx.data(),
                    pl.ny.data(), pl.nz.data(), pl.w.data(), &c->tree, s);
    if (e != hipSuccess) return bad(e, "treecode setup");
    c->tree.mixed = o.precision == IBIM_MIXED;
    c->tree.rnear = near_radius(o, h);
    bytes += c->tree.bytes;
    const double n4 = std::pow((double)o.tree_order, 4.0);
    c->pair_flops = 60.0 * c->tplan.near_evals + 36.0 * c->tplan.far_evals +
                    15.0 * c->tplan.proxy_evals + 12.0 * n4 * c->tplan.m2m_links;
  }
  if (c->sym.enabled) {
    // the quadratic scratch comes first: if the device cannot hold it, the
    // one-directional kernel (linear scratch) takes over
    if (dalloc(&c->sym_scratch, c->sym.scratch_doubles) != hipSuccess) {
      (void)hipGetLastError();
      c->sym.enabled = false;
    }
  }
  if (c->sym.enabled) {
    std::vector<uint32_t> bits;
    sym_careful_bits(c->sym.T, xrow, xtile, &bits);
    std::vector<int32_t> items;
    sym_items(c->sym, bits, M % kPairTile != 0, &items);
    c->n_sym_items = (int)(items.size() / 2);
    // flops: 68 per shared evaluation (66 in Debye units), 60 per one-way
    // pair (diagonal, careful, ragged)
    const bool unit = o.precision == IBIM_MIXED ? sym_debye_units_f32(c->kappa, P.h)
                                                : sym_debye_units(c->kappa);
    const double shared = unit ? 66.0 : 68.0;
    const int T = c->sym.T;
    auto nodes = [&](int X) { return (double)std::min(kPairTile, M - X * kPairTile); };
    double fl = 0.0;
    for (int I = 0; I < T; ++I) {
      fl += 60.0 * nodes(I) * nodes(I);
      for (int J = I + 1; J < T; ++J) {
        const size_t bI = (size_t)I * T + J;
        const bool slow = ((bits[bI >> 5] >> (bI & 31)) & 1u) || (J == T - 1 && M % kPairTile);
        fl += (slow ? 120.0 : shared) * nodes(I) * nodes(J);
      }
    }
    c->pair_flops = fl;
    UP(c->d_sym_items, items);
    UP(c->d_careful, bits);
    e = hipStreamSynchronize(s);  // items, bits are host temporaries
    bytes += c->sym.scratch_doubles * 8;
  } else if (o.summation != IBIM_SUM_TREE) {
    c->pair_flops = 60.0 * (double)M * (double)M;
    e = dalloc(&c->partial, (size_t)c->pair.nsplit * 2 * (size_t)M);
    bytes += (size_t)c->pair.nsplit * 2 * (size_t)M * 8;
  }
  if (e == hipSuccess) e = dalloc(&c->d_psi, (size_t)(n_charges > 0 ? n_charges : 1));
  if (e != hipSuccess) return bad(e, "setup");
  c->device_bytes = bytes;
  c->setup_peak_bytes = std::max(peak, bytes);
  return IBIM_OK;
}

int rhs_impl(ibim_ctx* c, double* g, hipStream_t s) {
  const DeviceProblem& P = c->P;
  const int nc = (int)c->q.size();
  hipLaunchKernelGGL(rhs_kernel, dim3((P.M + 255) / 256), dim3(256), 0, s, P.px, P.py, P.pz, P.nx,
                     P.ny, P.nz, P.M, c->d_zq, c->d_q, nc, 1.0 / c->eps_in, g);
  HIP_TRY(hipGetLastError(), "rhs kernel launch");
  return IBIM_OK;
}

int energy_launch(ibim_ctx* c, const double* x, hipStream_t s) {
  const int nc = (int)c->q.size();
  if (nc == 0) return IBIM_OK;
  const DeviceProblem& P = c->P;
  hipLaunchKernelGGL(psi_rxn_kernel, dim3(nc), dim3(256), 0, s, P.px, P.py, P.pz, P.nx, P.ny,
                     P.nz, P.w, P.M, x, c->d_zq, c->eps_out / c->eps_in, c->kappa,
                     P.h * P.h * P.h, c->d_psi);
  HIP_TRY(hipGetLastError(), "energy kernel launch");
  return IBIM_OK;
}

double energy_sum(const ibim_ctx* c, const double* psi) {
  double G = 0.0;
  for (size_t j = 0; j < c->q.size(); ++j) G += 0.5 * c->q[j] * psi[j];
  return G;
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_row_scaling(const ibim_ctx* c, const double* x, double* y, hipStream_t s) {
  const int64_t M = c->P.M;
  hipLaunchKernelGGL(unscale_kernel, dim3((unsigned)((2 * M + 255) / 256)), dim3(256), 0, s, x, y,
                     M, c->P.lam1, c->P.lam2);
  return hipGetLastError();
}

hipError_t launch_copy(const double* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

}  // namespace ibim

extern "C" {

void ibim_default_options(ibim_options* opt) {
  if (!opt) return;
  opt->precision = IBIM_FP64;
  opt->restart = 60;
  opt->max_iter = 300;
  opt->check_residual = 1;
  opt->device = 0;
  opt->r_near = 0.0;
  opt->hybrid = IBIM_CTR2;
  opt->precond = IBIM_PRECOND_DIAG;
  opt->summation = IBIM_SUM_DIRECT;
  opt->tree_order = 8;
  opt->tree_theta = 0.7;
  opt->tree_min_nodes = 0;
  opt->pair_scratch_max = 0;
}

const char* ibim_last_error(void) { return g_last_error.c_str(); }

int ibim_setup(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
               double eps_tube, double eps_in, double eps_out, double kappa,
               const double* charge_xyz, const double* charge_q, int n_charges,
               const ibim_options* opt, void* stream, ibim_ctx** out) {
  if (!out) return fail(IBIM_EINVAL, "out is NULL");
  *out = nullptr;
  ibim_options o;
  ibim_default_options(&o);
  if (opt) o = *opt;
  ibim_ctx* c = nullptr;
  if (int r = ctx_create_host(sdf, nx, ny, nz, origin, h, eps_tube, eps_in, eps_out, kappa,
                              charge_xyz, charge_q, n_charges, o, &c))
    return r;
  if (o.device < 0) {
    *out = c;
    return IBIM_OK;
  }
  if (int r = ctx_setup_device(c, as_stream(stream))) {
    std::string msg = ibim_last_error();
    ibim_destroy(c);
    return fail(r, msg);
  }
  *out = c;
  return IBIM_OK;
}

void ibim_destroy(ibim_ctx* ctx) {
  if (!ctx) return;
  ctx->release();
  delete ctx;
}

int ibim_context_options(const ibim_ctx* ctx, ibim_options* opt) {
  if (int r = check_ctx(ctx)) return r;
  if (!opt) return fail(IBIM_EINVAL, "opt is NULL");
  *opt = ctx->opt;
  return IBIM_OK;
}

int ibim_num_nodes(const ibim_ctx* ctx, int64_t* M) {
  if (int r = check_ctx(ctx)) return r;
  if (!M) return fail(IBIM_EINVAL, "M is NULL");
  *M = ctx->plan.M;
  return IBIM_OK;
}

int ibim_node_grid_index(const ibim_ctx* ctx, int64_t* idx) {
  if (int r = check_ctx(ctx)) return r;
  if (!idx) return fail(IBIM_EINVAL, "idx is NULL");
  std::memcpy(idx, ctx->plan.grid_index.data(), sizeof(int64_t) * ctx->plan.M);
  return IBIM_OK;
}

int ibim_node_geometry(const ibim_ctx* ctx, double* P, double* n, double* w) {
  if (int r = check_ctx(ctx)) return r;
  const HostPlan& pl = ctx->plan;
  for (int64_t m = 0; m < pl.M; ++m) {
    if (P) {
      P[3 * m] = pl.px[m];
      P[3 * m + 1] = pl.py[m];
      P[3 * m + 2] = pl.pz[m];
    }
    if (n) {
      n[3 * m] = pl.nx[m];
      n[3 * m + 1] = pl.ny[m];
      n[3 * m + 2] = pl.nz[m];
    }
    if (w) w[m] = pl.w[m];
  }
  return IBIM_OK;
}

int ibim_num_corrections(const ibim_ctx* ctx, int64_t* nnz) {
  if (int r = check_ctx(ctx)) return r;
  if (!nnz) return fail(IBIM_EINVAL, "nnz is NULL");
  *nnz = ctx->plan.crow[ctx->plan.M];
  return IBIM_OK;
}

int ibim_node_flags(const ibim_ctx* ctx, uint8_t* bad, int64_t* n_bad) {
  if (int r = check_ctx(ctx)) return r;
  const HostPlan& pl = ctx->plan;
  if (bad) std::memcpy(bad, pl.bad.data(), (size_t)pl.M);
  if (n_bad) *n_bad = pl.n_bad;
  return IBIM_OK;
}

int ibim_corrections(const ibim_ctx* ctx, int64_t* rowptr, int64_t* col, int32_t* axis,
                     double* alpha, double* beta, double* eta) {
  if (int r = check_ctx(ctx)) return r;
  const HostPlan& pl = ctx->plan;
  const int64_t nnz = pl.crow[pl.M];
  if (rowptr) std::memcpy(rowptr, pl.crow.data(), sizeof(int64_t) * (pl.M + 1));
  for (int64_t e = 0; e < nnz; ++e) {
    if (col) col[e] = pl.ccol[e];
    if (axis) axis[e] = pl.caxis[e];
    if (alpha) alpha[e] = pl.calpha[e];
    if (beta) beta[e] = pl.cbeta[e];
    if (eta) eta[e] = pl.ceta[e];
  }
  return IBIM_OK;
}

int ibim_correction_weights(const ibim_ctx* ctx, double* om11, double* om21, void* stream) {
  if (int r = check_dev(ctx)) return r;
  DeviceScope ds(ctx->opt.device);
  hipStream_t s = as_stream(stream);
  const size_t nnz = (size_t)ctx->P.nnz;
  if (om11) HIP_TRY(hipMemcpyAsync(om11, ctx->om11, nnz * 8, hipMemcpyDeviceToHost, s), "copy");
  if (om21) HIP_TRY(hipMemcpyAsync(om21, ctx->om21, nnz * 8, hipMemcpyDeviceToHost, s), "copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return IBIM_OK;
}

int ibim_rhs(ibim_ctx* ctx, double* g, void* stream) {
  if (int r = check_dev(ctx)) return r;
  if (!g) return fail(IBIM_EINVAL, "g is NULL");
  DeviceScope ds(ctx->opt.device);
  hipStream_t s = as_stream(stream);
  const DeviceProblem& P = ctx->P;
  const int nc = (int)ctx->q.size();
  hipLaunchKernelGGL(rhs_kernel, dim3((P.M + 255) / 256), dim3(256), 0, s, P.px, P.py, P.pz, P.nx,
                     P.ny, P.nz, P.M, ctx->d_zq, ctx->d_q, nc, 1.0 / ctx->eps_in, g);
  HIP_TRY(hipGetLastError(), "rhs kernel launch");
  return IBIM_OK;
}

int ibim_apply(ibim_ctx* ctx, const double* u, double* out, void* stream) {
  if (int r = check_dev(ctx)) return r;
  if (!u || !out || u == out) return fail(IBIM_EINVAL, "u and out must be distinct device vectors");
  DeviceScope ds(ctx->opt.device);
  return apply_impl(ctx, u, out, as_stream(stream));
}

int ibim_apply_noalloc(ibim_ctx* ctx, const double* u, double* out, void* stream) {
  if (int r = check_dev(ctx)) return r;
  if (!u || !out || u == out) return fail(IBIM_EINVAL, "u and out must be distinct device vectors");
  if (ctx->opt.summation == IBIM_SUM_TREE)
    return fail(IBIM_EINVAL, "ibim_apply_noalloc: treecode contexts are not supported");
  // partial sums needed by the symmetric kernels (the context's plan) and by
  // the one-directional kernels; the first that fits the static array is used
  const size_t cap = kNoAllocScratchDoubles;
  const bool sym_fits = ctx->sym.enabled && ctx->sym.scratch_doubles <= cap;
  const size_t one_way = (size_t)ctx->pair.nsplit * 2 * (size_t)ctx->P.M;
  if (!sym_fits && one_way > cap)
  {
    const size_t need = ctx->sym.enabled ? std::min(ctx->sym.scratch_doubles, one_way) : one_way;
    return fail(IBIM_EINVAL, "ibim_apply_noalloc: the partial sums need " +
                                 std::to_string(need * 8) + " bytes, more than the " +
                                 std::to_string(IBIM_NOALLOC_SCRATCH_BYTES) +
                                 "-byte static scratch");
  }
  DeviceScope ds(ctx->opt.device);
  if (!ds.ok) return fail(IBIM_EHIP, "hipSetDevice failed");
  double* scr = nullptr;
  if (int r = noalloc_scratch(ctx->opt.device, &scr)) return r;
  return apply_core(ctx, u, out, as_stream(stream), sym_fits, scr, scr, false);
}

namespace {

// GMRES driver of ibim_solve (x0 = 0) and ibim_solve_guess (x0 = x on entry).
int solve_impl(ibim_ctx* ctx, const double* rhs, double tol, double* x, ibim_solve_info* info,
               void* stream, bool warm) {
  if (int r = check_dev(ctx)) return r;
  if (!rhs || !x || rhs == x) return fail(IBIM_EINVAL, "rhs and x must be distinct device vectors");
  if (!(tol > 0)) return fail(IBIM_EINVAL, "tol must be > 0");
  DeviceScope ds(ctx->opt.device);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = as_stream(stream);
  if (int r = ensure_krylov(ctx)) return r;
  ctx->applies = 0;
  Krylov& K = ctx->kr;
  const int64_t N = K.n;
  const int m = K.m;
  const unsigned nblk = (unsigned)((N + 255) / 256);
  double hv[2];
  // the system handed to GMRES: A x = b, or Lambda^-1 A x = Lambda^-1 b
  const bool diag = ctx->opt.precond == IBIM_PRECOND_DIAG;
  const double* b = rhs;
  if (diag) {
    HIP_TRY(launch_row_scaling(ctx, rhs, K.bsc, s), "row scaling");
    b = K.bsc;
  }
  auto op = [&](const double* u, double* out) -> int {
    if (int r = apply_impl(ctx, u, out, s)) return r;
    if (diag) HIP_TRY(launch_row_scaling(ctx, out, out, s), "row scaling");
    return IBIM_OK;
  };

  HIP_TRY(K.dots(b, N, 1, b, N, K.scal + 1, 0, s), "dots");
  if (int r = fetch(ctx, K.scal + 1, 1, s, hv)) return r;
  const double bnorm = std::sqrt(hv[0]);
  if (!warm || bnorm == 0.0) {
    hipLaunchKernelGGL(fill_kernel, dim3(nblk), dim3(256), 0, s, x, N, 0.0);
    HIP_TRY(hipGetLastError(), "fill");
  }
  int total = 0;
  bool converged = false;
  double resid = bnorm;
  if (!std::isfinite(bnorm)) return fail(IBIM_ENAN, "right-hand side is not finite");
  if (bnorm == 0.0) {
    if (info) *info = ibim_solve_info{0, 0, 1, 0.0, 0.0, 0.0};
    return IBIM_OK;
  }
  bool first = !warm;
  while (total < ctx->opt.max_iter && !converged) {
    // r = b - A x (x = 0 on a cold first cycle, where A x = 0 exactly)
    if (first) {
      hipLaunchKernelGGL(copy_kernel, dim3(nblk), dim3(256), 0, s, b, K.tmp, N);
      HIP_TRY(hipGetLastError(), "copy");
    } else {
      if (int r = op(x, K.tmp2)) return r;
      HIP_TRY(K.residual(b, K.tmp2, K.tmp, N, s), "residual");
    }
    first = false;
    HIP_TRY(K.dots(K.tmp, N, 1, K.tmp, N, K.scal + 1, 0, s), "dots");
    if (int r = fetch(ctx, K.scal + 1, 1, s, hv)) return r;
    const double beta = std::sqrt(hv[0]);
    if (!std::isfinite(beta)) return fail(IBIM_ENAN, "NaN in the GMRES residual");
    if (beta <= tol * bnorm) {
      converged = true;
      resid = beta;
      break;
    }
    HIP_TRY(K.normalize(K.tmp, K.scal + 1, K.V, N, s), "normalize");
    HIP_TRY(K.init_g(K.scal + 1, s), "init_g");
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = K.V + (int64_t)j * N;
      double* w = K.V + (int64_t)(j + 1) * N;
      if (int r = op(vj, w)) return r;
      ++total;
      // classical Gram-Schmidt, twice
      HIP_TRY(K.dots(K.V, N, j + 1, w, N, K.hcol, 0, s), "dots");
      HIP_TRY(K.sub(K.V, N, j + 1, K.hcol, w, N, s), "sub");
      HIP_TRY(K.dots(K.V, N, j + 1, w, N, K.hcol2, 0, s), "dots");
      HIP_TRY(K.sub(K.V, N, j + 1, K.hcol2, w, N, s), "sub");
      HIP_TRY(K.dots(w, N, 1, w, N, K.scal, 0, s), "dots");
      HIP_TRY(K.normalize(w, K.scal, w, N, s), "normalize");
      HIP_TRY(K.givens(j, s), "givens");
      if (int r = fetch(ctx, K.status, 2, s, hv)) return r;
      resid = hv[0];
      jend = j + 1;
      if (!std::isfinite(resid)) return fail(IBIM_ENAN, "NaN in the GMRES recurrence");
      if (resid <= tol * bnorm || hv[1] == 0.0) {
        converged = true;
        break;
      }
      if (total >= ctx->opt.max_iter) break;
    }
    HIP_TRY(K.backsolve(jend, s), "backsolve");
    HIP_TRY(K.add(K.V, N, jend, K.y, x, N, s), "update");
  }
  double explicit_rel = -1.0;
  if (ctx->opt.check_residual) {
    if (int r = op(x, K.tmp2)) return r;
    HIP_TRY(K.residual(b, K.tmp2, K.tmp, N, s), "residual");
    HIP_TRY(K.dots(K.tmp, N, 1, K.tmp, N, K.scal + 2, 0, s), "dots");
    if (int r = fetch(ctx, K.scal + 2, 1, s, hv)) return r;
    explicit_rel = std::sqrt(hv[0]) / bnorm;
    if (!std::isfinite(explicit_rel)) return fail(IBIM_ENAN, "NaN in the explicit residual");
  } else {
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info)
    *info = ibim_solve_info{total, ctx->applies, converged ? 1 : 0, resid / bnorm, explicit_rel, secs};
  return converged ? IBIM_OK : IBIM_NOT_CONVERGED;
}

}  // namespace

int ibim_solve(ibim_ctx* ctx, const double* rhs, double tol, double* x, ibim_solve_info* info,
               void* stream) {
  return solve_impl(ctx, rhs, tol, x, info, stream, false);
}

int ibim_solve_guess(ibim_ctx* ctx, const double* rhs, double tol, double* x,
                     ibim_solve_info* info, void* stream) {
  return solve_impl(ctx, rhs, tol, x, info, stream, true);
}

int ibim_energy(ibim_ctx* ctx, const double* x, double* g_pol, void* stream) {
  if (int r = check_dev(ctx)) return r;
  if (!x || !g_pol) return fail(IBIM_EINVAL, "x and g_pol must not be NULL");
  DeviceScope ds(ctx->opt.device);
  hipStream_t s = as_stream(stream);
  const int nc = (int)ctx->q.size();
  if (nc == 0) {
    *g_pol = 0.0;
    return IBIM_OK;
  }
  if (int r = energy_launch(ctx, x, s)) return r;
  std::vector<double> psi(nc);
  HIP_TRY(hipMemcpyAsync(psi.data(), ctx->d_psi, nc * sizeof(double), hipMemcpyDeviceToHost, s),
          "copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  const double G = energy_sum(ctx, psi.data());
  if (!std::isfinite(G)) return fail(IBIM_ENAN, "energy is not finite");
  *g_pol = G;
  return IBIM_OK;
}

int ibim_pair_timing(ibim_ctx* ctx, int enable) {
  if (int r = check_dev(ctx)) return r;
  ctx->timing = enable != 0;
  if (enable) ctx->tcount = 0;
  return IBIM_OK;
}

int ibim_pair_work(const ibim_ctx* ctx, double* pairs, double* flops) {
  if (int r = check_dev(ctx)) return r;
  if (!pairs || !flops) return fail(IBIM_EINVAL, "NULL output");
  *pairs = (double)ctx->P.M * (double)ctx->P.M;
  *flops = ctx->pair_flops;
  return IBIM_OK;
}

int ibim_tree_plan(const ibim_ctx* ctx, int64_t* counts, int32_t* perm, int32_t* bstart,
                   int32_t* cstart, int32_t* cend, double* cbox, int32_t* kid, int32_t* dstart,
                   int32_t* dend, int32_t* frow, int32_t* fcol, int32_t* nrow, int32_t* nlo,
                   int32_t* nhi, double* gap) {
  if (int r = check_ctx(ctx)) return r;
  if (ctx->opt.summation != IBIM_SUM_TREE) return fail(IBIM_EINVAL, "not a treecode context");
  const ibim::TreePlan& t = ctx->tplan;
  if (counts) {
    counts[0] = t.M;
    counts[1] = (int64_t)t.bstart.size() - 1;
    counts[2] = (int64_t)t.pstart.size();
    counts[3] = (int64_t)t.fcol.size();
    counts[4] = (int64_t)t.nlo.size();
    counts[5] = (int64_t)t.ibatch.size();
    counts[6] = t.order;
    counts[7] = 0;
  }
  auto put = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
  };
  put(perm, t.perm);
  put(bstart, t.bstart);
  put(cstart, t.pstart);
  put(cend, t.pend);
  if (cbox && !t.pbox.empty()) std::memcpy(cbox, t.pbox.data(), t.pbox.size() * sizeof(double));
  put(kid, t.kid);
  put(dstart, t.dstart);
  put(dend, t.dend);
  put(frow, t.frow);
  put(fcol, t.fcol);
  put(nrow, t.nrow);
  put(nlo, t.nlo);
  put(nhi, t.nhi);
  if (gap) *gap = t.gap;
  return IBIM_OK;
}

int ibim_tree_pairs(const ibim_ctx* ctx, int64_t* n, int32_t* lower, int32_t* upper) {
  if (int r = check_ctx(ctx)) return r;
  if (!n) return fail(IBIM_EINVAL, "NULL count");
  if (ctx->opt.summation != IBIM_SUM_TREE) return fail(IBIM_EINVAL, "not a treecode context");
  const ibim::TreePlan& t = ctx->tplan;
  *n = (int64_t)t.pcol.size();
  if (lower && !t.pown.empty()) std::memcpy(lower, t.pown.data(), t.pown.size() * sizeof(int32_t));
  if (upper && !t.pcol.empty()) std::memcpy(upper, t.pcol.data(), t.pcol.size() * sizeof(int32_t));
  return IBIM_OK;
}

int ibim_tree_counts(const ibim_ctx* ctx, double* out) {
  if (int r = check_dev(ctx)) return r;
  if (!out) return fail(IBIM_EINVAL, "NULL output");
  if (ctx->opt.summation != IBIM_SUM_TREE) return fail(IBIM_EINVAL, "not a treecode context");
  const ibim::TreePlan& t = ctx->tplan;
  out[0] = t.far_evals;
  out[1] = t.near_evals;
  out[2] = t.proxy_evals;
  out[3] = (double)(t.bstart.size() - 1);
  out[4] = (double)t.pstart.size();
  out[5] = t.m2m_links;
  return IBIM_OK;
}

int ibim_pair_timing_read(ibim_ctx* ctx, int64_t* launches, double* total_ms) {
  if (int r = check_dev(ctx)) return r;
  if (!launches || !total_ms) return fail(IBIM_EINVAL, "NULL output");
  DeviceScope ds(ctx->opt.device);
  double tot = 0.0;
  if (ctx->tcount > 0) HIP_TRY(hipEventSynchronize(ctx->tev[2 * ctx->tcount - 1]), "sync");
  for (size_t i = 0; i < ctx->tcount; ++i) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, ctx->tev[2 * i], ctx->tev[2 * i + 1]), "hipEventElapsedTime");
    tot += t;
  }
  *launches = (int64_t)ctx->tcount;
  *total_ms = tot;
  return IBIM_OK;
}

}  // extern "C"
