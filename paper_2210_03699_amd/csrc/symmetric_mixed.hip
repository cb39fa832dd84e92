// Mixed-precision form of the symmetric pair sum: float32 pair evaluations
// (geometry relative to the node centroid, in units of the Debye length when
// kappa h >= 1e-6, see sym_debye_units_f32), float64 row and column sums, on the
// schedule of symmetric.hip.  The finishing kernel adds, for every near
// pair (R < r_near), its float64 value minus the float32 value the pair
// kernel summed; the latter is recomputed by the same device function with
// the same operands (forward when the target's tile is the row tile of the
// tile pair, reverse when it is the column tile, one-directional for
// diagonal, corrected and ragged tile pairs), so the difference is exact.
//
// Compiled without automatic contraction: every float32 fused multiply-add
// is explicit, so both kernels produce identical float32 values.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "operator.h"
#include "pair_math.h"
#include "sym_core.h"
#include "symmetric.h"

namespace ibim {
namespace {

constexpr int kT = kPairTile;

// Values of node m's float32 record: with kUnit (SymArgs::unit32) in units of the
// Debye length (positions times kappa, w u1 times kappa^2, w u2 times kappa;
// the second row of sums then comes out divided by kappa), as in the float64
// kernel.  The finishing kernel forms the same values with these functions.
template <bool kUnit>
__device__ __forceinline__ float mixed_pos(float v, double kappa) {
  return kUnit ? (float)kappa * v : v;
}
template <bool kUnit>
__device__ __forceinline__ float mixed_q1(double wm, double u, double kappa) {
  return (float)(kUnit ? (wm * (kappa * kappa)) * u : wm * u);
}
template <bool kUnit>
__device__ __forceinline__ float mixed_q2(double wm, double u, double kappa) {
  return (float)(kUnit ? (wm * kappa) * u : wm * u);
}
template <bool kUnit>
__device__ __forceinline__ PairConstsF mixed_consts(double c1, double c2, double kappa) {
  return PairConstsF{(float)c1, (float)c2, kUnit ? 1.0f : (float)kappa,
                     kUnit ? 1.0f : (float)(kappa * kappa)};
}

struct MixedRec {
  float px, py, pz, nx, ny, nz, a1, a2;
};
struct MixedLds {
  float4 A[sym::kSlots], B[sym::kSlots];  // (px,py,pz,nx) (ny,nz,a1,a2) per LDS slot
};

template <bool kUnit>
struct Mixed {
  using Rec = MixedRec;
  using Lds = MixedLds;
  using Consts = PairConstsF;
  static __device__ __forceinline__ Consts consts(const SymArgs& a) {
    return mixed_consts<kUnit>(a.c1, a.c2, a.kappa);
  }
  static __device__ __forceinline__ double scale2(const SymArgs& a) {
    return kUnit ? a.scale * a.kappa : a.scale;
  }
  static __device__ __forceinline__ Rec load(const SymArgs& a, int32_t m) {
    const double wm = a.w[m], k = a.kappa;
    return Rec{mixed_pos<kUnit>(a.fx[m], k), mixed_pos<kUnit>(a.fy[m], k),
               mixed_pos<kUnit>(a.fz[m], k), a.fnx[m], a.fny[m], a.fnz[m],
               mixed_q1<kUnit>(wm, a.u[m], k), mixed_q2<kUnit>(wm, a.u[a.M + m], k)};
  }
  static __device__ __forceinline__ void store(Lds& s, int i, const Rec& r) {
    s.A[i] = make_float4(r.px, r.py, r.pz, r.nx);
    s.B[i] = make_float4(r.ny, r.nz, r.a1, r.a2);
  }
  static __device__ __forceinline__ Rec at(Lds& s, unsigned off) {
    const float4 q0 = *sym::lds_at(s.A, off), q1 = *sym::lds_at(s.B, off);
    return Rec{q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
  }
  static __device__ __forceinline__ void one(const Rec& t, const Rec& r, const Consts& pc,
                                             double& d1, double& d2) {
    float e1, e2;
    pair_f32(t.px, t.py, t.pz, t.nx, t.ny, t.nz, r.px, r.py, r.pz, r.nx, r.ny, r.nz, r.a1, r.a2,
             pc, e1, e2);
    d1 = (double)e1;
    d2 = (double)e2;
  }
  // (C1, C2) returned, or added to when kAcc
  template <bool kAcc = false>
  static __device__ __forceinline__ void both(const Rec& f, const Rec& m, const Consts& pc,
                                              double& S1, double& S2, double& C1, double& C2) {
    float d1, d2, c1, c2;
    pair_f32_sym<kUnit>(f.px, f.py, f.pz, f.nx, f.ny, f.nz, f.a1, f.a2, m.px, m.py, m.pz, m.nx,
                        m.ny, m.nz, m.a1, m.a2, pc, d1, d2, c1, c2);
    S1 += (double)d1;
    S2 += (double)d2;
    C1 = kAcc ? C1 + (double)c1 : (double)c1;
    C2 = kAcc ? C2 + (double)c2 : (double)c2;
  }
};

template <bool kUnit>
__global__ __launch_bounds__(256) void pair_sym_mixed_kernel(SymArgs a) {
  __shared__ sym::Shared<Mixed<kUnit>> sh;
  const int2 it = a.items[blockIdx.x];
  sym::item<Mixed<kUnit>>(a, it.x, it.y, sh);
}

__global__ __launch_bounds__(256, 4) void pair_sym_mixed_batched_kernel(
    const SymArgs* __restrict__ probs, const int32_t* __restrict__ work, int n_work,
    int* counter) {
  __shared__ sym::Shared<Mixed<true>> sh;  // one layout for both policies
  sym::batched(probs, work, n_work, counter, [&](const SymArgs& a, int rb, int cb) {
    if (a.unit32)
      sym::item<Mixed<true>>(a, rb, cb, sh);
    else
      sym::item<Mixed<false>>(a, rb, cb, sh);
  });
}


__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per row k: partial sums, sparse corrections and near-pair fix-ups
// are spread over the lanes in a fixed assignment and reduced in a fixed tree.
template <bool kUnit>
__device__ __forceinline__ void finish_sym_mixed_row(const SymMixedFinishArgs& a, int32_t k,
                                                     int lane, bool unscale) {
  const int32_t M = a.M;
  const int T = a.T;
  const int X = k / kT, t = k % kT;
  double p1 = 0.0, p2 = 0.0;
  const int cb0 = X / a.b, nr = a.nCB - cb0, nc = X / a.rows + 1;
  for (int j = lane; j < nr + nc; j += 64) {
    const double* sp = j < nr ? a.rowpart + sym_row_slot(cb0 + j, X, a.b, a.nCB) * (2 * kT)
                              : a.colpart + sym_col_slot(j - nr, X, a.rows) * (2 * kT);
    p1 += sp[t];
    p2 += sp[kT + t];
  }
  for (int32_t e = a.crow[k] + lane; e < a.crow[k + 1]; e += 64) {
    const int32_t m = a.ccol[e];
    const double* B = a.blocks + 4 * (size_t)e;
    const double v1 = a.u[m], v2 = a.u[M + m];
    p1 += B[0] * v1 + B[1] * v2;
    p2 += B[2] * v1 + B[3] * v2;
  }
  // near pairs
  const double x = a.px[k], y = a.py[k], z = a.pz[k];
  const double nxk = a.nx[k], nyk = a.ny[k], nzk = a.nz[k];
  const double kap = a.c64.kappa;
  const PairConstsF c32 = mixed_consts<kUnit>(a.c64.c1, a.c64.c2, kap);
  const float fx = mixed_pos<kUnit>(a.fx[k], kap), fy = mixed_pos<kUnit>(a.fy[k], kap);
  const float fz = mixed_pos<kUnit>(a.fz[k], kap);
  const float fnx = a.fnx[k], fny = a.fny[k], fnz = a.fnz[k];
  const double wk = a.w[k];
  const float ak1 = mixed_q1<kUnit>(wk, a.u[k], kap), ak2 = mixed_q2<kUnit>(wk, a.u[M + k], kap);
  const bool ragged = M % kT != 0;
  double f1 = 0.0, f2 = 0.0;
  for (int64_t e = a.nrow[k] + lane; e < a.nrow[k + 1]; e += 64) {
    const int32_t m = a.ncol[e];
    const int Y = m / kT;
    const double wm = a.w[m];
    const double a1 = wm * a.u[m], a2 = wm * a.u[M + m];
    double d1, d2;
    pair_f64<false>(x, y, z, nxk, nyk, nzk, a.px[m], a.py[m], a.pz[m], a.nx[m], a.ny[m], a.nz[m],
                    a1, a2, a.c64, d1, d2);
    const float am1 = mixed_q1<kUnit>(wm, a.u[m], kap), am2 = mixed_q2<kUnit>(wm, a.u[M + m], kap);
    const float mx = mixed_pos<kUnit>(a.fx[m], kap), my = mixed_pos<kUnit>(a.fy[m], kap);
    const float mz = mixed_pos<kUnit>(a.fz[m], kap);
    const float mnx = a.fnx[m], mny = a.fny[m], mnz = a.fnz[m];
    float e1, e2;
    const int lo = X < Y ? X : Y, hi = X < Y ? Y : X;
    const int64_t bit = (int64_t)lo * T + hi;
    const bool careful = (a.careful[bit >> 5] >> (bit & 31)) & 1u;
    if (X == Y || careful || (ragged && hi == T - 1)) {
      pair_f32(fx, fy, fz, fnx, fny, fnz, mx, my, mz, mnx, mny, mnz, am1, am2, c32, e1, e2);
    } else if (X < Y) {
      float c1, c2;
      pair_f32_sym<kUnit>(fx, fy, fz, fnx, fny, fnz, ak1, ak2, mx, my, mz, mnx, mny, mnz, am1,
                          am2, c32, e1, e2, c1, c2);
    } else {
      float d1f, d2f;
      pair_f32_sym<kUnit>(mx, my, mz, mnx, mny, mnz, am1, am2, fx, fy, fz, fnx, fny, fnz, ak1,
                          ak2, c32, d1f, d2f, e1, e2);
    }
    // the pair kernel's second row carries the factor kappa at write-out
    f1 += d1 - (double)e1;
    f2 += kUnit ? d2 - kap * (double)e2 : d2 - (double)e2;
  }
  p1 = wave_sum(p1);
  p2 = wave_sum(p2);
  f1 = wave_sum(f1);
  f2 = wave_sum(f2);
  if (lane == 0) {
    double o1 = a.lam1 * a.u[k] + p1 + a.scale * f1;
    double o2 = a.lam2 * a.u[M + k] + p2 + a.scale * f2;
    if (unscale) {
      o1 = o1 / a.lam1;
      o2 = o2 / a.lam2;
    }
    a.out[k] = o1;
    a.out[M + k] = o2;
  }
}

__global__ __launch_bounds__(256) void finish_sym_mixed_kernel(SymMixedFinishArgs a) {
  const int lane = threadIdx.x & 63;
  const int32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= a.M) return;  // uniform in the wave
  if (a.unit32)
    finish_sym_mixed_row<true>(a, k, lane, false);
  else
    finish_sym_mixed_row<false>(a, k, lane, false);
}

// Several problems: the block's problem is the last one whose blk0 <= block.
__global__ __launch_bounds__(256) void finish_sym_mixed_batched_kernel(
    const SymMixedFinishArgs* fa, int count, int unscale) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (fa[mid].blk0 <= blk) lo = mid; else hi = mid - 1;
  }
  const SymMixedFinishArgs& a = fa[lo];
  const int64_t k = (blk - a.blk0) * 4 + (threadIdx.x >> 6);
  if (k >= a.M) return;  // uniform in the wave
  if (a.unit32)
    finish_sym_mixed_row<true>(a, (int32_t)k, threadIdx.x & 63, unscale != 0);
  else
    finish_sym_mixed_row<false>(a, (int32_t)k, threadIdx.x & 63, unscale != 0);
}

}  // namespace

hipError_t launch_pair_sym_mixed(const SymArgs& a, int n_items, hipStream_t stream) {
  if (a.unit32)
    hipLaunchKernelGGL(pair_sym_mixed_kernel<true>, dim3((unsigned)n_items), dim3(256), 0, stream,
                       a);
  else
    hipLaunchKernelGGL(pair_sym_mixed_kernel<false>, dim3((unsigned)n_items), dim3(256), 0,
                       stream, a);
  return hipGetLastError();
}

hipError_t launch_pair_sym_mixed_batched(const SymArgs* probs, const int32_t* work, int n_work,
                                         int* counter, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(pair_sym_mixed_batched_kernel, dim3((unsigned)grid), dim3(256), 0, stream,
                     probs, work, n_work, counter);
  return hipGetLastError();
}

int pair_sym_mixed_batched_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_sym_mixed_batched_kernel, 256, 0) !=
          hipSuccess || per < 1)
    per = 1;
  return cus * per;
}

SymMixedFinishArgs make_finish_sym_mixed_args(const DeviceProblem& P, const SymPlan& pl,
                                              const uint32_t* careful, const double* u,
                                              const double* scratch, double* out) {
  SymMixedFinishArgs f;
  f.u = u;
  f.rowpart = scratch;
  f.colpart = scratch + sym_row_slots_total(pl.T, pl.b, pl.nCB) * 2 * kT;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
  f.nrow = P.nrow;
  f.ncol = P.ncol;
  f.px = P.px; f.py = P.py; f.pz = P.pz;
  f.nx = P.nx; f.ny = P.ny; f.nz = P.nz;
  f.w = P.w;
  f.fx = P.px32; f.fy = P.py32; f.fz = P.pz32;
  f.fnx = P.nx32; f.fny = P.ny32; f.fnz = P.nz32;
  f.careful = careful;
  f.c64 = PairConsts{P.eps_out / P.eps_in, P.eps_in / P.eps_out, P.kappa, P.kappa * P.kappa};
  f.unit32 = sym_debye_units_f32(P.kappa, P.h) ? 1 : 0;
  f.scale = P.h * P.h * P.h / (4.0 * 3.14159265358979323846);
  f.M = P.M;
  f.T = pl.T;
  f.b = pl.b;
  f.nCB = pl.nCB;
  f.rows = pl.rows;
  f.lam1 = P.lam1;
  f.lam2 = P.lam2;
  f.out = out;
  f.blk0 = 0;
  return f;
}

hipError_t launch_finish_sym_mixed(const DeviceProblem& P, const SymPlan& pl,
                                   const uint32_t* careful, const double* u,
                                   const double* scratch, double* out, hipStream_t stream) {
  const SymMixedFinishArgs f = make_finish_sym_mixed_args(P, pl, careful, u, scratch, out);
  const unsigned blocks = (unsigned)((P.M + 3) / 4);
  hipLaunchKernelGGL(finish_sym_mixed_kernel, dim3(blocks), dim3(256), 0, stream, f);
  return hipGetLastError();
}

hipError_t launch_finish_sym_mixed_batched(SymMixedFinishArgs* args, int count,
                                           SymMixedFinishArgs* d_args, bool unscale,
                                           hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t blk = 0;
  for (int q = 0; q < count; ++q) {
    args[q].blk0 = blk;
    blk += (args[q].M + 3) / 4;
  }
  hipError_t e = hipMemcpyAsync(d_args, args, sizeof(SymMixedFinishArgs) * (size_t)count,
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_sym_mixed_batched_kernel, dim3((unsigned)blk), dim3(256), 0, stream,
                     d_args, count, unscale ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ibim
