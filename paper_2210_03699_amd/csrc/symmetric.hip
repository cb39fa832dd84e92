// Symmetric evaluation of the dense pair sum (float64).
//
// The four kernels of eq. (Kij-kernels) for the ordered pairs (k <- m) and
// (m <- k) share R, e^{-kR}, e^{-kR}(1 + kR), r.n_k, r.n_m and n_k.n_m: with
// r' = -r the reverse pair has r'.n_k = -r.n_m, r'.n_m = -r.n_k and the same
// product q.  One evaluation therefore yields both contributions, and the
// dense sum costs about half the instructions of the one-directional kernel.
//
// Tiles are 256 nodes.  Work item (rb, cb) covers row tiles
// I in [rb*rows, rb*rows + rows) and column tiles J in [cb*b, cb*b + b),
// pairs I <= J only.  For each column tile J the workgroup stages J's records
// in LDS and, for each row tile I (two at a time where both are plain tile
// pairs), evaluates all 256 x 256 pairs: wave w holds targets I[64w + l]
// (one per lane) and, in phase p, visits the 64 sources of sub-block
// (w + p) mod 4 in the rotated order l, l+1, ... (mod 64), eight at a time
// from one LDS base address (each sub-block is followed by copies of its
// first eight records, so the eight never wrap).  The row sums of a tile
// pair stay in registers and are carried across the item in lane-private
// LDS slots (items of up to four row tiles) or in their (cb, I) scratch
// slots; the column sums of J go to an LDS accumulator, which in any phase
// each wave updates in its own sub-block and each lane at its own slot, so
// every slot is summed in a fixed order.
// Diagonal tile pairs, pairs holding a corrected pair (either direction) and
// pairs with the ragged last tile are evaluated one direction at a time with
// the pairs of N_k skipped.  Row sums are written per (cb, I), column sums
// per (rb, J) (only rb <= J / rows occur, so those slots are packed); the
// finishing kernel adds them in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "operator.h"
#include "pair_math.h"
#include "sym_core.h"
#include "symmetric.h"
#include "weights.h"

namespace ibim {
namespace {

constexpr int kT = kPairTile;

// float64 arithmetic: records of 8 doubles, LDS as four double2 arrays.
// With kUnit (kappa > 0) lengths are measured in units of the Debye length
// 1/kappa: a record holds kappa P_m, kappa^2 w_m u1_m and kappa w_m u2_m.  In
// the dimensionless distance rho = kappa R the Yukawa factors read e^{-rho},
// 1 + rho and (for K21) a plain e^{-rho}/rho^3, which saves the two
// multiplications by kappa and kappa^2 of every pair; each kernel is a
// power of kappa times its dimensionless form, so the first sums come out
// unchanged and the second divided by kappa, which scale2 puts back when the
// partial sums are written.  Without kUnit (kappa = 0 or negligible) the
// records hold P_m, w_m u1_m and w_m u2_m and kappa enters each pair.
struct Fp64Rec {
  double px, py, pz, nx, ny, nz, a1, a2;
};
struct Fp64Lds {
  // (px,py) (pz,nx) (ny,nz) (a1,a2) per LDS slot (sym::slot)
  double2 A[sym::kSlots], B[sym::kSlots], C[sym::kSlots], D[sym::kSlots];
};
template <bool kUnit>
struct Fp64 {
  using Rec = Fp64Rec;
  using Lds = Fp64Lds;
  struct Consts {
    PairConsts k;  // one-directional evaluations
    ExpWave ew;    // table exponential of the symmetric evaluation
  };
  static __device__ __forceinline__ Consts consts(const SymArgs& a) {
    const double kap = kUnit ? 1.0 : a.kappa;
    return Consts{PairConsts{a.c1, a.c2, kap, kap * kap}, exp_wave_init(kap)};
  }
  // multiplier of the second row of partial sums at write-out
  static __device__ __forceinline__ double scale2(const SymArgs& a) {
    return kUnit ? a.scale * a.kappa : a.scale;
  }
  static __device__ __forceinline__ Rec load(const SymArgs& a, int32_t m) {
    const double wm = a.w[m];
    if (kUnit) {
      const double k = a.kappa, wk = wm * k;
      return Rec{k * a.px[m], k * a.py[m], k * a.pz[m], a.nx[m], a.ny[m], a.nz[m],
                 (wk * k) * a.u[m], wk * a.u[a.M + m]};
    }
    return Rec{a.px[m], a.py[m], a.pz[m], a.nx[m], a.ny[m], a.nz[m], wm * a.u[m],
               wm * a.u[a.M + m]};
  }
  static __device__ __forceinline__ void store(Lds& s, int i, const Rec& r) {
    s.A[i] = make_double2(r.px, r.py);
    s.B[i] = make_double2(r.pz, r.nx);
    s.C[i] = make_double2(r.ny, r.nz);
    s.D[i] = make_double2(r.a1, r.a2);
  }
  static __device__ __forceinline__ Rec at(Lds& s, unsigned off) {
    const double2 q0 = *sym::lds_at(s.A, off), q1 = *sym::lds_at(s.B, off);
    const double2 q2 = *sym::lds_at(s.C, off), q3 = *sym::lds_at(s.D, off);
    return Rec{q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
  }
  static __device__ __forceinline__ void one(const Rec& t, const Rec& r, const Consts& pc,
                                             double& d1, double& d2) {
    pair_f64<false>(t.px, t.py, t.pz, t.nx, t.ny, t.nz, r.px, r.py, r.pz, r.nx, r.ny, r.nz, r.a1,
                    r.a2, pc.k, d1, d2);
  }
  // Both directions of the pair (fixed f, rotating m): k <- m added to
  // (S1, S2), m <- k returned in (C1, C2), or added to them when kAcc.  With
  // u = (1 - e(1 + kR))/R^3 and t3 = e(1 + kR)/R^3 the kernel factors are
  // (1 - c t)/R^3 = 1/R^3 - c t3 and K21 R^3 / R^3 = n_k.n_m u + q (k^2 e/R^3
  // - 3 u/R^2) (k = 1 with kUnit).  Called with all 64 lanes of the
  // wavefront active (the exponential reads other lanes).
  template <bool kAcc = false>
  static __device__ __forceinline__ void both(const Rec& f, const Rec& m, const Consts& pc,
                                              double& S1, double& S2, double& C1, double& C2) {
    const double rx = f.px - m.px, ry = f.py - m.py, rz = f.pz - m.pz;  // r = x_k - P_m
    const double R2s = fma(rz, rz, fma(ry, ry, rx * rx));
    const double iR = rsqrt_pos(R2s);
    const double R = R2s * iR;
    const double iR2 = iR * iR;
    const double iR3 = iR2 * iR;
    const double e = exp_neg_wave(R, pc.ew);
    const double kr = kUnit ? R : pc.k.kappa * R;
    const double rny = fma(rz, m.nz, fma(ry, m.ny, rx * m.nx));  // r . n_m
    const double rnx = fma(rz, f.nz, fma(ry, f.ny, rx * f.nx));  // r . n_k
    const double nn = fma(f.nz, m.nz, fma(f.ny, m.ny, f.nx * m.nx));
    const double eiR3 = e * iR3;
    const double t3 = fma(eiR3, kr, eiR3);
    const double u = iR3 - t3;
    const double f1 = fma(-pc.k.c1, t3, iR3);
    const double f2 = fma(-pc.k.c2, t3, iR3);
    const double g12 = fma(-e, iR, iR);  // (1 - e)/R
    const double q = rnx * rny;
    const double k2e = kUnit ? eiR3 : pc.k.kappa2 * eiR3;
    const double g21 = fma(nn, u, q * fma(u * iR2, -3.0, k2e));
    // k <- m
    const double g11 = rny * f1, g22 = rnx * f2;
    S1 = fma(g11, m.a1, fma(-g12, m.a2, S1));
    S2 = fma(g21, m.a1, fma(g22, m.a2, S2));
    // m <- k: r.n_k and r.n_m swap roles with a sign change
    const double h11 = -rnx * f1, h22 = -rny * f2;
    if (kAcc) {
      C1 = fma(h11, f.a1, fma(-g12, f.a2, C1));
      C2 = fma(g21, f.a1, fma(h22, f.a2, C2));
    } else {
      C1 = fma(h11, f.a1, -g12 * f.a2);
      C2 = fma(g21, f.a1, h22 * f.a2);
    }
  }
};

template <bool kUnit>
__global__ __launch_bounds__(256) void pair_sym_fp64_kernel(SymArgs a) {
  __shared__ sym::Shared<Fp64<kUnit>> sh;
  const int2 it = a.items[blockIdx.x];
  sym::item<Fp64<kUnit>>(a, it.x, it.y, sh);
}

__global__ __launch_bounds__(256, 3) void pair_sym_batched_kernel(
    const SymArgs* __restrict__ probs, const int32_t* __restrict__ work, int n_work,
    int* counter) {
  __shared__ sym::Shared<Fp64<true>> sh;  // one layout for both policies
  sym::batched(probs, work, n_work, counter, [&](const SymArgs& a, int rb, int cb) {
    if (sym_debye_units(a.kappa))
      sym::item<Fp64<true>>(a, rb, cb, sh);
    else
      sym::item<Fp64<false>>(a, rb, cb, sh);
  });
}


// Row k of one problem: partial slots, Lambda u and the sparse blocks
// (divided by lambda when unscale is set).
__device__ __forceinline__ void finish_sym_row(const SymFinishArgs& a, int32_t k, bool unscale) {
  const int32_t M = a.M;
  const int X = k / kT, t = k % kT;
  double s1 = 0.0, s2 = 0.0;
  for (int cb = X / a.b; cb < a.nCB; ++cb) {
    const double* rp = a.rowpart + sym_row_slot(cb, X, a.b, a.nCB) * (2 * kT);
    s1 += rp[t];
    s2 += rp[kT + t];
  }
  const size_t c0 = sym_col_slot(0, X, a.rows);
  for (int rb = 0; rb <= X / a.rows; ++rb) {
    const double* cp = a.colpart + (c0 + rb) * (2 * kT);
    s1 += cp[t];
    s2 += cp[kT + t];
  }
  double o1 = a.lam1 * a.u[k] + s1;
  double o2 = a.lam2 * a.u[M + k] + s2;
  for (int32_t e = a.crow[k]; e < a.crow[k + 1]; ++e) {
    const int32_t m = a.ccol[e];
    const double* B = a.blocks + 4 * (size_t)e;
    const double v1 = a.u[m], v2 = a.u[M + m];
    o1 += B[0] * v1 + B[1] * v2;
    o2 += B[2] * v1 + B[3] * v2;
  }
  if (unscale) {
    o1 = o1 / a.lam1;
    o2 = o2 / a.lam2;
  }
  a.out[k] = o1;
  a.out[M + k] = o2;
}

__global__ __launch_bounds__(256) void finish_sym_kernel(SymFinishArgs a) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.M) return;
  finish_sym_row(a, k, false);
}

// Several problems: the block's problem is the last one whose blk0 <= block.
__global__ __launch_bounds__(256) void finish_sym_batched_kernel(const SymFinishArgs* fa,
                                                                 int count, int unscale) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (fa[mid].blk0 <= blk) lo = mid; else hi = mid - 1;
  }
  const SymFinishArgs& a = fa[lo];
  const int64_t k = (blk - a.blk0) * 256 + threadIdx.x;
  if (k >= a.M) return;
  finish_sym_row(a, (int32_t)k, unscale != 0);
}

}  // namespace

SymPlan make_sym_plan(int32_t M, size_t max_scratch_bytes) {
  SymPlan pl;
  pl.T = (M + kT - 1) / kT;
  // row tiles per item: a column tile staged in LDS serves `rows` row
  // tiles, and the column partial sums take about T^2 / (2 rows) slots of 4
  // KiB: 4 row tiles up to T = 2048 (M = 524,288), then doubled while T
  // exceeds 512 x rows, up to 64, which keeps the scratch under 32 GiB to
  // M ~ 5e6; fewer for small problems so that they still have ~2048 items
  int rows = 4;
  while (rows < 64 && rows * 512 < pl.T) rows *= 2;
  while (rows > 1) {
    const int64_t nrb = (pl.T + rows - 1) / rows;
    if (nrb * pl.T / 2 >= 2048) break;
    rows /= 2;
  }
  pl.rows = rows;
  pl.nRB = (pl.T + rows - 1) / rows;
  // column block length: the shortest that keeps the item count at or under
  // 8192, so that small problems still spread over many compute units, and
  // under 2048 per row tile of an item up to 32768 for larger items (items
  // of more row tiles are longer, and a launch needs many of them to end
  // evenly); at most 128 tiles: the row partial sums take about T^2 / (2 b)
  // slots
  const int64_t max_items = std::min<int64_t>(32768, std::max<int64_t>(8192, 2048 * rows));
  int b = 1;
  while (b < 128) {
    const int64_t nCB = (pl.T + b - 1) / b;
    const int64_t items = (int64_t)pl.nRB * nCB / 2;
    if (items <= max_items) break;
    b *= 2;
  }
  pl.b = b;
  pl.nCB = (pl.T + b - 1) / b;
  pl.scratch_doubles =
      (sym_row_slots_total(pl.T, b, pl.nCB) + sym_col_slot(0, pl.T, rows)) * 2 * kT;
  pl.enabled = pl.T >= 2 && pl.scratch_doubles * 8 <= max_scratch_bytes;
  return pl;
}

void sym_items(const SymPlan& pl, const std::vector<uint32_t>& careful, bool ragged,
               std::vector<int32_t>* items) {
  // Workgroups start in launch order, so the costliest items go first: a
  // tile pair holding a corrected pair, or one with the ragged last tile, is
  // evaluated one direction at a time with a global-memory pass for the
  // reverse direction (weighted 4 here), a diagonal tile pair one direction
  // only (1.25), a plain tile pair both ways at once (1).  Items of the plain
  // full cost follow, arranged for the L2 of the XCDs: workgroup i runs on
  // XCD i mod kXcds and each XCD has its own L2, while an item (rb, cb)
  // stages the b column tiles of cb one after another and reloads its
  // `rows` row tiles for each; listed in blocks of kBR row blocks x kBC
  // column blocks, with each XCD taking a contiguous stretch of that list,
  // the ~100 items an XCD runs at once share their row and column tiles.
  // The cheaper (partial) items come last, costliest first.
  constexpr int kXcds = 8, kBR = 16, kBC = 8;
  constexpr int kPlain = 4, kDiag = 5, kSlow = 16;  // costs of a tile pair, in quarters
  struct It {
    int rb, cb;
    int64_t cost;
  };
  auto cost_of = [&](int rb, int cb) {
    int64_t c = 0;
    for (int I = rb * pl.rows; I < std::min(rb * pl.rows + pl.rows, pl.T); ++I)
      for (int J = std::max(I, cb * pl.b); J < std::min(cb * pl.b + pl.b, pl.T); ++J) {
        const size_t bit = (size_t)I * pl.T + J;
        const bool slow = ((careful[bit >> 5] >> (bit & 31)) & 1u) || (ragged && J == pl.T - 1);
        c += I == J ? kDiag : slow ? kSlow : kPlain;
      }
    return c;
  };
  const int64_t plain_full = (int64_t)kPlain * pl.rows * pl.b;
  std::vector<It> costly, whole, rest;
  for (int rb0 = 0; rb0 < pl.nRB; rb0 += kBR)
    for (int cb0 = 0; cb0 < pl.nCB; cb0 += kBC)
      for (int rb = rb0; rb < std::min(rb0 + kBR, pl.nRB); ++rb)
        for (int cb = std::max(cb0, (rb * pl.rows) / pl.b); cb < std::min(cb0 + kBC, pl.nCB);
             ++cb) {
          const int64_t c = cost_of(rb, cb);
          if (c == 0) continue;
          (c > plain_full ? costly : c == plain_full ? whole : rest).push_back({rb, cb, c});
        }
  auto by_cost = [](const It& x, const It& y) { return x.cost > y.cost; };
  std::stable_sort(costly.begin(), costly.end(), by_cost);
  std::stable_sort(rest.begin(), rest.end(), by_cost);
  items->clear();
  auto put = [&](const It& it) {
    items->push_back(it.rb);
    items->push_back(it.cb);
  };
  for (const It& it : costly) put(it);
  // plain items: XCD x takes the x-th contiguous stretch, each item at the
  // next position that runs on x (another XCD's when x has run out)
  const size_t F = whole.size();
  std::vector<size_t> at(kXcds + 1, 0), next(kXcds);
  for (int x = 0; x < kXcds; ++x) at[x + 1] = at[x] + F / kXcds + ((size_t)x < F % kXcds);
  for (int x = 0; x < kXcds; ++x) next[x] = at[x];
  for (size_t q = 0; q < F; ++q) {
    int x = (int)((items->size() / 2) % kXcds);
    for (int t = 0; next[x] == at[x + 1] && t < kXcds; ++t) x = (x + 1) % kXcds;
    put(whole[next[x]++]);
  }
  for (const It& it : rest) put(it);
}

void sym_careful_bits(int T, const std::vector<int32_t>& xrow, const std::vector<int32_t>& xtile,
                      std::vector<uint32_t>* bits) {
  bits->assign(((size_t)T * T + 31) / 32, 0u);
  auto set = [&](int I, int J) {
    const size_t b = (size_t)I * T + J;
    (*bits)[b >> 5] |= 1u << (b & 31);
  };
  for (int I = 0; I < T; ++I)
    for (int32_t p = xrow[I]; p < xrow[I + 1]; ++p) {
      const int J = xtile[p];
      set(I, J);
      set(J, I);
    }
}

SymArgs make_sym_args(const DeviceProblem& P, const SymPlan& pl, const int32_t* items,
                      const uint32_t* careful, const double* u, double* scratch) {
  SymArgs a{};
  a.px = P.px; a.py = P.py; a.pz = P.pz;
  a.nx = P.nx; a.ny = P.ny; a.nz = P.nz;
  a.w = P.w;
  a.fx = P.px32; a.fy = P.py32; a.fz = P.pz32;
  a.fnx = P.nx32; a.fny = P.ny32; a.fnz = P.nz32;
  a.u = u;
  a.crow = P.crow;
  a.ccol = P.ccol;
  a.careful = careful;
  a.items = reinterpret_cast<const int2*>(items);
  a.M = P.M;
  a.T = pl.T;
  a.b = pl.b;
  a.rows = pl.rows;
  a.c1 = P.eps_out / P.eps_in;
  a.c2 = P.eps_in / P.eps_out;
  a.kappa = P.kappa;
  a.unit32 = sym_debye_units_f32(P.kappa, P.h) ? 1 : 0;
  a.scale = P.h * P.h * P.h / (4.0 * kPiD);
  a.rowpart = scratch;
  a.colpart = scratch + sym_row_slots_total(pl.T, pl.b, pl.nCB) * 2 * kT;
  return a;
}

hipError_t launch_pair_sym(const SymArgs& a, int n_items, hipStream_t stream) {
  if (sym_debye_units(a.kappa))
    hipLaunchKernelGGL(pair_sym_fp64_kernel<true>, dim3((unsigned)n_items), dim3(256), 0, stream,
                       a);
  else
    hipLaunchKernelGGL(pair_sym_fp64_kernel<false>, dim3((unsigned)n_items), dim3(256), 0, stream,
                       a);
  return hipGetLastError();
}

hipError_t launch_pair_sym_batched(const SymArgs* probs, const int32_t* work, int n_work,
                                   int* counter, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(pair_sym_batched_kernel, dim3((unsigned)grid), dim3(256), 0, stream, probs,
                     work, n_work, counter);
  return hipGetLastError();
}

int pair_sym_batched_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_sym_batched_kernel, 256, 0) !=
          hipSuccess || per < 1)
    per = 1;
  return cus * per;
}

SymFinishArgs make_finish_sym_args(const DeviceProblem& P, const SymPlan& pl, const double* u,
                                   const double* scratch, double* out) {
  SymFinishArgs f;
  f.u = u;
  f.rowpart = scratch;
  f.colpart = scratch + sym_row_slots_total(pl.T, pl.b, pl.nCB) * 2 * kT;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
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

hipError_t launch_finish_sym(const DeviceProblem& P, const SymPlan& pl, const double* u,
                             const double* scratch, double* out, hipStream_t stream) {
  const SymFinishArgs f = make_finish_sym_args(P, pl, u, scratch, out);
  const unsigned blocks = (unsigned)((P.M + 255) / 256);
  hipLaunchKernelGGL(finish_sym_kernel, dim3(blocks), dim3(256), 0, stream, f);
  return hipGetLastError();
}

hipError_t launch_finish_sym_batched(SymFinishArgs* args, int count, SymFinishArgs* d_args,
                                     bool unscale, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t blk = 0;
  for (int q = 0; q < count; ++q) {
    args[q].blk0 = blk;
    blk += (args[q].M + 255) / 256;
  }
  hipError_t e = hipMemcpyAsync(d_args, args, sizeof(SymFinishArgs) * (size_t)count,
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_sym_batched_kernel, dim3((unsigned)blk), dim3(256), 0, stream, d_args,
                     count, unscale ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ibim
