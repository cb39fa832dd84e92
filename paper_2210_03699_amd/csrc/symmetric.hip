// Symmetric evaluation of the dense pair sum (float64).
//
// The four kernels of eq. (Kij-kernels) for the ordered pairs (k <- m) and
// (m <- k) share R, e^{-kR}, e^{-kR}(1 + kR), r.n_k, r.n_m and n_k.n_m: with
// r' = -r the reverse pair has r'.n_k = -r.n_m, r'.n_m = -r.n_k and the same
// product q.  One evaluation therefore yields both contributions, and the
// dense sum costs about half the instructions of the one-directional kernel.
//
// Tiles are 256 nodes.  Work item (rb, cb) covers row tiles
// I in [rb*kRows, rb*kRows + kRows) and column tiles J in [cb*b, cb*b + b),
// pairs I <= J only.  For each column tile J the workgroup stages J's records
// in LDS and, for each row tile I, evaluates all 256 x 256 pairs: wave w holds
// targets I[64w + l] (one per lane) and, in phase p, visits the 64 sources of
// sub-block (w + p) mod 4 in the rotated order l, l+1, ... (mod 64).  The
// row sums stay in registers across the item; the column sums of J go to an
// LDS accumulator, which in any phase each wave updates in its own sub-block
// and each lane at its own slot, so every slot is summed in a fixed order.
// Diagonal tile pairs, pairs holding a corrected pair (either direction) and
// pairs with the ragged last tile are evaluated one direction at a time with
// the pairs of N_k skipped.  Row sums are written per (cb, I), column sums
// per (rb, J); the finishing kernel adds them in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "operator.h"
#include "pair_math.h"
#include "symmetric.h"
#include "weights.h"

namespace ibim {
namespace {

constexpr int kT = kPairTile;
constexpr int kRows = kSymRows;

struct Rec {
  double px, py, pz, nx, ny, nz, a1, a2;
};

__device__ __forceinline__ Rec load_rec(const SymArgs& a, int32_t m) {
  const double wm = a.w[m];
  return Rec{a.px[m], a.py[m], a.pz[m], a.nx[m], a.ny[m], a.nz[m], wm * a.u[m],
             wm * a.u[a.M + m]};
}

// Sums over the sources of tile Y for the target of this lane in tile X
// (k = X*256 + tid), pairs of N_k skipped.  src(j) returns source j of Y.
template <class Src>
__device__ __forceinline__ void one_way(const SymArgs& a, int X, int Y, const Src& src,
                                        double& S1, double& S2) {
  const int tid = threadIdx.x;
  const int32_t M = a.M;
  const int32_t k = X * kT + tid;
  const int32_t kc = k < M ? k : M - 1;
  const double tx = a.px[kc], ty = a.py[kc], tz = a.pz[kc];
  const double tnx = a.nx[kc], tny = a.ny[kc], tnz = a.nz[kc];
  const int32_t s0 = Y * kT;
  const int n = min(kT, M - s0);
  int32_t p = a.crow[kc];
  const int32_t pe = a.crow[kc + 1];
  while (p < pe && a.ccol[p] < s0) ++p;
  int32_t nxt = p < pe ? a.ccol[p] : INT_MAX;
  const PairConsts pc{a.c1, a.c2, a.kappa, a.kappa * a.kappa};
  for (int j = 0; j < n; ++j) {
    const Rec r = src(j);
    double d1, d2;
    pair_f64<false>(tx, ty, tz, tnx, tny, tnz, r.px, r.py, r.pz, r.nx, r.ny, r.nz, r.a1, r.a2,
                    pc, d1, d2);
    const bool ex = (s0 + j == nxt);
    if (ex) {
      ++p;
      nxt = p < pe ? a.ccol[p] : INT_MAX;
    }
    S1 += ex ? 0.0 : d1;
    S2 += ex ? 0.0 : d2;
  }
}

// Element of a shared double2 array at a byte offset.
__device__ __forceinline__ double2* lds_at(double2* base, unsigned byte_off) {
  return reinterpret_cast<double2*>(reinterpret_cast<char*>(base) + byte_off);
}

__device__ __forceinline__ bool careful_pair(const SymArgs& a, int I, int J) {
  const int64_t bit = (int64_t)I * a.T + J;
  return (a.careful[bit >> 5] >> (bit & 31)) & 1u;
}

struct SymShared {
  double2 sA[kT], sB[kT], sC[kT], sD[kT];  // records of J: (px,py) (pz,nx) (ny,nz) (a1,a2)
  double2 cacc[kT];                        // column sums of J (row 1, row 2)
  double racc1[kRows][kT], racc2[kRows][kT];  // row sums, lane-private slots
};

// One work item (rb, cb).  Called by all 256 threads of the workgroup.
__device__ void sym_item(const SymArgs& a, int rb, int cb, SymShared& sh) {
  double2* const sA = sh.sA;
  double2* const sB = sh.sB;
  double2* const sC = sh.sC;
  double2* const sD = sh.sD;
  double2* const cacc = sh.cacc;
  auto& racc1 = sh.racc1;
  auto& racc2 = sh.racc2;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, l = tid & 63;
  const int T = a.T;
  const int32_t M = a.M;
  const int I0 = rb * kRows;
  const int J0 = cb * a.b, J1 = min(J0 + a.b, T);
  const PairConsts pc{a.c1, a.c2, a.kappa, a.kappa * a.kappa};

  for (int i = 0; i < kRows; ++i) racc1[i][tid] = racc2[i][tid] = 0.0;

  for (int J = max(J0, I0); J < J1; ++J) {
    {
      const int32_t m = J * kT + tid;
      if (m < M) {
        const Rec r = load_rec(a, m);
        sA[tid] = make_double2(r.px, r.py);
        sB[tid] = make_double2(r.pz, r.nx);
        sC[tid] = make_double2(r.ny, r.nz);
        sD[tid] = make_double2(r.a1, r.a2);
      }
      cacc[tid] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int i = 0; i < kRows; ++i) {
      const int I = I0 + i;
      if (I >= T || I > J) continue;  // uniform
      double S1 = racc1[i][tid], S2 = racc2[i][tid];
      const bool slow = I == J || careful_pair(a, I, J) || (J == T - 1 && M % kT != 0);
      if (slow) {
        // row I from the sources of J (LDS broadcasts)
        one_way(a, I, J, [&](int j) {
          const double2 q0 = sA[j], q1 = sB[j], q2 = sC[j], q3 = sD[j];
          return Rec{q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
        }, S1, S2);
        racc1[i][tid] = S1;
        racc2[i][tid] = S2;
        if (I != J) {
          // row J from the sources of I (uniform global loads)
          double c1 = 0.0, c2 = 0.0;
          one_way(a, J, I, [&](int j) { return load_rec(a, I * kT + j); }, c1, c2);
          cacc[tid].x += c1;
          cacc[tid].y += c2;
        }
        __syncthreads();
        continue;
      }
      const int32_t k = I * kT + tid;
      const Rec f = load_rec(a, k);
      for (int ph = 0; ph < 4; ++ph) {
        // byte offsets into the double2 arrays: sub-block base | ((l + s) mod 64) * 16
        const unsigned sb16 = (unsigned)(((wv + ph) & 3) * 64) << 4;
        unsigned x16 = (unsigned)l << 4;
#pragma unroll 2
        for (int s = 0; s < 64; ++s) {
          const unsigned off = (x16 & 1008u) | sb16;
          x16 += 16u;
          const double2 q0 = *lds_at(sA, off), q1 = *lds_at(sB, off);
          const double2 q2 = *lds_at(sC, off), q3 = *lds_at(sD, off);
          // r = x_k - P_m
          const double rx = f.px - q0.x, ry = f.py - q0.y, rz = f.pz - q1.x;
          const double R2s = fma(rz, rz, fma(ry, ry, rx * rx));
          const double iR = rsqrt_pos(R2s);
          const double R = R2s * iR;
          const double iR2 = iR * iR;
          const double iR3 = iR2 * iR;
          const double kr = pc.kappa * R;
          const double e = exp_neg(kr);
          const double te = fma(e, kr, e);
          const double rny = fma(rz, q2.y, fma(ry, q2.x, rx * q1.y));  // r . n_m
          const double rnx = fma(rz, f.nz, fma(ry, f.ny, rx * f.nx));  // r . n_k
          const double nn = fma(f.nz, q2.y, fma(f.ny, q2.x, f.nx * q1.y));
          // kernel factors with 1/R^3 folded in
          const double f1 = fma(-pc.c1, te, 1.0) * iR3;
          const double f2 = fma(-pc.c2, te, 1.0) * iR3;
          const double g12 = (1.0 - e) * iR;
          const double phi2 = 1.0 - te;
          const double q = rnx * rny;
          const double g21 = fma(phi2, fma(q * iR2, -3.0, nn), pc.kappa2 * e * q) * iR3;
          // k <- m
          const double g11 = rny * f1, g22 = rnx * f2;
          S1 = fma(g11, q3.x, fma(-g12, q3.y, S1));
          S2 = fma(g21, q3.x, fma(g22, q3.y, S2));
          // m <- k: r.n_k and r.n_m swap roles with a sign change
          const double h11 = -rnx * f1, h22 = -rny * f2;
          const double C1 = fma(h11, f.a1, -g12 * f.a2);
          const double C2 = fma(g21, f.a1, h22 * f.a2);
          double2* c = lds_at(cacc, off);
          atomicAdd(&c->x, C1);
          atomicAdd(&c->y, C2);
        }
        __syncthreads();
      }
      racc1[i][tid] = S1;
      racc2[i][tid] = S2;
    }
    // column sums of J
    double* cp = a.colpart + ((size_t)rb * T + J) * (2 * kT);
    cp[tid] = a.scale * cacc[tid].x;
    cp[kT + tid] = a.scale * cacc[tid].y;
    __syncthreads();  // LDS is refilled for the next column tile
  }
  // row sums of this item's row tiles that met at least one J >= I
  for (int i = 0; i < kRows; ++i) {
    const int I = I0 + i;
    if (I >= T || I > J1 - 1) continue;
    double* rp = a.rowpart + ((size_t)cb * T + I) * (2 * kT);
    rp[tid] = a.scale * racc1[i][tid];
    rp[kT + tid] = a.scale * racc2[i][tid];
  }
}

__global__ __launch_bounds__(256) void pair_sym_fp64_kernel(SymArgs a) {
  __shared__ SymShared sh;
  const int2 item = a.items[blockIdx.x];
  sym_item(a, item.x, item.y, sh);
}

// Persistent form over the items of several problems: entry i of `work` is
// (problem, item index); workgroups take entries from *counter (initially 0).
__global__ __launch_bounds__(256, 4) void pair_sym_batched_kernel(
    const SymArgs* __restrict__ probs, const int32_t* __restrict__ work, int n_work,
    int* counter) {
  __shared__ SymShared sh;
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    // the item index is uniform: keep it (and so the argument record) scalar
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // every thread has read `next` before it is overwritten
    if (it >= n_work) break;
    const int pi = __builtin_amdgcn_readfirstlane(work[2 * it]);
    const int ii = __builtin_amdgcn_readfirstlane(work[2 * it + 1]);
    const SymArgs a = probs[pi];
    const int2 item = a.items[ii];
    sym_item(a, __builtin_amdgcn_readfirstlane(item.x), __builtin_amdgcn_readfirstlane(item.y), sh);
    __syncthreads();  // LDS is reused by the next item
  }
}

struct SymFinishArgs {
  const double* u;
  const double* rowpart;
  const double* colpart;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  int32_t M;
  int T, b, nCB;
  double lam1, lam2;
  double* out;
};

__global__ __launch_bounds__(256) void finish_sym_kernel(SymFinishArgs a) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.M) return;
  const int32_t M = a.M;
  const int X = k / kT, t = k % kT;
  double s1 = 0.0, s2 = 0.0;
  for (int cb = X / a.b; cb < a.nCB; ++cb) {
    const double* rp = a.rowpart + ((size_t)cb * a.T + X) * (2 * kT);
    s1 += rp[t];
    s2 += rp[kT + t];
  }
  for (int rb = 0; rb <= X / kRows; ++rb) {
    const double* cp = a.colpart + ((size_t)rb * a.T + X) * (2 * kT);
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
  a.out[k] = o1;
  a.out[M + k] = o2;
}

}  // namespace

SymPlan make_sym_plan(int32_t M, size_t max_scratch_bytes) {
  SymPlan pl;
  pl.T = (M + kT - 1) / kT;
  pl.nRB = (pl.T + kRows - 1) / kRows;
  // column block length: enough items to fill the device several times over
  int b = 4;
  while (b < 64) {
    const int64_t nCB = (pl.T + b - 1) / b;
    const int64_t items = (int64_t)pl.nRB * nCB / 2;
    if (items <= 8192) break;
    b *= 2;
  }
  pl.b = b;
  pl.nCB = (pl.T + b - 1) / b;
  pl.scratch_doubles = ((size_t)pl.nRB + pl.nCB) * pl.T * 2 * kT;
  pl.enabled = pl.T >= 2 && pl.scratch_doubles * 8 <= max_scratch_bytes;
  return pl;
}

void sym_items(const SymPlan& pl, std::vector<int32_t>* items) {
  struct It {
    int rb, cb, pairs;
  };
  std::vector<It> v;
  for (int rb = 0; rb < pl.nRB; ++rb)
    for (int cb = (rb * kRows) / pl.b; cb < pl.nCB; ++cb) {
      int pairs = 0;
      for (int I = rb * kRows; I < std::min(rb * kRows + kRows, pl.T); ++I)
        for (int J = cb * pl.b; J < std::min(cb * pl.b + pl.b, pl.T); ++J) pairs += I <= J;
      if (pairs > 0) v.push_back({rb, cb, pairs});
    }
  // larger items first (they are dispatched first), ties in index order
  std::stable_sort(v.begin(), v.end(), [](const It& x, const It& y) { return x.pairs > y.pairs; });
  items->clear();
  for (const It& it : v) {
    items->push_back(it.rb);
    items->push_back(it.cb);
  }
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
  a.u = u;
  a.crow = P.crow;
  a.ccol = P.ccol;
  a.careful = careful;
  a.items = reinterpret_cast<const int2*>(items);
  a.M = P.M;
  a.T = pl.T;
  a.b = pl.b;
  a.c1 = P.eps_out / P.eps_in;
  a.c2 = P.eps_in / P.eps_out;
  a.kappa = P.kappa;
  a.scale = P.h * P.h * P.h / (4.0 * kPiD);
  a.rowpart = scratch;
  a.colpart = scratch + (size_t)pl.nCB * pl.T * 2 * kT;
  return a;
}

hipError_t launch_pair_sym(const SymArgs& a, int n_items, hipStream_t stream) {
  hipLaunchKernelGGL(pair_sym_fp64_kernel, dim3((unsigned)n_items), dim3(256), 0, stream, a);
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

hipError_t launch_finish_sym(const DeviceProblem& P, const SymPlan& pl, const double* u,
                             const double* scratch, double* out, hipStream_t stream) {
  SymFinishArgs f;
  f.u = u;
  f.rowpart = scratch;
  f.colpart = scratch + (size_t)pl.nCB * pl.T * 2 * kT;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
  f.M = P.M;
  f.T = pl.T;
  f.b = pl.b;
  f.nCB = pl.nCB;
  f.lam1 = P.lam1;
  f.lam2 = P.lam2;
  f.out = out;
  const unsigned blocks = (unsigned)((P.M + 255) / 256);
  hipLaunchKernelGGL(finish_sym_kernel, dim3(blocks), dim3(256), 0, stream, f);
  return hipGetLastError();
}

}  // namespace ibim
