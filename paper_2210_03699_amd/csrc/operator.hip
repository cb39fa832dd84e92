// Dense pair sum and sparse correction of the discrete CTR-IBIM operator.
//
// Row k of eq. (corr-trapz-rule-sys1/2):
//   (A u)_1k = lambda1 u1_k + h^3 sum_{m not in N_k} [K11 a1_m - K12 a2_m]
//            + sum_{m in N_k} [h^2 w11 a1_m - h^3 w12 a2_m]
//   (A u)_2k = lambda2 u2_k + h^3 sum_{m not in N_k} [K21 a1_m - K22 a2_m]
//            + sum_{m in N_k} [h^2 w21 a1_m - h^2 w22 a2_m],   a = w u,
// with the kernels of eq. (Kij-kernels) at x = P(y_k), y = P(y_m).
//
// The pair sum is the hot loop (M^2 pairs, exp and rsqrt per pair, not a
// dense contraction, so it runs on the vector ALUs).  Targets are tiled one
// per thread; source tiles are staged in LDS as 64-byte records
// (P, n, a1, a2) and read back as wavefront-uniform broadcasts.  Sources are
// split into chunks across workgroups for small problems; the chunk partial
// sums are reduced in a fixed order by the finishing kernel, so results do
// not depend on scheduling.  The pairs of N_k are skipped exactly: source
// tiles that hold a corrected pair of the target tile (a few percent) run a
// loop in which each thread walks its row's sorted correction list; all other
// tiles run a loop without any test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "operator.h"
#include "pair_math.h"
#include "weights.h"

namespace ibim {
namespace {

constexpr int kThreads = kPairThreads;
constexpr int kTile = kPairTile;
constexpr int kXcd = kXcdCount;

// One work item: target tile `tile`, source chunk `split`.  src: LDS tile,
// per source (px,py) (pz,nx) (ny,nz) (a1,a2).
__device__ inline void pair_chunk_fp64(const PairArgs& a, int split, int tile, double2* src) {
  const int tid = threadIdx.x;
  const int32_t M = a.M;
  const int32_t k = tile * kThreads + tid;
  const int32_t kc = k < M ? k : M - 1;
  const double tx = a.px[kc], ty = a.py[kc], tz = a.pz[kc];
  const double tnx = a.nx[kc], tny = a.ny[kc], tnz = a.nz[kc];
  const int32_t s_begin = split * a.chunk_tiles * kTile;
  const int32_t s_end = min(M, s_begin + a.chunk_tiles * kTile);

  // next excluded source of this row (correction list is sorted by column)
  int32_t p = a.crow[kc];
  const int32_t pe = a.crow[kc + 1];
  while (p < pe && a.ccol[p] < s_begin) ++p;
  int32_t nxt = p < pe ? a.ccol[p] : INT_MAX;
  // next source tile that holds an excluded pair of this target tile (uniform)
  int32_t xp = a.xrow[tile];
  const int32_t xe = a.xrow[tile + 1];
  while (xp < xe && a.xtile[xp] * kTile < s_begin) ++xp;

  const PairConsts pc{a.c1, a.c2, a.kappa, a.kappa * a.kappa};
  double S1 = 0.0, S2 = 0.0;
  for (int32_t s0 = s_begin; s0 < s_end; s0 += kTile) {
    const int32_t m = s0 + tid;
    if (m < s_end) {
      const double wm = a.w[m];
      src[4 * tid + 0] = make_double2(a.px[m], a.py[m]);
      src[4 * tid + 1] = make_double2(a.pz[m], a.nx[m]);
      src[4 * tid + 2] = make_double2(a.ny[m], a.nz[m]);
      src[4 * tid + 3] = make_double2(wm * a.u[m], wm * a.u[M + m]);
    }
    __syncthreads();
    const int n = min(kTile, s_end - s0);
    const bool careful = xp < xe && a.xtile[xp] * kTile == s0;
    if (!careful) {
      // no corrected pair of this target tile among these sources
#pragma unroll 2
      for (int j = 0; j < n; ++j) {
        const double2 q0 = src[4 * j], q1 = src[4 * j + 1], q2 = src[4 * j + 2], q3 = src[4 * j + 3];
        pair_f64<true>(tx, ty, tz, tnx, tny, tnz, q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y,
                       pc, S1, S2);
      }
    } else {
      ++xp;
      for (int j = 0; j < n; ++j) {
        double d1, d2;
        const double2 q0 = src[4 * j], q1 = src[4 * j + 1], q2 = src[4 * j + 2], q3 = src[4 * j + 3];
        pair_f64<false>(tx, ty, tz, tnx, tny, tnz, q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y,
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
    __syncthreads();
  }
  if (k < M) {
    double* out = a.partial + (size_t)split * 2 * (size_t)M;
    out[k] = a.scale * S1;
    out[M + k] = a.scale * S2;
  }
}

__global__ __launch_bounds__(kThreads) void pair_fp64_kernel(PairArgs a) {
  __shared__ double2 src[kTile * 4];
  int split, tile;
  pair_block_to_work(blockIdx.x, a.nsplit, &split, &tile);
  pair_chunk_fp64(a, split, tile, src);
}

__global__ __launch_bounds__(kThreads) void pair_batched_fp64_kernel(
    const PairArgs* __restrict__ reqs, const int32_t* __restrict__ items, int n_items,
    int* counter) {
  __shared__ double2 src[kTile * 4];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // everyone has read `next` before it is overwritten
    if (it >= n_items) break;
    const PairArgs a = reqs[__builtin_amdgcn_readfirstlane(items[3 * it])];
    pair_chunk_fp64(a, __builtin_amdgcn_readfirstlane(items[3 * it + 2]),
                    __builtin_amdgcn_readfirstlane(items[3 * it + 1]), src);
  }
}

struct FinishArgs {
  const double* u;
  const double* partial;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  int32_t M;
  int nsplit;
  double lam1, lam2;
  double* out;
};

__global__ __launch_bounds__(256) void finish_kernel(FinishArgs a) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.M) return;
  const int32_t M = a.M;
  double s1 = 0.0, s2 = 0.0;
  for (int s = 0; s < a.nsplit; ++s) {
    const double* pp = a.partial + (size_t)s * 2 * (size_t)M;
    s1 += pp[k];
    s2 += pp[M + k];
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

void exclusion_tiles(int32_t M, const int64_t* crow, const int32_t* ccol,
                     std::vector<int32_t>* xrow, std::vector<int32_t>* xtile) {
  const int ntile = (M + kThreads - 1) / kThreads;
  std::vector<std::vector<int32_t>> lists(ntile);
  for (int32_t k = 0; k < M; ++k)
    for (int64_t e = crow[k]; e < crow[k + 1]; ++e) lists[k / kThreads].push_back(ccol[e] / kTile);
  xrow->assign(ntile + 1, 0);
  xtile->clear();
  for (int t = 0; t < ntile; ++t) {
    std::sort(lists[t].begin(), lists[t].end());
    lists[t].erase(std::unique(lists[t].begin(), lists[t].end()), lists[t].end());
    xtile->insert(xtile->end(), lists[t].begin(), lists[t].end());
    (*xrow)[t + 1] = (int32_t)xtile->size();
  }
}

PairPlan make_pair_plan(int32_t M, int precision) {
  (void)precision;
  PairPlan pl;
  pl.ntile = (M + kThreads - 1) / kThreads;
  const int src_tiles = (M + kTile - 1) / kTile;
  // aim for about 16384 workgroups so the tail of the grid is short
  int want = (16384 + pl.ntile - 1) / pl.ntile;
  want = ((want + kXcd - 1) / kXcd) * kXcd;
  const int max_split = src_tiles / 4 > 0 ? src_tiles / 4 : 1;
  int ns = want < max_split ? want : max_split;
  if (ns < 1) ns = 1;
  pl.chunk_tiles = (src_tiles + ns - 1) / ns;
  pl.nsplit = (src_tiles + pl.chunk_tiles - 1) / pl.chunk_tiles;
  return pl;
}

PairArgs make_pair_args(const DeviceProblem& P, const PairPlan& plan, const double* u,
                        double* partial) {
  PairArgs a{};
  a.px = P.px; a.py = P.py; a.pz = P.pz;
  a.nx = P.nx; a.ny = P.ny; a.nz = P.nz;
  a.w = P.w;
  a.fx = P.px32; a.fy = P.py32; a.fz = P.pz32;
  a.fnx = P.nx32; a.fny = P.ny32; a.fnz = P.nz32;
  a.u = u;
  a.crow = P.crow;
  a.ccol = P.ccol;
  a.xrow = P.xrow;
  a.xtile = P.xtile;
  a.M = P.M;
  a.nsplit = plan.nsplit;
  a.chunk_tiles = plan.chunk_tiles;
  a.c1 = P.eps_out / P.eps_in;
  a.c2 = P.eps_in / P.eps_out;
  a.kappa = P.kappa;
  a.scale = P.h * P.h * P.h / (4.0 * kPiD);
  a.partial = partial;
  return a;
}

hipError_t launch_pair(const DeviceProblem& P, const PairPlan& plan, int precision,
                       const double* u, double* partial, hipStream_t stream) {
  (void)precision;
  const PairArgs a = make_pair_args(P, plan, u, partial);
  const unsigned blocks = (unsigned)plan.ntile * (unsigned)plan.nsplit;
  hipLaunchKernelGGL(pair_fp64_kernel, dim3(blocks), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_pair_batched_fp64(const PairArgs* reqs, const int32_t* items, int n_items,
                                    int* counter, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(pair_batched_fp64_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                     reqs, items, n_items, counter);
  return hipGetLastError();
}

int pair_batched_grid_fp64() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_fp64_kernel, kThreads, 0) !=
          hipSuccess || per < 1)
    per = 1;
  return cus * per;
}

hipError_t launch_pair_batched_mixed(const PairArgs* reqs, const int32_t* items, int n_items,
                                     int* counter, int grid, hipStream_t stream);
int pair_batched_grid_mixed();

hipError_t launch_pair_batched(int precision, const PairArgs* reqs, const int32_t* items,
                               int n_items, int* counter, int grid, hipStream_t stream) {
  if (precision == 1)
    return launch_pair_batched_mixed(reqs, items, n_items, counter, grid, stream);
  return launch_pair_batched_fp64(reqs, items, n_items, counter, grid, stream);
}

int pair_batched_grid(int precision) {
  return precision == 1 ? pair_batched_grid_mixed() : pair_batched_grid_fp64();
}

hipError_t launch_finish(const DeviceProblem& P, const PairPlan& plan, int precision,
                         const double* u, const double* partial, double* out, hipStream_t stream) {
  (void)precision;
  FinishArgs f;
  f.u = u;
  f.partial = partial;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
  f.M = P.M;
  f.nsplit = plan.nsplit;
  f.lam1 = P.lam1;
  f.lam2 = P.lam2;
  f.out = out;
  const unsigned blocks = (unsigned)((P.M + 255) / 256);
  hipLaunchKernelGGL(finish_kernel, dim3(blocks), dim3(256), 0, stream, f);
  return hipGetLastError();
}

}  // namespace ibim
