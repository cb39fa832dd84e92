// Mixed-precision form of the dense pair sum.
//
// Every pair is evaluated in float32 from float32 geometry (positions taken
// relative to the node centroid) and float32 amplitudes a = (float)(w u);
// each contribution is converted to float64 and summed in float64.  Pairs
// closer than r_near (float64 distance; the near list) are then corrected
// in the finishing kernel by adding (float64 value - float32 value), the
// float32 value recomputed by the same device function from the same float32
// inputs.  This translation unit is compiled without automatic contraction
// and the float32 function spells out every fused multiply-add, so the two
// float32 evaluations agree bit for bit and the near pairs end up exactly at
// their float64 values (up to the rounding of the float64 sums).  The
// correction weights, the sparse correction and the Krylov solver stay
// float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <vector>

#include "device_mem.h"
#include "operator.h"
#include "pair_math.h"
#include "weights.h"

namespace ibim {
namespace {

constexpr int kThreads = kPairThreads;
constexpr int kTile = kPairTile;

// One work item of the mixed form; src: LDS tile, per source
// (px,py,pz,nx) (ny,nz,a1,a2) in float32.
__device__ inline void pair_chunk_mixed(const PairArgs& a, int split, int tile, float4* src) {
  const int tid = threadIdx.x;
  const int32_t M = a.M;
  const int32_t k = tile * kThreads + tid;
  const int32_t kc = k < M ? k : M - 1;
  const float tx = a.fx[kc], ty = a.fy[kc], tz = a.fz[kc];
  const float tnx = a.fnx[kc], tny = a.fny[kc], tnz = a.fnz[kc];
  const int32_t s_begin = split * a.chunk_tiles * kTile;
  const int32_t s_end = min(M, s_begin + a.chunk_tiles * kTile);

  int32_t p = a.crow[kc];
  const int32_t pe = a.crow[kc + 1];
  while (p < pe && a.ccol[p] < s_begin) ++p;
  int32_t nxt = p < pe ? a.ccol[p] : INT_MAX;
  int32_t xp = a.xrow[tile];
  const int32_t xe = a.xrow[tile + 1];
  while (xp < xe && a.xtile[xp] * kTile < s_begin) ++xp;

  const PairConstsF c{(float)a.c1, (float)a.c2, (float)a.kappa, (float)(a.kappa * a.kappa)};
  double S1 = 0.0, S2 = 0.0;
  for (int32_t s0 = s_begin; s0 < s_end; s0 += kTile) {
    const int32_t m = s0 + tid;
    if (m < s_end) {
      const double wm = a.w[m];
      src[2 * tid + 0] = make_float4(a.fx[m], a.fy[m], a.fz[m], a.fnx[m]);
      src[2 * tid + 1] = make_float4(a.fny[m], a.fnz[m], (float)(wm * a.u[m]),
                                     (float)(wm * a.u[M + m]));
    }
    __syncthreads();
    const int n = min(kTile, s_end - s0);
    const bool careful = xp < xe && a.xtile[xp] * kTile == s0;
    if (!careful) {
#pragma unroll 2
      for (int j = 0; j < n; ++j) {
        const float4 q0 = src[2 * j], q1 = src[2 * j + 1];
        float d1, d2;
        pair_f32(tx, ty, tz, tnx, tny, tnz, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, c,
                 d1, d2);
        S1 += (double)d1;
        S2 += (double)d2;
      }
    } else {
      ++xp;
      for (int j = 0; j < n; ++j) {
        const float4 q0 = src[2 * j], q1 = src[2 * j + 1];
        float d1, d2;
        pair_f32(tx, ty, tz, tnx, tny, tnz, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, c,
                 d1, d2);
        const bool ex = (s0 + j == nxt);
        if (ex) {
          ++p;
          nxt = p < pe ? a.ccol[p] : INT_MAX;
        }
        S1 += ex ? 0.0 : (double)d1;
        S2 += ex ? 0.0 : (double)d2;
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

__global__ __launch_bounds__(kThreads) void pair_mixed_kernel(PairArgs a) {
  __shared__ float4 src[kTile * 2];
  int split, tile;
  pair_block_to_work(blockIdx.x, a.nsplit, &split, &tile);
  pair_chunk_mixed(a, split, tile, src);
}

__global__ __launch_bounds__(kThreads) void pair_batched_mixed_kernel(
    const PairArgs* __restrict__ reqs, const int32_t* __restrict__ items, int n_items,
    int* counter) {
  __shared__ float4 src[kTile * 2];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // everyone has read `next` before it is overwritten
    if (it >= n_items) break;
    const PairArgs a = reqs[__builtin_amdgcn_readfirstlane(items[3 * it])];
    pair_chunk_mixed(a, __builtin_amdgcn_readfirstlane(items[3 * it + 2]),
                     __builtin_amdgcn_readfirstlane(items[3 * it + 1]), src);
  }
}

struct FinishMixedArgs {
  const double* u;
  const double* partial;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  const int64_t* nrow;
  const int32_t* ncol;
  const double *px, *py, *pz, *nx, *ny, *nz, *w;
  const float *fx, *fy, *fz, *fnx, *fny, *fnz;
  PairConsts c64;
  PairConstsF c32;
  double scale;
  int32_t M;
  int nsplit;
  double lam1, lam2;
  double* out;
};

__global__ __launch_bounds__(256) void finish_mixed_kernel(FinishMixedArgs a) {
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
  // near pairs: replace the float32 value already summed by the float64 one
  const double x = a.px[k], y = a.py[k], z = a.pz[k];
  const double nxk = a.nx[k], nyk = a.ny[k], nzk = a.nz[k];
  const float fx = a.fx[k], fy = a.fy[k], fz = a.fz[k];
  const float fnx = a.fnx[k], fny = a.fny[k], fnz = a.fnz[k];
  double f1 = 0.0, f2 = 0.0;
  for (int64_t e = a.nrow[k]; e < a.nrow[k + 1]; ++e) {
    const int32_t m = a.ncol[e];
    const double wm = a.w[m];
    const double a1 = wm * a.u[m], a2 = wm * a.u[M + m];
    double d1, d2;
    pair_f64<false>(x, y, z, nxk, nyk, nzk, a.px[m], a.py[m], a.pz[m], a.nx[m], a.ny[m], a.nz[m],
                    a1, a2, a.c64, d1, d2);
    float e1, e2;
    pair_f32(fx, fy, fz, fnx, fny, fnz, a.fx[m], a.fy[m], a.fz[m], a.fnx[m], a.fny[m], a.fnz[m],
             (float)a1, (float)a2, a.c32, e1, e2);
    f1 += d1 - (double)e1;
    f2 += d2 - (double)e2;
  }
  a.out[k] = o1 + a.scale * f1;
  a.out[M + k] = o2 + a.scale * f2;
}

struct NearArgs {
  const double* px;
  const double* py;
  const double* pz;
  const int64_t* grid_index;
  const int32_t* node_of;
  const int32_t* crow;
  const int32_t* ccol;
  int nx, ny, nz;
  int W;
  double rn2;
  int32_t M;
  const int64_t* rowptr;  // fill pass only
  int32_t* count;         // count pass only
  int32_t* col;           // fill pass only
};

// One wavefront per row: nodes within the offset ball, closer than r_near in
// float64, not corrected by the row (fill == false counts, true writes).  The
// lanes take consecutive cells of the offset cube [-W, W]^3, clipped to the
// grid, in (di, dj, dl) order and a ballot compacts the hits, so each row's
// list is in cell order.
template <bool kFill>
__global__ __launch_bounds__(256) void near_kernel(NearArgs a) {
  const int lane = threadIdx.x & 63;
  const int32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= a.M) return;  // whole wavefronts
  const int64_t q = a.grid_index[k];
  const int i = (int)(q / ((int64_t)a.ny * a.nz));
  const int j = (int)((q / a.nz) % a.ny);
  const int l = (int)(q % a.nz);
  const double x = a.px[k], y = a.py[k], z = a.pz[k];
  const int32_t c0 = a.crow[k], c1 = a.crow[k + 1];
  int64_t out = kFill ? a.rowptr[k] : 0;
  int32_t cnt = 0;
  const int W = a.W;
  const int i0 = max(-W, -i), j0 = max(-W, -j), l0 = max(-W, -l);
  const int si = min(W, a.nx - 1 - i) - i0 + 1, sj = min(W, a.ny - 1 - j) - j0 + 1,
            sl = min(W, a.nz - 1 - l) - l0 + 1;
  const int ncell = si * sj * sl;  // below 2^31: the grid is (host check)
  // this lane's cell (ci, cj, cl) in the mixed radix (si, sj, sl), advanced by
  // 64 cells per step as the digits (ai, aj, al) with carries
  int cl = lane % sl, cj = (lane / sl) % sj, ci = lane / (sl * sj);
  const int al = 64 % sl, aj = (64 / sl) % sj, ai = 64 / (sl * sj);
  for (int base = 0; base < ncell; base += 64) {
    bool hit = false;
    int32_t m = -1;
    const int di = i0 + ci, dj = j0 + cj, dl = l0 + cl;
    if (base + lane < ncell && di * di + dj * dj + dl * dl <= W * W) {
      m = a.node_of[((int64_t)(i + di) * a.ny + (j + dj)) * a.nz + (l + dl)];
      if (m >= 0) {
        const double rx = x - a.px[m], ry = y - a.py[m], rz = z - a.pz[m];
        if (rx * rx + ry * ry + rz * rz < a.rn2) {
          bool corrected = false;
          for (int32_t e = c0; e < c1; ++e) corrected |= (a.ccol[e] == m);
          hit = !corrected;
        }
      }
    }
    cl += al;
    int carry = cl >= sl;
    cl -= carry ? sl : 0;
    cj += aj + carry;
    carry = cj >= sj;
    cj -= carry ? sj : 0;
    ci += ai + carry;
    const unsigned long long mask = __ballot(hit);
    if (kFill && hit) a.col[out + __popcll(mask & ((1ull << lane) - 1ull))] = m;
    out += __popcll(mask);
    cnt += __popcll(mask);
  }
  if (!kFill && lane == 0) a.count[k] = cnt;
}

}  // namespace

hipError_t launch_pair_mixed(const DeviceProblem& P, const PairPlan& plan, const double* u,
                             double* partial, hipStream_t stream) {
  const PairArgs a = make_pair_args(P, plan, u, partial);
  const unsigned blocks = (unsigned)plan.ntile * (unsigned)plan.nsplit;
  hipLaunchKernelGGL(pair_mixed_kernel, dim3(blocks), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_pair_batched_mixed(const PairArgs* reqs, const int32_t* items, int n_items,
                                     int* counter, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(pair_batched_mixed_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                     reqs, items, n_items, counter);
  return hipGetLastError();
}

int pair_batched_grid_mixed() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_mixed_kernel, kThreads, 0) !=
          hipSuccess || per < 1)
    per = 1;
  return cus * per;
}

hipError_t launch_finish_mixed(const DeviceProblem& P, const PairPlan& plan, const double* u,
                               const double* partial, double* out, hipStream_t stream) {
  FinishMixedArgs f;
  f.u = u;
  f.partial = partial;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
  f.nrow = P.nrow;
  f.ncol = P.ncol;
  f.px = P.px; f.py = P.py; f.pz = P.pz; f.nx = P.nx; f.ny = P.ny; f.nz = P.nz; f.w = P.w;
  f.fx = P.px32; f.fy = P.py32; f.fz = P.pz32; f.fnx = P.nx32; f.fny = P.ny32; f.fnz = P.nz32;
  f.c64 = PairConsts{P.eps_out / P.eps_in, P.eps_in / P.eps_out, P.kappa, P.kappa * P.kappa};
  f.c32 = PairConstsF{(float)(P.eps_out / P.eps_in), (float)(P.eps_in / P.eps_out),
                      (float)P.kappa, (float)(P.kappa * P.kappa)};
  f.scale = P.h * P.h * P.h / (4.0 * kPiD);
  f.M = P.M;
  f.nsplit = plan.nsplit;
  f.lam1 = P.lam1;
  f.lam2 = P.lam2;
  f.out = out;
  hipLaunchKernelGGL(finish_mixed_kernel, dim3((unsigned)((P.M + 255) / 256)), dim3(256), 0,
                     stream, f);
  return hipGetLastError();
}

hipError_t build_near_list(DeviceProblem& P, const int32_t* node_of, const int64_t* grid_index,
                           int nx, int ny, int nz, double r_near, double eps,
                           hipStream_t stream) {
  NearArgs a{};
  a.px = P.px; a.py = P.py; a.pz = P.pz;
  a.grid_index = grid_index;
  a.node_of = node_of;
  a.crow = P.crow;
  a.ccol = P.ccol;
  a.nx = nx; a.ny = ny; a.nz = nz;
  if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  // reach in cells, capped by the grid diagonal (every grid cell is within it)
  const double reach = std::ceil((r_near + 2.0 * eps) / P.h);
  const double diag = std::ceil(std::sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz));
  a.W = (int)std::min(reach, diag);
  a.rn2 = r_near * r_near;
  a.M = P.M;
  const unsigned blocks = (unsigned)((P.M + 3) / 4);  // four rows (wavefronts) per block
  int32_t* d_count = nullptr;
  hipError_t e = device_alloc((void**)&d_count, sizeof(int32_t) * (size_t)P.M);
  if (e != hipSuccess) return e;
  a.count = d_count;
  hipLaunchKernelGGL(near_kernel<false>, dim3(blocks), dim3(256), 0, stream, a);
  std::vector<int32_t> cnt(P.M);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt.data(), d_count, sizeof(int32_t) * (size_t)P.M, hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  device_free(d_count);
  if (e != hipSuccess) return e;
  std::vector<int64_t> rowptr(P.M + 1, 0);
  for (int32_t k = 0; k < P.M; ++k) rowptr[k + 1] = rowptr[k] + cnt[k];
  P.nnear = rowptr[P.M];
  e = device_alloc((void**)&P.nrow, sizeof(int64_t) * (size_t)(P.M + 1));
  if (e == hipSuccess)
    e = device_alloc((void**)&P.ncol, sizeof(int32_t) * (size_t)(P.nnear > 0 ? P.nnear : 1));
  if (e == hipSuccess)
    e = hipMemcpyAsync(P.nrow, rowptr.data(), sizeof(int64_t) * (size_t)(P.M + 1),
                       hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  a.rowptr = P.nrow;
  a.col = P.ncol;
  hipLaunchKernelGGL(near_kernel<true>, dim3(blocks), dim3(256), 0, stream, a);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

}  // namespace ibim
