// Device operator A = Lambda + h^3 K W + h^2 Omega W (eq. linear-system).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ibim {

constexpr int kPairThreads = 256;  // targets per workgroup of the pair kernels (one per lane)
constexpr int kPairTile = 256;     // sources staged per LDS tile
constexpr int kXcdCount = 8;       // MI355X: workgroup b runs on XCD b % 8

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  When
// nsplit is a multiple of 8, XCD x gets the source chunks
// [x*nsplit/8, (x+1)*nsplit/8) of every target tile, so each L2 holds only
// one eighth of the sources; otherwise chunk b % nsplit of tile b / nsplit.
__device__ inline void pair_block_to_work(int b, int nsplit, int* split, int* tile) {
  if (nsplit % kXcdCount == 0) {
    const int x = b % kXcdCount, j = b / kXcdCount, per = nsplit / kXcdCount;
    *split = x * per + j % per;
    *tile = j / per;
  } else {
    *split = b % nsplit;
    *tile = b / nsplit;
  }
}

// Geometry and correction structure resident on the device for one problem.
struct DeviceProblem {
  int32_t M = 0;
  int64_t nnz = 0;
  // node data, structure of arrays (targets and sources are the same nodes)
  double* px = nullptr;
  double* py = nullptr;
  double* pz = nullptr;
  double* nx = nullptr;
  double* ny = nullptr;
  double* nz = nullptr;
  double* w = nullptr;
  // float32 copies for the mixed-precision pair kernel (positions relative
  // to the centroid)
  float* px32 = nullptr;
  float* py32 = nullptr;
  float* pz32 = nullptr;
  float* nx32 = nullptr;
  float* ny32 = nullptr;
  float* nz32 = nullptr;
  double centre[3] = {0, 0, 0};
  // corrections: CSR sorted by column, 2x2 blocks (h powers and w folded in)
  int32_t* crow = nullptr;  // M+1 (nnz < 2^31)
  int32_t* ccol = nullptr;  // nnz
  double* blocks = nullptr; // 4*nnz
  // per target tile, the sorted source tiles that hold one of its corrected pairs
  int32_t* xrow = nullptr;
  int32_t* xtile = nullptr;
  // near list of the mixed path: CSR of (row, col) pairs with R < r_near
  // (float64 distance), pairs of N_k excluded
  int64_t* nrow = nullptr;
  int32_t* ncol = nullptr;
  int64_t nnear = 0;
  double eps_in = 1, eps_out = 1, kappa = 0, h = 0;
  double lam1 = 0, lam2 = 0;
};

// Launch plan of the dense pair sum (targets tiled, sources split).
struct PairPlan {
  int ntile = 0;        // target tiles
  int nsplit = 1;       // source chunks (each a whole number of source tiles)
  int chunk_tiles = 0;  // source tiles per chunk
};

PairPlan make_pair_plan(int32_t M, int precision);

// Arguments of one problem's pair sum: workgroup (split, tile) sums the
// sources of chunk `split` for the targets of tile `tile`.
struct PairArgs {
  const double *px, *py, *pz, *nx, *ny, *nz, *w;  // float64 geometry
  const float *fx, *fy, *fz, *fnx, *fny, *fnz;     // float32 geometry (mixed form)
  const double* u;
  const int32_t* crow;
  const int32_t* ccol;
  const int32_t* xrow;   // per target tile: range in xtile
  const int32_t* xtile;  // sorted source tiles holding a corrected pair of the tile
  int32_t M;
  int nsplit;
  int chunk_tiles;
  double c1;     // eps_out / eps_in
  double c2;     // eps_in / eps_out
  double kappa;
  double scale;  // h^3 / (4 pi)
  double* partial;
};

PairArgs make_pair_args(const DeviceProblem& P, const PairPlan& plan, const double* u,
                        double* partial);

// One persistent launch over a work list of several problems: item i is
// (problem items[3i], target tile items[3i+1], source chunk items[3i+2]);
// workgroups take items from *counter (which must be 0) until the list is
// exhausted.  Each item is computed exactly as in the single-problem kernel.
hipError_t launch_pair_batched(int precision, const PairArgs* reqs, const int32_t* items,
                               int n_items, int* counter, int grid, hipStream_t stream);

// Workgroups of the persistent launch that fit on the device at once.
int pair_batched_grid(int precision);

// Host: per target tile, the sorted list of source tiles containing one of
// its corrected pairs (CSR: xrow has one entry per tile plus one).
void exclusion_tiles(int32_t M, const int64_t* crow, const int32_t* ccol,
                     std::vector<int32_t>* xrow, std::vector<int32_t>* xtile);

// partial: nsplit * 2M float64 scratch.  Writes partial sums of
// h^3 sum_m K(k, m) (w u)(m) over each source chunk, pairs in N_h(y_k) skipped.
hipError_t launch_pair(const DeviceProblem& P, const PairPlan& plan, int precision,
                       const double* u, double* partial, hipStream_t stream);

// out = Lambda u + sum_chunks partial + blocks * u (+ near-pair float64 fix-up
// for the mixed path).
hipError_t launch_finish(const DeviceProblem& P, const PairPlan& plan, int precision,
                         const double* u, const double* partial, double* out, hipStream_t stream);

// Mixed-precision pair sum (float32 pairs, float64 sums) and its finishing
// kernel (adds float64 minus float32 values of the near pairs).
hipError_t launch_pair_mixed(const DeviceProblem& P, const PairPlan& plan, const double* u,
                             double* partial, hipStream_t stream);
hipError_t launch_finish_mixed(const DeviceProblem& P, const PairPlan& plan, const double* u,
                               const double* partial, double* out, hipStream_t stream);

// Builds P.nrow / P.ncol: for every node, the nodes m not in N_k with
// |P_k - P_m| < r_near, found by scanning grid offsets within
// (r_near + 2 eps)/h.  node_of: device grid -> node map (-1 off the tube);
// grid_index: device node -> linear grid index.  Synchronises the stream.
hipError_t build_near_list(DeviceProblem& P, const int32_t* node_of, const int64_t* grid_index,
                           int nx, int ny, int nz, double r_near, double eps,
                           hipStream_t stream);

}  // namespace ibim
