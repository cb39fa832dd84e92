// Device operator A = Lambda + h^3 K W + h^2 Omega W (eq. linear-system).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ibim {

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
  int32_t* nrow = nullptr;
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

}  // namespace ibim
