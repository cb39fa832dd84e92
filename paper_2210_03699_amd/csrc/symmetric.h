// Symmetric (both directions per evaluation) float64 pair sum.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "operator.h"
#include "pair_math.h"

namespace ibim {

// Largest row-and-column scratch of the symmetric kernel (an eighth of the
// 288 GB of HBM; it grows as M^2 / rows, and with the row tiles per item of
// make_sym_plan this covers M ~ 6.5e6).
// Larger problems, and setups where the allocation fails, use the
// one-directional kernel, whose scratch grows only linearly.
constexpr size_t kSymScratchMax = size_t(32) << 30;
// Largest kappa R the float64 symmetric kernel's table exponential accepts
// (2^{-kappa R log2 e} must stay a normal number); problems whose largest
// pair distance (the diagonal of their nodes' bounding box) times kappa is
// larger use the one-directional float64 kernel.
constexpr double kSymMaxKappaR = 708.0;
// The symmetric kernels evaluate pairs in units of the Debye length 1/kappa
// when kappa is large enough for those units to stay in range; otherwise
// kappa enters every pair.  float64: kappa above 1e-30 (below it R^-3 in
// those units could overflow).  float32 (mixed form): kappa h at least 1e-6,
// so that kappa^2 w u and (kappa R)^-3 stay far inside the float32 range.
__host__ __device__ inline bool sym_debye_units(double kappa) { return kappa > 1e-30; }
__host__ __device__ inline bool sym_debye_units_f32(double kappa, double h) {
  return kappa * h >= 1e-6;
}

// Column-sum slot of (row block rb, column tile J), rb <= J / rows, for row
// blocks of `rows` tiles: the slots of tile J follow those of tiles 0 .. J-1
// (a packed lower triangle).
__host__ __device__ inline size_t sym_col_slot(int rb, int J, int rows) {
  const size_t q = (size_t)(J / rows), r = (size_t)(J % rows);
  return (size_t)rows * q * (q + 1) / 2 + r * (q + 1) + (size_t)rb;
}

// Row-sum slot of (column block cb, row tile X), cb >= X / b, for column
// blocks of b tiles: the slots of tile X follow those of tiles 0 .. X-1,
// which hold nCB - floor(X'/b) slots each (a packed upper triangle).
__host__ __device__ inline size_t sym_row_slot(int cb, int X, int b, int nCB) {
  const int64_t q = X / b, r = X % b;
  const int64_t before = (int64_t)X * nCB - (b * q * (q - 1) / 2 + q * r);
  return (size_t)(before + (cb - q));
}
// Row-sum slots of all T tiles.
__host__ __device__ inline size_t sym_row_slots_total(int T, int b, int nCB) {
  const int64_t q = T / b, r = T % b;
  return (size_t)((int64_t)T * nCB - (b * q * (q - 1) / 2 + q * r));
}

// Decomposition of the upper triangle of tile pairs into work items.
struct SymPlan {
  bool enabled = false;
  int T = 0;    // tiles of 256 nodes
  int b = 0;     // column tiles per item
  int rows = 0;  // row tiles per item (1 to 64, see make_sym_plan)
  int nRB = 0;   // row blocks (`rows` tiles each)
  int nCB = 0;  // column blocks
  size_t scratch_doubles = 0;  // row sums (sym_row_slots_total) + column sums (sym_col_slot(0, T, rows)), 512 doubles each
};

struct SymArgs {
  const double *px, *py, *pz, *nx, *ny, *nz, *w;
  const float *fx, *fy, *fz, *fnx, *fny, *fnz;  // float32 geometry (mixed form)
  const double* u;
  const int32_t* crow;
  const int32_t* ccol;
  const uint32_t* careful;  // bit I*T + J: tile pair (I, J) holds a pair of N_k (either way)
  const int2* items;        // (row block, column block) in launch order (sym_items)
  int32_t M;
  int T;
  int b;
  int rows;  // row tiles per item
  int unit32;  // the mixed kernel works in Debye units (sym_debye_units_f32)
  double c1, c2, kappa;
  double scale;       // h^3 / (4 pi)
  double* rowpart;    // [sym_row_slot(cb, I, b, nCB)][2][256]
  double* colpart;    // [sym_col_slot(rb, J, rows)][2][256]
};

// Plan for M nodes; disabled when the scratch would exceed max_scratch_bytes
// (the one-directional kernel is used then).
SymPlan make_sym_plan(int32_t M, size_t max_scratch_bytes);
// Work items as (rb, cb) pairs in launch order: the costliest first (those
// holding tile pairs of the careful bit matrix, see sym_careful_bits, or of
// the ragged last tile), then the plain ones arranged so that the items an
// XCD runs at once (item i runs on XCD i mod 8) share row and column tiles.
void sym_items(const SymPlan& pl, const std::vector<uint32_t>& careful, bool ragged,
               std::vector<int32_t>* items);
// Bit matrix of tile pairs that need the exclusion-aware evaluation.
void sym_careful_bits(int T, const std::vector<int32_t>& xrow, const std::vector<int32_t>& xtile,
                      std::vector<uint32_t>* bits);

// Arguments for problem P with input u; scratch holds plan.scratch_doubles.
SymArgs make_sym_args(const DeviceProblem& P, const SymPlan& pl, const int32_t* items,
                      const uint32_t* careful, const double* u, double* scratch);
hipError_t launch_pair_sym(const SymArgs& a, int n_items, hipStream_t stream);
// One persistent launch over several problems: work holds (problem, item) int32 pairs.
hipError_t launch_pair_sym_batched(const SymArgs* probs, const int32_t* work, int n_work,
                                   int* counter, int grid, hipStream_t stream);
int pair_sym_batched_grid();
hipError_t launch_finish_sym(const DeviceProblem& P, const SymPlan& pl, const double* u,
                             const double* scratch, double* out, hipStream_t stream);

// Finishing kernels' arguments (one problem); blk0 is the problem's first
// block in a batched finishing launch.
struct SymFinishArgs {
  const double* u;
  const double* rowpart;
  const double* colpart;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  int32_t M;
  int T, b, nCB, rows;
  double lam1, lam2;
  double* out;
  int64_t blk0;
};
SymFinishArgs make_finish_sym_args(const DeviceProblem& P, const SymPlan& pl, const double* u,
                                   const double* scratch, double* out);
// One launch finishing many problems (the solve server): args is a pinned
// host array of count entries (blk0 filled here), d_args a device array it
// is copied to on the stream.  Each problem's out is what launch_finish_sym
// writes, divided by lambda1 (psi rows) and lambda2 (psi_n rows) when
// unscale is set, as the row scaling of the scaled system does.
hipError_t launch_finish_sym_batched(SymFinishArgs* args, int count, SymFinishArgs* d_args,
                                     bool unscale, hipStream_t stream);

// Mixed form (float32 pairs, float64 sums) on the same schedule, and its
// finishing kernel, which also replaces the float32 value of every near pair
// by its float64 value (recomputing the float32 value exactly as the pair
// kernel produced it: forward, reverse or one-directional evaluation).
hipError_t launch_pair_sym_mixed(const SymArgs& a, int n_items, hipStream_t stream);
hipError_t launch_pair_sym_mixed_batched(const SymArgs* probs, const int32_t* work, int n_work,
                                         int* counter, int grid, hipStream_t stream);
int pair_sym_mixed_batched_grid();
hipError_t launch_finish_sym_mixed(const DeviceProblem& P, const SymPlan& pl,
                                   const uint32_t* careful, const double* u,
                                   const double* scratch, double* out, hipStream_t stream);

struct SymMixedFinishArgs {
  const double* u;
  const double* rowpart;
  const double* colpart;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  const int64_t* nrow;
  const int32_t* ncol;
  const double *px, *py, *pz, *nx, *ny, *nz, *w;
  const float *fx, *fy, *fz, *fnx, *fny, *fnz;
  const uint32_t* careful;
  PairConsts c64;  // float64 constants (the float32 ones are derived from them)
  int unit32;      // as SymArgs::unit32: the float32 values are in Debye units
  double scale;
  int32_t M;
  int T, b, nCB, rows;
  double lam1, lam2;
  double* out;
  int64_t blk0;
};
SymMixedFinishArgs make_finish_sym_mixed_args(const DeviceProblem& P, const SymPlan& pl,
                                              const uint32_t* careful, const double* u,
                                              const double* scratch, double* out);
// As launch_finish_sym_batched, for the mixed form.
hipError_t launch_finish_sym_mixed_batched(SymMixedFinishArgs* args, int count,
                                           SymMixedFinishArgs* d_args, bool unscale,
                                           hipStream_t stream);

}  // namespace ibim
