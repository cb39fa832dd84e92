// Device side of the treecode summation (plan in tree.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "operator.h"
#include "tree.h"

namespace ibim {

// Device copy of a TreePlan plus the per-application buffers.
struct TreeDevice {
  int32_t M = 0;
  int n_batches = 0, n_slots = 0, order = 0;
  int32_t *perm = nullptr, *pos = nullptr;
  int32_t* bstart = nullptr;
  int32_t *dstart = nullptr, *dend = nullptr, *kid = nullptr, *mlist = nullptr;
  std::vector<int32_t> mlevel;  // host: clusters of height h are mlist[mlevel[h] .. mlevel[h + 1])
  int32_t* fcol = nullptr;  // proxy clusters of the work items' far entries
  int32_t *nlo = nullptr, *nhi = nullptr;  // direct source ranges
  int32_t *xrow = nullptr, *xcol = nullptr;
  int32_t *ibatch = nullptr, *ifar0 = nullptr, *ifar1 = nullptr, *inear0 = nullptr,
          *inear1 = nullptr, *istart = nullptr, *iorder = nullptr;
  // two-way pairs (TreePlan::prow, pcol, pown, inrow, incol)
  int32_t *prow = nullptr, *pcol = nullptr, *pown = nullptr, *inrow = nullptr, *incol = nullptr;
  int n_items = 0, n_pairs = 0;
  bool mixed = false;      // target-proxy evaluations in float32 (IBIM_MIXED)
  double rnear = 0.0;      // mixed form: direct pairs nearer than this stay float64
  double* pbox = nullptr;  // 6 per proxy cluster: lo x, y, z, hi x, y, z
  double* cheb = nullptr;  // Chebyshev points on [-1, 1], barycentric weights, D (order^2)
  // geometry in tree order
  double *tx = nullptr, *ty = nullptr, *tz = nullptr;
  double *tnx = nullptr, *tny = nullptr, *tnz = nullptr, *tw = nullptr;
  // per application
  double *ta1 = nullptr, *ta2 = nullptr;  // w u1, w u2 in tree order
  double* pq = nullptr;                   // proxy charges (Q1, Q2) per point
  double* S = nullptr;                    // per work item: 2 x 256 partial sums
  double *rowS = nullptr, *colS = nullptr;  // per two-way pair: 2 x 256 row, column sums
  size_t bytes = 0;

  void release();
};

// Uploads the plan (and the tree-order geometry of P) to the device.
hipError_t tree_upload(const TreePlan& pl, const DeviceProblem& P, const double* host_px,
                       const double* host_py, const double* host_pz, const double* host_nx,
                       const double* host_ny, const double* host_nz, const double* host_w,
                       TreeDevice* T, hipStream_t s);
// Pair sum (gather, proxy charges, batches) into T.S.
hipError_t launch_tree_sum(const TreeDevice& T, const DeviceProblem& P, const double* u,
                           hipStream_t s);
// out = Lambda u + h^3/(4 pi) S (back in node order) + corrections.
hipError_t launch_tree_finish(const TreeDevice& T, const DeviceProblem& P, const double* u,
                              double* out, hipStream_t s);

}  // namespace ibim
