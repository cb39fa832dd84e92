// Treecode summation of the dense pair sum (the far-field acceleration the
// paper obtains with a black-box fast multipole method, Section 2.5): the
// sources of a well-separated cluster are replaced by charges at the tensor
// Chebyshev points of its bounding box, obtained by interpolating the kernels
// in the source variable (the interpolation bbFMM uses for its multipole
// expansions); near clusters are summed directly with the pairs of N_k
// skipped.  Host planning here, device kernels in treecode.hip.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ibim {

constexpr int kTreeBatch = 256;  // targets per batch (one workgroup)
constexpr int kTreeMaxOrder = 16;

struct TreeParams {
  int order = 8;        // Chebyshev points per dimension (degree order - 1)
  double theta = 0.7;   // separation: (r_batch + r_cluster) < theta * distance
};

// Everything the device needs, in "tree order" (nodes permuted so that every
// cluster and every batch is a contiguous range).
struct TreePlan {
  bool enabled = false;
  int order = 0;
  int32_t M = 0;
  std::vector<int32_t> perm;  // tree position -> node
  std::vector<int32_t> pos;   // node -> tree position
  // batches: target ranges [bstart[b], bstart[b + 1])
  std::vector<int32_t> bstart;
  std::vector<int32_t> border;  // batch indices, most work first
  // clusters with proxies: source range, bounding box (lo x, y, z, hi x, y, z)
  std::vector<int32_t> pstart, pend;
  std::vector<double> pbox;
  // per batch: proxy clusters (far) and merged source ranges (near), CSR
  std::vector<int32_t> frow, fcol;
  std::vector<int32_t> nrow, nlo, nhi;
  // N_k in tree positions, ascending, per tree position (CSR)
  std::vector<int32_t> xrow, xcol;
  double gap = 0.0;         // largest |x_k - P_m| over m in N_k
  double far_evals = 0.0;   // target-proxy evaluations per application
  double near_evals = 0.0;  // direct pair evaluations per application
  double proxy_evals = 0.0; // source-proxy terms of the upward pass
};

// Builds the plan from the projected points, the correction sets (CSR with
// 64-bit row pointers, columns ascending) and the grid spacing.
int build_tree_plan(const TreeParams& prm, int64_t M, const double* px, const double* py,
                    const double* pz, const int64_t* crow, const int32_t* ccol, double h,
                    TreePlan* plan, std::string* err);

}  // namespace ibim
