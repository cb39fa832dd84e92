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
constexpr int kTreeMaxOrder = 12;

struct TreeParams {
  int order = 8;        // Chebyshev points per dimension (degree order - 1)
  double theta = 0.7;   // separation: (r_batch + r_cluster) < theta * distance
  // cost of one target-proxy evaluation in direct pairs: a separated
  // cluster is summed through its order^3 proxies when it holds more than
  // proxy_cost * order^3 nodes (kTreeProxyCost64 or kTreeProxyCost32)
  double proxy_cost = 0.44;
  // near pairs of leaves evaluated once for both directions
  bool two_way = true;
};
// Measured VALU instructions of a target-proxy evaluation over those of a
// direct pair (N_k skip included): float64 33 / 75, the mixed form (float32
// proxies and direct pairs on float64-formed differences) 16 / 62.
constexpr double kTreeProxyCost64 = 0.44;
constexpr double kTreeProxyCost32 = 0.26;

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
  // clusters with proxies (every cluster of more than proxy_cost * order^3
  // nodes, in tree preorder): source range, bounding box (lo x, y, z, hi x,
  // y, z)
  std::vector<int32_t> pstart, pend;
  std::vector<double> pbox;
  // charges of a proxy cluster: from the sources of [dstart, dend) directly
  // (its children without proxies, or itself when it is a leaf) plus, by
  // exact interpolation of their proxies, from its children with proxies
  // (kid, 2 per cluster, -1 if none); mlist orders the clusters by height
  // above the leaves, mlevel[h] .. mlevel[h + 1] being height h
  std::vector<int32_t> dstart, dend, kid;
  std::vector<int32_t> mlist, mlevel;
  // per batch: proxy clusters (far) and merged source ranges (near,
  // summed one direction at a time), CSR
  std::vector<int32_t> frow, fcol;
  std::vector<int32_t> nrow, nlo, nhi;
  // two-way pairs of leaves (two_way plans): batches b < b' that are near
  // each other both ways and hold no pair of N_k either way.  Pair q (batch
  // b = pown[q]'s list prow[b] .. prow[b + 1], ascending b' = pcol[q]) is
  // evaluated once for both directions; its row sums (for b) and column sums
  // (for b') go to slot q, and batch b' finds its slots in incol[inrow[b'] ..
  // inrow[b' + 1]] (ascending)
  std::vector<int32_t> prow, pcol, pown, inrow, incol;
  // work items: a batch's lists cut into parts of similar work, so that the
  // device has many more workgroups than compute units; item i covers the
  // far entries [ifar0, ifar1) and near ranges [inear0, inear1) of batch
  // ibatch[i]; the items of batch b are istart[b] .. istart[b + 1]; iorder
  // lists them most work first
  std::vector<int32_t> ibatch, ifar0, ifar1, inear0, inear1, istart, iorder;
  // N_k in tree positions, ascending, per tree position (CSR)
  std::vector<int32_t> xrow, xcol;
  double gap = 0.0;         // largest |x_k - P_m| over m in N_k
  double far_evals = 0.0;   // target-proxy evaluations per application
  double near_evals = 0.0;  // direct pair evaluations per application (ordered pairs)
  double proxy_evals = 0.0; // source-proxy terms of the direct proxy charges
  double m2m_links = 0.0;   // child-to-parent proxy transfers
};

// Builds the plan from the projected points, the correction sets (CSR with
// 64-bit row pointers, columns ascending) and the grid spacing.
int build_tree_plan(const TreeParams& prm, int64_t M, const double* px, const double* py,
                    const double* pz, const int64_t* crow, const int32_t* ccol, double h,
                    TreePlan* plan, std::string* err);

// Device bytes that uploading the plan allocates (index arrays, permuted
// geometry, Chebyshev tables, proxy charges and per-item partial sums).
size_t tree_device_bytes(const TreePlan& plan);

}  // namespace ibim
