// Host planning of the treecode: cluster tree, batches, interaction lists.
//
// The tree is a binary space partition of the projected points P(y_m): a
// cluster with more than one batch of points is split across its longest
// bounding-box side, the left part taking the nearest multiple of the batch
// size to half the points, so every leaf (a batch of targets) holds exactly
// kTreeBatch points except the last one.  A cluster C is approximated for a
// batch B by its proxies when evaluating them costs less than its points
// (more than proxy_cost * order^3 points) and
//   r_B + r_C < theta * d   and   d - r_B - r_C > gap,
// d the distance of the box centres, r the half diagonals; the second
// condition keeps every pair (k, m) with m in N_k in the direct part, where it
// is skipped by index.  Clusters that are neither far nor splittable into
// far parts are summed directly.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ibim.h"
#include "tree.h"

namespace ibim {
namespace {

struct Node {
  int32_t s = 0, e = 0;
  int32_t kid[2] = {-1, -1};
  double lo[3], hi[3];
  double c[3], r = 0.0;
};

struct Builder {
  const double* p[3];
  std::vector<int32_t>* perm;
  std::vector<Node> nodes;

  void box(Node& nd) const {
    for (int d = 0; d < 3; ++d) {
      nd.lo[d] = INFINITY;
      nd.hi[d] = -INFINITY;
    }
    for (int32_t i = nd.s; i < nd.e; ++i) {
      const int32_t m = (*perm)[i];
      for (int d = 0; d < 3; ++d) {
        nd.lo[d] = std::min(nd.lo[d], p[d][m]);
        nd.hi[d] = std::max(nd.hi[d], p[d][m]);
      }
    }
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      nd.c[d] = 0.5 * (nd.lo[d] + nd.hi[d]);
      r2 += 0.25 * (nd.hi[d] - nd.lo[d]) * (nd.hi[d] - nd.lo[d]);
    }
    nd.r = std::sqrt(r2);
  }

  // The shape depends on the counts only: a cluster of n > kTreeBatch points
  // splits into ceil(nb/2) batches and the rest (nb batches in all).
  static int32_t split(int32_t s, int32_t e) {
    const int32_t nb = (e - s + kTreeBatch - 1) / kTreeBatch;
    return s + ((nb + 1) / 2) * kTreeBatch;
  }
  static int count(int32_t s, int32_t e) {
    if (e - s <= kTreeBatch) return 1;
    const int32_t mid = split(s, e);
    return 1 + count(s, mid) + count(mid, e);
  }

  // Node id (preorder) of [s, e) and its subtree from id on; large subtrees
  // are built as tasks of the enclosing parallel region (disjoint ranges of
  // perm and of nodes, so the result does not depend on the schedule).
  void build(int32_t s, int32_t e, int id) {
    Node& nd = nodes[id];
    nd.s = s;
    nd.e = e;
    box(nd);
    if (e - s > kTreeBatch) {
      int d = 0;
      for (int q = 1; q < 3; ++q)
        if (nd.hi[q] - nd.lo[q] > nd.hi[d] - nd.lo[d]) d = q;
      const int32_t mid = split(s, e);
      const double* pd = p[d];
      std::nth_element(perm->begin() + s, perm->begin() + mid, perm->begin() + e,
                       [pd](int32_t a, int32_t b) { return pd[a] < pd[b] || (pd[a] == pd[b] && a < b); });
      const int l = id + 1, r = id + 1 + count(s, mid);
      nd.kid[0] = l;
      nd.kid[1] = r;
#pragma omp task if (mid - s > 32 * kTreeBatch) default(none) firstprivate(s, mid, l)
      build(s, mid, l);
      build(mid, e, r);
#pragma omp taskwait
    }
  }

  void build_all(int32_t M) {
    nodes.assign((size_t)count(0, M), Node());
#pragma omp parallel
#pragma omp single
    build(0, M, 0);
  }
};

}  // namespace

int build_tree_plan(const TreeParams& prm, int64_t M64, const double* px, const double* py,
                    const double* pz, const int64_t* crow, const int32_t* ccol, double h,
                    TreePlan* plan, std::string* err) {
  if (prm.order < 2 || prm.order > kTreeMaxOrder) {
    *err = "tree order must be in [2, " + std::to_string(kTreeMaxOrder) + "]";
    return IBIM_EINVAL;
  }
  if (!(prm.theta > 0.0 && prm.theta <= 1.0)) {
    *err = "tree theta must be in (0, 1]";
    return IBIM_EINVAL;
  }
  if (M64 < 1 || M64 > INT32_MAX / 2) {
    *err = "node count out of range for the treecode";
    return IBIM_EINVAL;
  }
  TreePlan& pl = *plan;
  pl = TreePlan();
  const int32_t M = (int32_t)M64;
  const int n3 = prm.order * prm.order * prm.order;
  // clusters of more than nfar nodes carry proxies (and can be far)
  const int nfar = (int)(prm.proxy_cost * n3);
  pl.M = M;
  pl.order = prm.order;

  // gap: the largest distance of a corrected pair
  double gap = 0.0;
  for (int32_t k = 0; k < M; ++k)
    for (int64_t e = crow[k]; e < crow[k + 1]; ++e) {
      const int32_t m = ccol[e];
      const double dx = px[k] - px[m], dy = py[k] - py[m], dz = pz[k] - pz[m];
      gap = std::max(gap, std::sqrt(dx * dx + dy * dy + dz * dz));
    }
  pl.gap = gap * (1.0 + 1e-9) + 1e-9 * h;

  pl.perm.resize(M);
  std::iota(pl.perm.begin(), pl.perm.end(), 0);
  Builder B;
  B.p[0] = px;
  B.p[1] = py;
  B.p[2] = pz;
  B.perm = &pl.perm;
  B.build_all(M);
  const std::vector<Node>& nd = B.nodes;
  pl.pos.resize(M);
  for (int32_t t = 0; t < M; ++t) pl.pos[pl.perm[t]] = t;

  // batches: the leaves, in tree order
  std::vector<int> leaves;
  for (int i = 0; i < (int)nd.size(); ++i)
    if (nd[i].kid[0] < 0) leaves.push_back(i);
  std::sort(leaves.begin(), leaves.end(), [&](int a, int b) { return nd[a].s < nd[b].s; });
  const int nb = (int)leaves.size();
  pl.bstart.resize(nb + 1);
  for (int b = 0; b < nb; ++b) pl.bstart[b] = nd[leaves[b]].s;
  pl.bstart[nb] = M;
  for (int b = 0; b < nb; ++b)
    if (pl.bstart[b] != b * kTreeBatch) {  // every leaf but the last holds kTreeBatch points
      *err = "internal error: unaligned treecode batch";
      return IBIM_EINVAL;
    }

  // interaction lists
  std::vector<std::vector<int>> far(nb);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> near(nb);
  const double theta = prm.theta;
#pragma omp parallel for schedule(dynamic, 16)
  for (int b = 0; b < nb; ++b) {
    const Node& L = nd[leaves[b]];
    std::vector<int> stack{0};
    while (!stack.empty()) {
      const int ci = stack.back();
      stack.pop_back();
      const Node& C = nd[ci];
      const double dx = L.c[0] - C.c[0], dy = L.c[1] - C.c[1], dz = L.c[2] - C.c[2];
      const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
      const bool sep = L.r + C.r < theta * d && d - L.r - C.r > pl.gap;
      if (sep && C.e - C.s > nfar) {
        far[b].push_back(ci);
      } else if (C.kid[0] < 0 || C.e - C.s <= nfar) {
        near[b].push_back({C.s, C.e});
      } else {
        stack.push_back(C.kid[1]);
        stack.push_back(C.kid[0]);
      }
    }
    std::sort(far[b].begin(), far[b].end());
    auto& nr = near[b];
    std::sort(nr.begin(), nr.end());
    std::vector<std::pair<int32_t, int32_t>> merged;
    for (const auto& r : nr) {
      if (!merged.empty() && merged.back().second == r.first)
        merged.back().second = r.second;
      else
        merged.push_back(r);
    }
    nr.swap(merged);
  }

  // two-way pairs: leaves b < b' near each other both ways (their near
  // ranges cover each other) with no pair of N_k between them either way are
  // taken out of both batches' near ranges and evaluated once for both
  // directions in b's work items
  std::vector<std::vector<int32_t>> pairs(nb);
  if (prm.two_way) {
    auto leaves_of = [&](const std::vector<std::pair<int32_t, int32_t>>& rs) {
      std::vector<int32_t> v;
      for (const auto& r : rs)
        for (int32_t q = r.first / kTreeBatch; q * kTreeBatch < r.second; ++q) v.push_back(q);
      return v;  // ascending: the ranges are sorted and disjoint
    };
    std::vector<std::vector<int32_t>> nl(nb), careful(nb);
    for (int b = 0; b < nb; ++b) nl[b] = leaves_of(near[b]);
    for (int32_t k = 0; k < M; ++k)
      for (int64_t e = crow[k]; e < crow[k + 1]; ++e) {
        const int32_t bk = pl.pos[k] / kTreeBatch, bm = pl.pos[ccol[e]] / kTreeBatch;
        if (bk != bm) careful[std::min(bk, bm)].push_back(std::max(bk, bm));
      }
    for (auto& c : careful) {
      std::sort(c.begin(), c.end());
      c.erase(std::unique(c.begin(), c.end()), c.end());
    }
    auto has = [](const std::vector<int32_t>& v, int32_t x) {
      return std::binary_search(v.begin(), v.end(), x);
    };
    for (int b = 0; b < nb; ++b)
      for (int32_t q : nl[b])
        if (q > b && has(nl[q], b) && !has(careful[b], q)) pairs[b].push_back(q);
    // near ranges without the two-way partners (either side), merged again
    std::vector<std::vector<int32_t>> drop(nb);
    for (int b = 0; b < nb; ++b)
      for (int32_t q : pairs[b]) {
        drop[b].push_back(q);
        drop[q].push_back(b);
      }
    for (int b = 0; b < nb; ++b) {
      std::sort(drop[b].begin(), drop[b].end());
      std::vector<std::pair<int32_t, int32_t>> rs;
      for (int32_t q : nl[b]) {
        if (has(drop[b], q)) continue;
        const int32_t s = q * kTreeBatch, e = std::min(M, s + kTreeBatch);
        if (!rs.empty() && rs.back().second == s)
          rs.back().second = e;
        else
          rs.push_back({s, e});
      }
      near[b].swap(rs);
    }
  }

  // proxy slots: every cluster of more than nfar points, in preorder (a
  // parent before its children)
  std::vector<int32_t> slot(nd.size(), -1);
  int ns = 0;
  for (size_t ci = 0; ci < nd.size(); ++ci)
    if (nd[ci].e - nd[ci].s > nfar) slot[ci] = ns++;
  pl.kid.assign(2 * (size_t)ns, -1);
  pl.dstart.resize(ns);
  pl.dend.resize(ns);
  std::vector<int> height(ns, 0);
  for (size_t ci = 0; ci < nd.size(); ++ci) {
    const int sl = slot[ci];
    if (sl < 0) continue;
    pl.pstart.push_back(nd[ci].s);
    pl.pend.push_back(nd[ci].e);
    // boxes padded to a width of at least h in every direction (flat clusters)
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = nd[ci].lo[d];
      hi[d] = nd[ci].hi[d];
      if (hi[d] - lo[d] < h) {
        const double c = 0.5 * (lo[d] + hi[d]);
        lo[d] = c - 0.5 * h;
        hi[d] = c + 0.5 * h;
      }
    }
    pl.pbox.insert(pl.pbox.end(), lo, lo + 3);
    pl.pbox.insert(pl.pbox.end(), hi, hi + 3);
    // direct part: the children without proxies (contiguous: the left child
    // ends where the right one starts), or the cluster itself for a leaf
    int32_t ds = nd[ci].e, de = nd[ci].s;
    if (nd[ci].kid[0] < 0) {
      ds = nd[ci].s;
      de = nd[ci].e;
    } else {
      for (int q = 0; q < 2; ++q) {
        const Node& K = nd[nd[ci].kid[q]];
        if (slot[nd[ci].kid[q]] >= 0) {
          pl.kid[2 * sl + q] = slot[nd[ci].kid[q]];
          pl.m2m_links += 1.0;
        } else {
          ds = std::min(ds, K.s);
          de = std::max(de, K.e);
        }
      }
      if (ds > de) ds = de = nd[ci].s;
    }
    pl.dstart[sl] = ds;
    pl.dend[sl] = de;
    pl.proxy_evals += (double)(de - ds) * n3;
  }
  // heights (children follow their parent in preorder)
  for (int sl = ns - 1; sl >= 0; --sl)
    for (int q = 0; q < 2; ++q)
      if (pl.kid[2 * sl + q] >= 0) height[sl] = std::max(height[sl], height[pl.kid[2 * sl + q]] + 1);
  const int hmax = ns > 0 ? *std::max_element(height.begin(), height.end()) : -1;
  pl.mlevel.assign(1, 0);
  for (int hh = 0; hh <= hmax; ++hh) {
    for (int sl = 0; sl < ns; ++sl)
      if (height[sl] == hh) pl.mlist.push_back(sl);
    pl.mlevel.push_back((int32_t)pl.mlist.size());
  }

  pl.frow.assign(1, 0);
  pl.nrow.assign(1, 0);
  pl.prow.assign(1, 0);
  std::vector<double> work(nb);
  auto batch_size = [&](int b) { return (double)(pl.bstart[b + 1] - pl.bstart[b]); };
  std::vector<std::vector<int32_t>> incoming(nb);
  for (int b = 0; b < nb; ++b) {
    const double nt = batch_size(b);
    for (int ci : far[b]) pl.fcol.push_back(slot[ci]);
    pl.frow.push_back((int32_t)pl.fcol.size());
    double ns_near = 0.0;
    for (const auto& r : near[b]) {
      pl.nlo.push_back(r.first);
      pl.nhi.push_back(r.second);
      ns_near += r.second - r.first;
    }
    pl.nrow.push_back((int32_t)pl.nlo.size());
    double ns_pair = 0.0;
    for (int32_t q : pairs[b]) {
      incoming[q].push_back((int32_t)pl.pcol.size());
      pl.pcol.push_back(q);
      pl.pown.push_back(b);
      ns_pair += batch_size(q);
    }
    pl.prow.push_back((int32_t)pl.pcol.size());
    pl.far_evals += nt * n3 * (double)far[b].size();
    pl.near_evals += nt * ns_near + 2.0 * nt * ns_pair;
    work[b] = (double)far[b].size() * n3 * prm.proxy_cost + ns_near;
  }
  pl.inrow.assign(1, 0);
  for (int b = 0; b < nb; ++b) {
    pl.incol.insert(pl.incol.end(), incoming[b].begin(), incoming[b].end());
    pl.inrow.push_back((int32_t)pl.incol.size());
  }

  // work items: about kItems in all (at least kMinPart of work per target each)
  constexpr double kItems = 8192.0, kMinPart = 4096.0;
  double total = 0.0;
  for (int b = 0; b < nb; ++b) total += work[b];
  const double part = std::max(kMinPart, total / kItems);
  const double wfar = (double)n3 * prm.proxy_cost;  // one far cluster, in direct pairs
  std::vector<double> iwork;
  pl.istart.assign(1, 0);
  for (int b = 0; b < nb; ++b) {
    int32_t f = pl.frow[b], r = pl.nrow[b];
    const int32_t fe = pl.frow[b + 1], re = pl.nrow[b + 1];
    do {
      const int32_t f0 = f, r0 = r;
      double acc = 0.0;
      while (f < fe && (acc == 0.0 || acc + wfar <= part)) {
        acc += wfar;
        ++f;
      }
      while (f == fe && r < re && (acc == 0.0 || acc + (pl.nhi[r] - pl.nlo[r]) <= part)) {
        acc += pl.nhi[r] - pl.nlo[r];
        ++r;
      }
      pl.ibatch.push_back(b);
      pl.ifar0.push_back(f0);
      pl.ifar1.push_back(f);
      pl.inear0.push_back(r0);
      pl.inear1.push_back(r);
      iwork.push_back(acc);
    } while (f < fe || r < re);
    pl.istart.push_back((int32_t)pl.ibatch.size());
  }
  pl.iorder.resize(pl.ibatch.size());
  std::iota(pl.iorder.begin(), pl.iorder.end(), 0);
  std::stable_sort(pl.iorder.begin(), pl.iorder.end(),
                   [&](int a, int b) { return iwork[a] > iwork[b]; });

  // N_k in tree positions
  pl.xrow.resize(M + 1);
  pl.xrow[0] = 0;
  for (int32_t t = 0; t < M; ++t) {
    const int32_t k = pl.perm[t];
    pl.xrow[t + 1] = pl.xrow[t] + (int32_t)(crow[k + 1] - crow[k]);
  }
  pl.xcol.resize(pl.xrow[M]);
  for (int32_t t = 0; t < M; ++t) {
    const int32_t k = pl.perm[t];
    int32_t* o = pl.xcol.data() + pl.xrow[t];
    for (int64_t e = crow[k]; e < crow[k + 1]; ++e) *o++ = pl.pos[ccol[e]];
    std::sort(pl.xcol.data() + pl.xrow[t], o);
  }
  pl.enabled = true;
  return IBIM_OK;
}

size_t tree_device_bytes(const TreePlan& pl) {
  const size_t n = (size_t)pl.order, n3 = n * n * n, M = (size_t)pl.M;
  const size_t ints = pl.perm.size() + pl.pos.size() + pl.bstart.size() + pl.dstart.size() +
                      pl.dend.size() + pl.kid.size() + pl.mlist.size() + pl.ibatch.size() +
                      pl.ifar0.size() + pl.ifar1.size() + pl.inear0.size() + pl.inear1.size() +
                      pl.istart.size() + pl.iorder.size() + pl.fcol.size() + pl.nlo.size() +
                      pl.nhi.size() + pl.xrow.size() + pl.xcol.size() + pl.prow.size() +
                      pl.pcol.size() + pl.pown.size() + pl.inrow.size() + pl.incol.size();
  // work-item partial sums, and row and column sums of the two-way pairs
  const size_t dbls = pl.pbox.size() + (2 * n + n * n) + 9 * M + pl.pstart.size() * n3 * 2 +
                      (pl.ibatch.size() + 2 * pl.pcol.size()) * 2 * (size_t)kTreeBatch;
  return ints * 4 + dbls * 8;
}

}  // namespace ibim
