"""Host checks of the treecode options (no GPU): invalid combinations are
rejected before any device work, through the C ABI's host-only contexts."""
import numpy as np
import pytest

import workloads
from paper_2210_03699_amd import ibim


@pytest.mark.parametrize("kw", [
    {"summation": ibim.SUM_TREE, "tree_order": 1},
    {"summation": ibim.SUM_TREE, "tree_order": 13},
    {"summation": ibim.SUM_TREE, "tree_theta": 0.0},
    {"summation": ibim.SUM_TREE, "tree_theta": 1.5},
    {"summation": 2},
    {"summation": ibim.SUM_TREE, "tree_min_nodes": -1},
])
def test_bad_tree_options_rejected(kw):
    wl = workloads.born_sphere(h=0.4)
    with pytest.raises(ibim.IbimError):
        ibim.Problem.from_workload(wl, device=-1, **kw)


def test_tree_options_accepted_on_host():
    wl = workloads.born_sphere(h=0.4)
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE, tree_order=6,
                                   tree_theta=0.5)
    assert p.M > 0
    p.close()


def test_tree_resolved_by_size():
    """IBIM_SUM_TREE serves problems of at least tree_min_nodes nodes; smaller
    ones keep the direct sum; the precision is the one requested."""
    wl = workloads.born_sphere(h=0.4)
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE)
    assert (p.summation, p.precision) == (ibim.SUM_TREE, ibim.FP64)
    M = p.M
    p.close()
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE, tree_min_nodes=M)
    assert (p.summation, p.precision) == (ibim.SUM_TREE, ibim.FP64)
    p.tree_plan()  # a treecode context has a plan
    p.close()
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE, tree_min_nodes=M,
                                   precision=ibim.MIXED)
    assert (p.summation, p.precision) == (ibim.SUM_TREE, ibim.MIXED)
    p.close()
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE,
                                   tree_min_nodes=M + 1, precision=ibim.MIXED)
    assert (p.summation, p.precision) == (ibim.SUM_DIRECT, ibim.MIXED)
    with pytest.raises(ibim.IbimError):
        p.tree_plan()  # not a treecode context
    p.close()


def _box(P):
    lo, hi = P.min(0), P.max(0)
    return 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo)


PLAN_CASES = {
    "sphere": (lambda: workloads.kirkwood_sphere(h=0.25, radius=4.0, r_charges=2.0), 4, 0.7),
    "sphere_theta0.5": (lambda: workloads.kirkwood_sphere(h=0.25, radius=4.0, r_charges=2.0),
                        3, 0.5),
    "ses_hyb": (lambda: workloads.ses_molecule(60, 14.0, 0.35, 2.0, seed=11), 4, 0.8),
    "sphere_mixed_order8": (lambda: workloads.kirkwood_sphere(h=0.25, radius=6.0, r_charges=2.0),
                            8, 0.7),
}
# cost of a target-proxy evaluation in direct pairs: clusters of more than
# this times n^3 nodes carry proxies
PROXY_COST = {ibim.FP64: 0.44, ibim.MIXED: 0.26}


@pytest.mark.parametrize("name", list(PLAN_CASES))
def test_tree_plan_invariants(name):
    """The plan the treecode runs: every batch sees every source exactly once
    (far clusters, direct ranges and two-way pairs of leaves, evaluated once
    for both batches), far clusters pass the separation
    test recomputed from the node positions, clusters with proxies hold more
    nodes than c n^3 (c the cost of a target-proxy evaluation in direct pairs:
    0.44 float64, 0.26 mixed), two-way pairs are leaves that are near each
    other and hold no pair of N_k, every pair of N_k is in the direct
    part, and each cluster's charges come from its children and its own
    direct sources without overlap."""
    make, order, theta = PLAN_CASES[name]
    wl = make()
    hyb = ibim.HYB if name == "ses_hyb" else ibim.CTR2
    prec = ibim.MIXED if "mixed" in name else ibim.FP64
    p = ibim.Problem.from_workload(wl, device=-1, summation=ibim.SUM_TREE, tree_order=order,
                                   tree_theta=theta, hybrid=hyb, precision=prec)
    t = p.tree_plan()
    P, _, _ = p.node_geometry()
    c = p.corrections()
    M, nfar = p.M, int(PROXY_COST[prec] * order ** 3)
    perm, bst = t["perm"], t["bstart"]
    assert np.array_equal(np.sort(perm), np.arange(M))
    pos = np.empty(M, np.int64)
    pos[perm] = np.arange(M)
    B = len(bst) - 1
    assert bst[0] == 0 and bst[-1] == M
    assert np.all(bst[:-1] == 256 * np.arange(B))  # full batches but the last
    Pt = P[perm]
    # gap: the largest corrected-pair distance
    rows = np.repeat(np.arange(M), np.diff(c["row"]))
    dist = np.linalg.norm(P[rows] - P[c["col"]], axis=1)
    assert abs(t["gap"] - dist.max()) <= 1e-8 * dist.max() + 1e-8 * wl.h
    cl = [(t["cstart"][i], t["cend"][i]) for i in range(len(t["cstart"]))]
    lo, hi = p.tree_pairs()
    assert len(lo) > 0  # the cases are large enough to have two-way pairs
    assert np.all(lo < hi)
    assert np.all(np.diff(lo.astype(np.int64) * B + hi) > 0)  # ordered, no repeats
    partners = [[] for _ in range(B)]
    for b1, b2 in zip(lo, hi):
        partners[b1].append(b2)
        partners[b2].append(b1)
    # batches holding a pair of N_k between them (either way)
    bt = pos // 256
    careful = set(zip(bt[rows], bt[c["col"]]))
    for b1, b2 in zip(lo, hi):
        assert (b1, b2) not in careful and (b2, b1) not in careful
    far_total = 0
    for b in range(B):
        cover = np.zeros(M, np.int32)
        cb, rb = _box(Pt[bst[b]:bst[b + 1]])
        for f in t["fcol"][t["frow"][b]:t["frow"][b + 1]]:
            s, e = cl[f]
            cover[s:e] += 1
            cc, rc = _box(Pt[s:e])
            d = np.linalg.norm(cb - cc)
            assert e - s > nfar and rb + rc < theta * d and d - rb - rc > t["gap"]
            far_total += 1
        near = np.zeros(M, bool)
        for r in range(t["nrow"][b], t["nrow"][b + 1]):
            cover[t["nlo"][r]:t["nhi"][r]] += 1
            near[t["nlo"][r]:t["nhi"][r]] = True
        for q in partners[b]:
            cover[bst[q]:bst[q + 1]] += 1
            near[bst[q]:bst[q + 1]] = True
        assert np.all(cover == 1), b
        for tt in range(bst[b], bst[b + 1]):
            k = perm[tt]
            assert np.all(near[pos[c["col"][c["row"][k]:c["row"][k + 1]]]])
    assert far_total > 0  # the cases are large enough to have a far field
    for i, (s, e) in enumerate(cl):
        assert e - s > nfar
        cover = np.zeros(e - s, np.int32)
        cover[t["dstart"][i] - s:t["dend"][i] - s] += 1
        for q in t["kid"][2 * i:2 * i + 2]:
            if q >= 0:
                assert s <= cl[q][0] < cl[q][1] <= e
                cover[cl[q][0] - s:cl[q][1] - s] += 1
        assert np.all(cover == 1)
        assert np.all(t["cbox"][i, :3] <= Pt[s:e].min(0)) and np.all(t["cbox"][i, 3:] >= Pt[s:e].max(0))
    p.close()
