"""Host checks of the treecode options (no GPU): invalid combinations are
rejected before any device work, through the C ABI's host-only contexts."""
import pytest

import workloads
from paper_2210_03699_amd import ibim


@pytest.mark.parametrize("kw", [
    {"summation": ibim.SUM_TREE, "precision": ibim.MIXED},
    {"summation": ibim.SUM_TREE, "tree_order": 1},
    {"summation": ibim.SUM_TREE, "tree_order": 13},
    {"summation": ibim.SUM_TREE, "tree_theta": 0.0},
    {"summation": ibim.SUM_TREE, "tree_theta": 1.5},
    {"summation": 2},
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
