"""Problems past half a million tube nodes: the Kirkwood sphere (R = 10,
20 charges) at h = 0.1 (M = 754,301) and h = 0.07 (M = 1,540,232, the size of
the largest molecular workload the method is aimed at).

At these sizes the symmetric pair kernel spans 8 and 16 row tiles per work item
and keeps a row- and column-sum scratch of 2.5 and 5.8 GB (it grows as
M^2 / rows); the check is that its packed layout, the row sums carried in
their slots from one column tile to the next, and the finishing kernels
read back exactly what the work items wrote.  Sampled rows
of ``apply`` (float64, mixed, treecode in float64 and mixed) are compared with the oracle's rows
(computed here, weights only at the sampled rows); the solves are compared
with each other and with the Kirkwood series (discretisation error).
"""
import sys

import numpy as np
import pytest

import analytic
import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_03699_amd import ibim  # noqa: E402

DEV = "cuda:0"
N_ROWS = 48


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[0.1, 0.07])
def large(request):
    wl = workloads.kirkwood_sphere(h=request.param)
    _say(f"[large h={request.param}] grid={wl.sdf.shape}")
    o0 = oracle.Oracle.from_workload(wl, weight_rows=np.zeros(1, dtype=np.int64))
    rng = np.random.Generator(np.random.PCG64(91))
    rows = np.sort(rng.choice(o0.M, size=N_ROWS, replace=False))
    del o0
    orc = oracle.Oracle.from_workload(wl, weight_rows=rows)
    u = workloads.random_vector(2 * orc.M, 92)
    ref1, ref2 = orc.apply_rows(u, rows)
    _say(f"[large h={request.param}] M={orc.M} oracle rows done")
    return request.param, wl, rows, u, ref1, ref2, orc.M


MODES = {"fp64": ({"precision": ibim.FP64}, 1e-12), "mixed": ({"precision": ibim.MIXED}, 1e-6),
         "tree": ({"summation": ibim.SUM_TREE}, 1e-6),
         "tree_mixed": ({"summation": ibim.SUM_TREE, "precision": ibim.MIXED}, 1e-6)}


@pytest.mark.parametrize("mode", list(MODES))
def test_large_sampled_apply(large, mode):
    h, wl, rows, u, ref1, ref2, M = large
    kw, bar = MODES[mode]
    prob = ibim.Problem.from_workload(wl, device=0, **kw)
    assert prob.M == M and M > 524288  # an unpacked column-sum scratch would exceed 4 GiB here
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    e1 = np.max(np.abs(out[rows] - ref1)) / np.max(np.abs(ref1))
    e2 = np.max(np.abs(out[M + rows] - ref2)) / np.max(np.abs(ref2))
    _say(f"[large h={h}] {mode} sampled apply rel err {e1:.3e} {e2:.3e}")
    assert e1 < bar and e2 < bar
    prob.close()


def test_large_solves(large):
    h, wl, rows, u, ref1, ref2, M = large
    modes = ("fp64", "mixed", "tree", "tree_mixed")
    g = {}
    for mode in modes:
        prob = ibim.Problem.from_workload(wl, device=0, **MODES[mode][0])
        _, info = prob.solve_energy(wl.tol)
        assert info["converged"]
        g[mode] = info["g_pol"]
        _say(f"[large h={h}] {mode} iters={info['iters']} G={info['g_pol']:.15e} "
             f"t={info['seconds']:.2f}s")
        prob.close()
    exact = analytic.kirkwood_energy(wl.charge_xyz, wl.charge_q, 10.0, wl.eps_in, wl.eps_out,
                                     wl.kappa)
    ref = g["fp64"]
    for mode in modes:
        assert abs(g[mode] - ref) <= 1e-6 * abs(ref)
    assert abs(ref - exact) <= 1e-2 * abs(exact)  # discretisation error
    _say(f"[large h={h}] G_pol vs Kirkwood series {abs(ref - exact) / abs(exact):.2e}")
