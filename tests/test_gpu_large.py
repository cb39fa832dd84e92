"""A problem past half a million tube nodes: the Kirkwood sphere (R = 10,
20 charges) at h = 0.1, eps = 3h, M ~ 7.5e5.

At this size the symmetric pair kernel keeps a column-sum scratch of several
GB (it grows as M^2); the check is that its packed layout and the finishing
kernels read back exactly what the work items wrote.  Sampled rows of
``apply`` in float64 and mixed precision are compared with the oracle's rows
(computed here, weights only at the sampled rows), and the float64 and mixed
solves with each other and with the Kirkwood series (discretisation error).
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


@pytest.fixture(scope="module")
def large():
    wl = workloads.kirkwood_sphere(h=0.1)
    _say(f"[large] grid={wl.sdf.shape}")
    o0 = oracle.Oracle.from_workload(wl, weight_rows=np.zeros(1, dtype=np.int64))
    rng = np.random.Generator(np.random.PCG64(91))
    rows = np.sort(rng.choice(o0.M, size=N_ROWS, replace=False))
    del o0
    orc = oracle.Oracle.from_workload(wl, weight_rows=rows)
    u = workloads.random_vector(2 * orc.M, 92)
    ref1, ref2 = orc.apply_rows(u, rows)
    _say(f"[large] M={orc.M} oracle rows done")
    return wl, rows, u, ref1, ref2, orc.M


@pytest.mark.parametrize("precision,bar", [(ibim.FP64, 1e-12), (ibim.MIXED, 1e-6)])
def test_large_sampled_apply(large, precision, bar):
    wl, rows, u, ref1, ref2, M = large
    prob = ibim.Problem.from_workload(wl, device=0, precision=precision)
    assert prob.M == M and M > 524288  # an unpacked column-sum scratch would exceed 4 GiB here
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    e1 = np.max(np.abs(out[rows] - ref1)) / np.max(np.abs(ref1))
    e2 = np.max(np.abs(out[M + rows] - ref2)) / np.max(np.abs(ref2))
    _say(f"[large] precision={precision} sampled apply rel err {e1:.3e} {e2:.3e}")
    assert e1 < bar and e2 < bar
    prob.close()


def test_large_solves(large):
    wl, rows, u, ref1, ref2, M = large
    g = {}
    for precision in (ibim.FP64, ibim.MIXED):
        prob = ibim.Problem.from_workload(wl, device=0, precision=precision)
        _, info = prob.solve_energy(wl.tol)
        assert info["converged"]
        g[precision] = info["g_pol"]
        _say(f"[large] precision={precision} iters={info['iters']} G={info['g_pol']:.15e} "
             f"t={info['seconds']:.2f}s")
        prob.close()
    exact = analytic.kirkwood_energy(wl.charge_xyz, wl.charge_q, 10.0, wl.eps_in, wl.eps_out,
                                     wl.kappa)
    assert abs(g[ibim.MIXED] - g[ibim.FP64]) <= 1e-6 * abs(g[ibim.FP64])
    assert abs(g[ibim.FP64] - exact) <= 1e-2 * abs(exact)  # discretisation error
