"""GPU checks of ``ibim_apply_noalloc`` (the allocation-free operator
application) against ``ibim_apply`` on the same contexts.

Two calls in a row, the second on a smaller problem, so the second reads a
static scratch that still holds the first call's partial sums: the result
must not depend on them.  Symmetric-kernel calls must equal ``ibim_apply``
bit for bit (same kernels, same plan); a problem whose symmetric partial sums
exceed the static array runs the one-directional kernels and must agree with
``ibim_apply`` within float64 rounding (1e-12 of each block row's largest
entry, the operator bar used against the oracle).  Treecode contexts are
rejected with an error.
"""
import sys

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_03699_amd import ibim  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b, M):
    return max(np.max(np.abs(a[:M] - b[:M])) / np.max(np.abs(b[:M])),
               np.max(np.abs(a[M:] - b[M:])) / np.max(np.abs(b[M:])))


@pytest.mark.parametrize("precision", [ibim.FP64, ibim.MIXED])
def test_noalloc_equals_apply_two_calls(precision):
    big = workloads.kirkwood_sphere(h=0.25, radius=4.0, r_charges=3.0, n_charges=6, seed=9)
    small = workloads.born_sphere(h=0.4)
    seen = []
    for name, wl in (("larger", big), ("smaller", small)):
        prob = ibim.Problem.from_workload(wl, device=0, precision=precision)
        seen.append(prob.M)
        u = torch.from_numpy(workloads.random_vector(2 * prob.M, 21)).to(DEV)
        ref = prob.apply(u).cpu().numpy()
        out = torch.full((2 * prob.M,), float("nan"), dtype=torch.float64, device=DEV)
        prob.apply_noalloc(u, out)
        got = out.cpu().numpy()
        _say(f"[noalloc {precision}] {name} M={prob.M}: max |diff| "
             f"{np.max(np.abs(got - ref)):.3e}")
        assert np.array_equal(got, ref), f"{name}: noalloc differs from ibim_apply"
        prob.close()
    assert seen[1] < seen[0]


def test_noalloc_one_directional_when_symmetric_sums_do_not_fit():
    """Kirkwood sphere at h = 0.2 (M = 188,926): the symmetric partial sums
    (354 MB) exceed the 256 MiB array, the one-directional ones (73 MB) fit;
    then a smaller problem (symmetric sums)."""
    for name, wl in (("kirkwood", workloads.kirkwood_sphere(h=0.2)),
                     ("born", workloads.born_sphere(h=0.3))):
        prob = ibim.Problem.from_workload(wl, device=0)
        if name == "kirkwood":
            assert prob.M > 180000, prob.M  # past the size the static array holds symmetric sums for
        u = torch.from_numpy(workloads.random_vector(2 * prob.M, 22)).to(DEV)
        ref = prob.apply(u).cpu().numpy()
        out = torch.full((2 * prob.M,), float("nan"), dtype=torch.float64, device=DEV)
        prob.apply_noalloc(u, out)
        got = out.cpu().numpy()
        err = _rel(got, ref, prob.M)
        _say(f"[noalloc] {name} M={prob.M}: rel diff vs ibim_apply {err:.3e}")
        assert np.all(np.isfinite(got)) and err < 1e-12
        prob.close()


def test_noalloc_rejects_treecode_contexts():
    wl = workloads.born_sphere(h=0.4)
    prob = ibim.Problem.from_workload(wl, device=0, summation=ibim.SUM_TREE)
    u = torch.zeros(2 * prob.M, dtype=torch.float64, device=DEV)
    out = torch.empty_like(u)
    with pytest.raises(ibim.IbimError, match="treecode"):
        prob.apply_noalloc(u, out)
    prob.close()
