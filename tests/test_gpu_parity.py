"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (float64 path): correction weights and ``apply`` agree with the oracle
to 1e-12 relative to the largest entry of each block row; the GMRES solution
to 1e-9 and the polarisation energy to 1e-10 relative; index work (node
order, correction sets) exactly.  The full-size Kirkwood case is checked on
sampled rows against values stored by ``tests/golden/make_golden.py``.
"""
import json
import os
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _blockwise_rel(a, b, M):
    """max |a - b| / max |b| over each half (psi rows, psi_n rows)."""
    r1 = np.max(np.abs(a[:M] - b[:M])) / np.max(np.abs(b[:M]))
    r2 = np.max(np.abs(a[M:] - b[M:])) / np.max(np.abs(b[M:]))
    return max(r1, r2)


CASES = {
    "born_h0.4": lambda: workloads.born_sphere(h=0.4),
    "born_h0.2": lambda: workloads.born_sphere(h=0.2),
    "offset_sphere": lambda: workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23)),
    "tiny_sphere": lambda: workloads.born_sphere(h=0.3, radius=0.6, eps_factor=1.5),
    "torus": lambda: workloads.torus_case(h=0.1),
    "kirkwood_small": lambda: workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0,
                                                        n_charges=5, seed=7, tol=1e-10),
    "ses_molecule": lambda: workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11, tol=1e-10),
    # degenerate parameters: no screening (kappa = 0, K12 and K21 vanish), no
    # dielectric jump (eps_in = eps_out, lambda = 1), strong screening (kappa R ~ 7)
    "laplace": lambda: workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23),
                                             kappa=0.0),
    "no_jump": lambda: workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23),
                                             eps_in=2.0, eps_out=2.0, kappa=0.3),
    "strong_screening": lambda: workloads.born_sphere(h=0.25, radius=1.7,
                                                      offset=(0.37, 0.11, -0.23), kappa=3.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    wl = CASES[request.param]()
    _say(f"[case {request.param}] grid={wl.sdf.shape}")
    prob = ibim.Problem.from_workload(wl, device=0)
    orc = oracle.Oracle.from_workload(wl)
    _say(f"[case {request.param}] M={prob.M} nnz={prob.nnz}")
    return request.param, wl, prob, orc


def test_sizes_and_sets(pair):
    name, wl, prob, orc = pair
    assert prob.M == orc.M and prob.nnz == orc.nnz
    assert np.array_equal(prob.corrections()["row"], orc.corrections()["row"])


def test_weights_match_oracle(pair):
    name, wl, prob, orc = pair
    om11, om21 = prob.correction_weights()
    co = orc.corrections()
    cl = prob.corrections()
    # reorder the oracle's entries (plane order) to the library's (column order)
    perm = np.empty(prob.nnz, dtype=np.int64)
    for k in range(prob.M):
        s = slice(co["row"][k], co["row"][k + 1])
        perm[s] = co["row"][k] + np.argsort(co["col"][s], kind="stable")
    assert np.array_equal(cl["col"], co["col"][perm])
    for got, ref in ((om11, co["om11"][perm]), (om21, co["om21"][perm])):
        if np.max(np.abs(ref)) == 0.0:  # omega^(21) carries kappa^2: zero without screening
            assert np.max(np.abs(got)) == 0.0, name
            continue
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < 1e-12, (name, err)


def test_apply_matches_oracle(pair):
    name, wl, prob, orc = pair
    u = workloads.random_vector(2 * prob.M, 11)
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    ref = orc.apply(u)
    err = _blockwise_rel(out, ref, prob.M)
    _say(f"[{name}] apply rel err {err:.3e}")
    assert err < 1e-12, (name, err)


def test_apply_is_deterministic(pair):
    name, wl, prob, orc = pair
    u = torch.from_numpy(workloads.random_vector(2 * prob.M, 12)).to(DEV)
    a = prob.apply(u).cpu().numpy()
    b = prob.apply(u).cpu().numpy()
    assert np.array_equal(a, b)


def test_rhs_matches_oracle(pair):
    name, wl, prob, orc = pair
    g = prob.rhs().cpu().numpy()
    ref = orc.rhs(wl.charge_xyz, wl.charge_q)
    assert _blockwise_rel(g, ref, prob.M) < 1e-13


def test_solve_and_energy_match_oracle(pair):
    name, wl, prob, orc = pair
    tol = 1e-10
    x, info = prob.solve_energy(tol)
    xo, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, tol)
    _say(f"[{name}] iters gpu={info['iters']} oracle={info_o['iters']} "
         f"G={info['g_pol']:.15e} G_oracle={info_o['g_pol']:.15e}")
    assert info["converged"] and info["status"] == 0
    # same Krylov iterates up to rounding; a residual within rounding of the
    # tolerance may stop one iteration apart (classical vs modified Gram-Schmidt)
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert info["explicit_rel_resid"] < 10 * tol
    assert _blockwise_rel(x.cpu().numpy(), xo, prob.M) < 1e-9
    assert abs(info["g_pol"] - info_o["g_pol"]) <= 1e-10 * abs(info_o["g_pol"])
    # the energy step alone, on the oracle's own solution
    g_on_oracle_x = prob.energy(torch.from_numpy(xo).to(DEV))
    assert abs(g_on_oracle_x - info_o["g_pol"]) <= 1e-12 * abs(info_o["g_pol"])


# The one-directional kernels: the path of problems whose symmetric partial
# sums would exceed the scratch cap (32 GiB by default, M above ~2e6), forced
# here by a one-byte cap.
ONEDIR = ["born_h0.2", "offset_sphere", "torus", "kirkwood_small", "ses_molecule"]


@pytest.mark.parametrize("name", ONEDIR)
@pytest.mark.parametrize("precision,bar", [(ibim.FP64, 1e-12), (ibim.MIXED, 1e-6)])
def test_one_directional_apply_matches_oracle(name, precision, bar):
    wl = CASES[name]()
    prob = ibim.Problem.from_workload(wl, device=0, precision=precision, pair_scratch_max=1)
    orc = oracle.Oracle.from_workload(wl)
    u = workloads.random_vector(2 * prob.M, 11)
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    err = _blockwise_rel(out, orc.apply(u), prob.M)
    pairs, flops = prob.pair_work()
    _say(f"[{name} one-directional precision={precision}] apply rel err {err:.3e} "
         f"flops/pair {flops / pairs:.1f}")
    assert flops == 60.0 * prob.M * prob.M  # the one-directional count: no shared evaluation
    assert err < bar, (name, err)
    prob.close()


@pytest.mark.parametrize("name", ["kirkwood_small", "ses_molecule"])
def test_one_directional_solve_matches_oracle(name):
    wl = CASES[name]()
    prob = ibim.Problem.from_workload(wl, device=0, pair_scratch_max=1)
    orc = oracle.Oracle.from_workload(wl)
    x, info = prob.solve_energy(1e-10)
    _, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10)
    _say(f"[{name} one-directional] iters {info['iters']} / {info_o['iters']} "
         f"G {info['g_pol']:.15e} / {info_o['g_pol']:.15e}")
    assert info["converged"] and abs(info["iters"] - info_o["iters"]) <= 1
    assert abs(info["g_pol"] - info_o["g_pol"]) <= 1e-10 * abs(info_o["g_pol"])
    prob.close()


@pytest.mark.parametrize("kappa", [1e-9, 1e-3])
@pytest.mark.parametrize("precision, bar", [(ibim.FP64, 1e-12), (ibim.MIXED, 1e-6)])
def test_weak_screening_apply_matches_oracle(kappa, precision, bar):
    """The symmetric kernels evaluate pairs in units of the Debye length 1/kappa
    when those units stay in range: float64 for kappa > 1e-30, float32 (the
    mixed form) for kappa h >= 1e-6.  At h = 0.25, kappa = 1e-9 runs the
    float64 kernel in Debye units (positions ~1e-9, kappa^2 w u ~1e-21) and the
    mixed kernel in plain units; kappa = 1e-3 runs both in Debye units.  Each
    is held to the oracle at its precision's bar."""
    wl = workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23), kappa=kappa)
    prob = ibim.Problem.from_workload(wl, device=0, precision=precision)
    orc = oracle.Oracle.from_workload(wl)
    u = workloads.random_vector(2 * prob.M, 13)
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    err = _blockwise_rel(out, orc.apply(u), prob.M)
    pairs, flops = prob.pair_work()
    _say(f"[kappa={kappa} precision={precision}] apply rel err {err:.3e} "
         f"flops/pair {flops / pairs:.2f}")
    assert np.all(np.isfinite(out))
    assert err < bar, err
    prob.close()


@pytest.mark.parametrize("kappa, symmetric", [(100.0, True), (150.0, False)])
def test_extreme_screening_apply_matches_oracle(kappa, symmetric):
    """The float64 symmetric kernel's table exponential takes kappa R up to 708
    (e^{-kappa R} a normal number); a problem whose kappa times its nodes'
    bounding-box diagonal exceeds that is served by the one-directional
    kernel.  On a sphere of radius 1.7 the diagonal is about 5.9, so kappa =
    100 stays symmetric (kappa R up to ~590, e^{-kappa R} ~ 1e-256) and
    kappa = 150 switches."""
    wl = workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23), kappa=kappa)
    prob = ibim.Problem.from_workload(wl, device=0)
    orc = oracle.Oracle.from_workload(wl)
    p, _, _ = prob.node_geometry()
    span = float(np.linalg.norm(p.max(axis=0) - p.min(axis=0)))
    assert (kappa * span <= 708.0) == symmetric, (kappa, span)
    u = workloads.random_vector(2 * prob.M, 12)
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    err = _blockwise_rel(out, orc.apply(u), prob.M)
    pairs, flops = prob.pair_work()
    _say(f"[kappa={kappa}] kappa*span {kappa * span:.1f} apply rel err {err:.3e} "
         f"flops/pair {flops / pairs:.1f}")
    assert (flops < 60.0 * prob.M * prob.M) == symmetric
    assert err < 1e-12, err
    prob.close()


def test_restarted_solve_matches_oracle():
    wl = workloads.born_sphere(h=0.4)
    prob = ibim.Problem.from_workload(wl, device=0, restart=4, max_iter=200)
    orc = oracle.Oracle.from_workload(wl)
    x, info = prob.solve_energy(1e-10)
    xo, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10, restart=4, maxit=200)
    # restart cycles compound rounding differences, so the stopping iteration
    # may shift by a few; both meet the tolerance and agree on the energy
    assert info["converged"] and info_o["status"] == 0
    assert abs(info["iters"] - info_o["iters"]) <= 4
    assert info["explicit_rel_resid"] < 1e-9
    assert abs(info["g_pol"] - info_o["g_pol"]) <= 1e-9 * abs(info_o["g_pol"])


def test_unscaled_gmres_matches_oracle():
    """IBIM_PRECOND_NONE: GMRES on A x = b as written, against the oracle's."""
    wl = workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0, n_charges=5, seed=7,
                                   tol=1e-10)
    prob = ibim.Problem.from_workload(wl, device=0, precond=ibim.PRECOND_NONE)
    orc = oracle.Oracle.from_workload(wl)
    x, info = prob.solve_energy(1e-10)
    xo, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10, precond=0)
    _say(f"[unscaled] iters {info['iters']} oracle {info_o['iters']}")
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert abs(info["g_pol"] - info_o["g_pol"]) <= 1e-10 * abs(info_o["g_pol"])


HYBRID_CASES = {
    "hyb_ses": (lambda: workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11, tol=1e-10),
                ibim.HYB),
    "kreg_sphere": (lambda: workloads.born_sphere(h=0.4, offset=(0.13, -0.07, 0.21)),
                    ibim.KREG),
}


@pytest.mark.parametrize("name", list(HYBRID_CASES))
def test_hybrid_rows_match_oracle(name):
    """HYB-IBIM / K-reg rows: flags, weights (K-reg entries zero), apply and solve."""
    make, hybrid = HYBRID_CASES[name]
    wl = make()
    prob = ibim.Problem.from_workload(wl, device=0, hybrid=hybrid)
    orc = oracle.Oracle.from_workload(wl, hybrid=hybrid)
    bad = orc.bad_nodes()
    assert np.array_equal(prob.node_flags(), bad) and bad.any()
    om11, om21 = prob.correction_weights()
    cl = prob.corrections()
    assert np.all(om11[cl["axis"] < 0] == 0.0) and np.all(om21[cl["axis"] < 0] == 0.0)
    u = workloads.random_vector(2 * prob.M, 11)
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    err = _blockwise_rel(out, orc.apply(u), prob.M)
    x, info = prob.solve_energy(1e-10)
    xo, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10)
    eg = abs(info["g_pol"] - info_o["g_pol"]) / abs(info_o["g_pol"])
    _say(f"[{name}] M={prob.M} bad={int(bad.sum())} apply {err:.2e} G {eg:.2e} "
         f"iters {info['iters']}/{info_o['iters']}")
    assert err < 1e-12
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert eg <= 1e-10


def test_warm_start():
    """ibim_solve_guess: from the solution it stops at once; from a nearby
    guess it needs fewer iterations than from zero and reaches the same G_pol."""
    wl = workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0, n_charges=5, seed=7,
                                   tol=1e-10)
    prob = ibim.Problem.from_workload(wl, device=0)
    g = prob.rhs()
    x, info = prob.solve(g, 1e-10)
    G = prob.energy(x)
    x1, info1 = prob.solve(g, 1e-10, x=x.clone(), warm=True)
    assert info1["converged"] and info1["iters"] <= 1
    x2, info2 = prob.solve(g, 1e-10, x=0.9 * x, warm=True)
    G2 = prob.energy(x2)
    _say(f"[warm] cold {info['iters']} from solution {info1['iters']} from 0.9x {info2['iters']}")
    assert info2["converged"] and info2["iters"] < info["iters"]
    assert abs(G2 - G) <= 1e-9 * abs(G)
    # against the oracle's cold solve: both to a residual of 1e-12
    x3, info3 = prob.solve(g, 1e-12, x=0.9 * x, warm=True)
    G3 = prob.energy(x3)
    orc = oracle.Oracle.from_workload(wl)
    _, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, 1e-12)
    e = abs(G3 - info_o["g_pol"]) / abs(info_o["g_pol"])
    _say(f"[warm] warm-started G_pol vs oracle cold solve {e:.2e} "
         f"(iters {info3['iters']} / {info_o['iters']})")
    assert info3["converged"] and e <= 1e-10


def test_zero_charges_give_the_zero_solution():
    """Degenerate input: no charges, so g = 0 and the solve returns at once."""
    wl = workloads.born_sphere(h=0.4)
    prob = ibim.Problem(wl.sdf, wl.origin, wl.h, wl.eps_tube, wl.eps_in, wl.eps_out, wl.kappa,
                        device=0)
    g = prob.rhs()
    assert torch.count_nonzero(g).item() == 0
    x, info = prob.solve(g, 1e-10)
    assert info["converged"] and info["iters"] == 0
    assert torch.count_nonzero(x).item() == 0
    assert prob.energy(x) == 0.0


def test_not_converged_is_reported():
    wl = workloads.born_sphere(h=0.4)
    prob = ibim.Problem.from_workload(wl, device=0, max_iter=3)
    x, info = prob.solve(prob.rhs(), 1e-30)
    assert info["status"] == 1 and not info["converged"] and info["iters"] == 3


def test_born_energy_near_closed_form():
    wl = workloads.born_sphere(h=0.2)
    prob = ibim.Problem.from_workload(wl, device=0)
    x, info = prob.solve_energy(1e-10)
    exact = analytic.born_energy(1.0, 2.0, wl.eps_in, wl.eps_out, wl.kappa)
    assert abs(info["g_pol"] - exact) / abs(exact) < 1e-4


# --------------------------------------------------------------------------
# full size: Kirkwood sphere R = 10, 20 charges, h = 0.25, eps = 3h
GOLDENS = {"kirkwood": "kirkwood_R10_h0.25.json", "ses500": "ses500_h0.3.json",
           "ses2000": "ses2000_h0.35.json", "ses2000_twin": "ses2000_twin_h0.7.json"}


@pytest.fixture(scope="module", params=list(GOLDENS))
def full(request):
    """Full-size workloads against stored oracle values (sampled rows and G_pol)."""
    path = os.path.join(os.path.dirname(__file__), "golden", GOLDENS[request.param])
    if not os.path.exists(path):
        pytest.skip(f"stored oracle values for {request.param} are missing")
    gold = json.load(open(path))
    wl = workloads.by_name(request.param)
    _say(f"[{request.param} full] setup")
    prob = ibim.Problem.from_workload(wl, device=0)
    return request.param, wl, prob, gold


def test_full_sizes(full):
    name, wl, prob, gold = full
    assert prob.M == gold["M"] and prob.nnz == gold["nnz"]


def test_full_sampled_apply(full):
    name, wl, prob, gold = full
    M = prob.M
    rows = np.array(gold["rows"])
    u = workloads.random_vector(2 * M, gold["u_seed"])
    out = prob.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    r1 = np.array(gold["apply_rows_1"])
    r2 = np.array(gold["apply_rows_2"])
    e1 = np.max(np.abs(out[rows] - r1)) / np.max(np.abs(r1))
    e2 = np.max(np.abs(out[M + rows] - r2)) / np.max(np.abs(r2))
    _say(f"[{name} full] sampled apply rel err {e1:.3e} {e2:.3e}")
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("precision", [ibim.FP64, ibim.MIXED])
def test_full_tree_sampled_apply(full, precision):
    """The treecode (8 points per dimension, theta 0.7; far field in float32 for
    the mixed form) on the same rows: an approximation of the exact sum,
    within 1e-6 of the largest entry."""
    name, wl, prob, gold = full
    tree = ibim.Problem.from_workload(wl, device=0, summation=ibim.SUM_TREE, precision=precision)
    M = tree.M
    rows = np.array(gold["rows"])
    u = workloads.random_vector(2 * M, gold["u_seed"])
    out = tree.apply(torch.from_numpy(u).to(DEV)).cpu().numpy()
    tree.close()
    r1 = np.array(gold["apply_rows_1"])
    r2 = np.array(gold["apply_rows_2"])
    e1 = np.max(np.abs(out[rows] - r1)) / np.max(np.abs(r1))
    e2 = np.max(np.abs(out[M + rows] - r2)) / np.max(np.abs(r2))
    _say(f"[{name} full] treecode (precision {precision}) sampled apply rel err {e1:.3e} {e2:.3e}")
    assert e1 < 1e-6 and e2 < 1e-6


def test_full_sampled_weights(full):
    name, wl, prob, gold = full
    om11, om21 = prob.correction_weights()
    cl = prob.corrections()
    # the stored entries are in the oracle's plane order: match by (row, col)
    rows = np.array(gold["rows"][:64])
    ent_col = np.array(gold["corr_col"])
    ref11 = np.array(gold["corr_om11"])
    ref21 = np.array(gold["corr_om21"])
    got11, got21 = [], []
    pos = 0
    for r in rows:
        a, b = cl["row"][r], cl["row"][r + 1]
        n = b - a
        cols = ent_col[pos:pos + n]
        for c in cols:
            idx = a + int(np.nonzero(cl["col"][a:b] == c)[0][0])
            got11.append(om11[idx])
            got21.append(om21[idx])
        pos += n
    assert pos == len(ent_col)
    assert np.max(np.abs(np.array(got11) - ref11)) < 1e-12 * np.max(np.abs(ref11))
    assert np.max(np.abs(np.array(got21) - ref21)) < 1e-12 * np.max(np.abs(ref21))


def test_full_solve(full):
    name, wl, prob, gold = full
    if "g_pol" not in gold:
        # ses2000: an oracle solve (~46 applications of 1e11 pairs) is out of
        # the oracle's reach here; its solve is pinned on the h = 0.7 twin.  At
        # full size: the right-hand side on the stored rows, and the FP64 and
        # mixed solves against each other and their explicit residuals.
        M = prob.M
        g = prob.rhs()
        rows = np.array(gold["rows"])
        gh = g.cpu().numpy()
        assert np.max(np.abs(gh[rows] - gold["rhs_rows_1"])) < 1e-13 * np.max(np.abs(gh[:M]))
        x, info = prob.solve_energy(wl.tol)
        mixed = ibim.Problem.from_workload(wl, device=0, precision=ibim.MIXED)
        xm, info_m = mixed.solve_energy(wl.tol)
        mixed.close()
        _say(f"[{name} full] fp64 iters={info['iters']} G={info['g_pol']:.15e}; "
             f"mixed iters={info_m['iters']} G={info_m['g_pol']:.15e}")
        assert info["converged"] and info_m["converged"]
        assert info["explicit_rel_resid"] < 10 * wl.tol
        assert info_m["explicit_rel_resid"] < 10 * wl.tol
        assert abs(info_m["g_pol"] - info["g_pol"]) <= 1e-6 * abs(info["g_pol"])
        return
    M = prob.M
    g = prob.rhs()
    rows = np.array(gold["rows"])
    gh = g.cpu().numpy()
    assert np.max(np.abs(gh[rows] - gold["rhs_rows_1"])) < 1e-13 * np.max(np.abs(gh[:M]))
    x, info = prob.solve(g, wl.tol)
    G = prob.energy(x)
    _say(f"[{name} full] iters={info['iters']} (oracle {gold['gmres']['iters']}) "
         f"G={G:.15e} oracle={gold['g_pol']:.15e} t={info['seconds']:.2f}s")
    assert abs(info["iters"] - gold["gmres"]["iters"]) <= 1
    assert abs(G - gold["g_pol"]) <= 1e-10 * abs(gold["g_pol"])
    xh = x.cpu().numpy()
    x1 = np.array(gold["x_rows_1"])
    assert np.max(np.abs(xh[rows] - x1)) <= 1e-9 * np.max(np.abs(x1))
    if name == "kirkwood":
        exact = analytic.kirkwood_energy(wl.charge_xyz, wl.charge_q, 10.0, wl.eps_in,
                                         wl.eps_out, wl.kappa)
        assert abs(G - exact) / abs(exact) < 1e-2  # discretisation error, not parity
