"""GPU tests of the continuous-batching solve server (``ibim_server_*``).

Every request must give bit-identical results whether it runs alone or in a
mix with other problems (the batched pair launch computes each work item as
the single-problem kernel does, and the per-request GMRES sequence is the
one of ``ibim_solve``), and the same bits as ``ibim_solve`` + ``ibim_energy``
through the single-problem entry points.  Admission must respect the HBM
budget, and a bad request must fail alone.  One energy is checked against
the FP64 oracle.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_03699_amd import ibim  # noqa: E402

GiB = 1 << 30


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# different sizes, so the batched work list mixes tile counts and ragged tails
MIX = {
    "born_h0.4": lambda: workloads.born_sphere(h=0.4),
    "offset_sphere": lambda: workloads.born_sphere(h=0.25, radius=1.7,
                                                   offset=(0.37, 0.11, -0.23)),
    "tiny_sphere": lambda: workloads.born_sphere(h=0.3, radius=0.6, eps_factor=1.5),
    "kirkwood_small": lambda: workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0,
                                                        n_charges=5, seed=7, tol=1e-10),
    "torus": lambda: workloads.torus_case(h=0.1),
    "ses_molecule": lambda: workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11, tol=1e-10),
}


@pytest.fixture(scope="module")
def wls():
    return {k: f() for k, f in MIX.items()}


def _serve(wls, names, budget=8 * GiB, slots=8, **opt):
    srv = ibim.Server(budget, max_slots=slots, host_threads=4, **opt)
    try:
        tickets = {n: srv.submit_workload(wls[n]) for n in names}
        srv.run_until_idle()
        out = {}
        for n, t in tickets.items():
            st, g, info = srv.poll(t)
            assert st == ibim.REQ_DONE, n
            out[n] = (g, srv.solution(t), info)
        return out, srv.stats()
    finally:
        srv.close()


def _direct(wl, **opt):
    prob = ibim.Problem.from_workload(wl, device=0, **opt)
    x, info = prob.solve_energy(wl.tol)
    torch.cuda.synchronize()
    out = (info["g_pol"], x.cpu().numpy(), info)
    prob.close()
    return out


def _same(a, b, name):
    ga, xa, ia = a
    gb, xb, ib = b
    assert ga == gb, f"{name}: G_pol {ga!r} != {gb!r}"
    assert np.array_equal(xa, xb), f"{name}: solutions differ (max {np.max(np.abs(xa - xb))})"
    assert ia["iters"] == ib["iters"], name
    assert ia["converged"] == ib["converged"], name


@pytest.mark.parametrize("precision,restart,hybrid", [(ibim.FP64, 60, ibim.CTR2),
                                                      (ibim.FP64, 4, ibim.CTR2),
                                                      (ibim.MIXED, 60, ibim.CTR2),
                                                      (ibim.FP64, 60, ibim.HYB)])
def test_alone_equals_mixed_equals_direct(wls, precision, restart, hybrid):
    names = list(MIX)
    _say(f"[serving] precision={precision} restart={restart} hybrid={hybrid}: mix of {len(names)}")
    mixed, stats = _serve(wls, names, precision=precision, restart=restart, hybrid=hybrid)
    _say(f"[serving] rounds={stats['rounds']} max_active={stats['max_active_seen']} "
         f"items={stats['batched_items']}")
    assert stats["finished"] == len(names) and stats["failed"] == 0
    # requests are set up on the admission threads while rounds run, so a small
    # one may finish before the last joins: the mix shares rounds, not
    # necessarily all at once
    assert stats["max_active_seen"] >= 2
    assert stats["bytes_in_use"] == 0
    for n in names:
        alone, _ = _serve(wls, [n], slots=1, precision=precision, restart=restart, hybrid=hybrid)
        _same(alone[n], mixed[n], f"{n} alone vs mix")
        direct = _direct(wls[n], precision=precision, restart=restart, hybrid=hybrid)
        _same(direct, mixed[n], f"{n} ibim_solve vs server")
        if restart >= 60:
            assert mixed[n][2]["converged"]
        _say(f"[serving] {n}: iters={mixed[n][2]['iters']} G={mixed[n][0]:.12e}")


def test_request_admitted_while_another_is_mid_solve(wls):
    """Continuous batching, not a queue: with two slots, a request submitted
    after the first has run several rounds is admitted while the first is
    still in its solve, the two share rounds, and both end with the same bits
    as when each runs alone.  The unscaled system is used so that the first
    request needs many rounds."""
    opt = dict(precond=ibim.PRECOND_NONE)
    a_name, b_name = "kirkwood_small", "born_h0.4"
    srv = ibim.Server(8 * GiB, max_slots=2, host_threads=2, **opt)
    try:
        ta = srv.submit_workload(wls[a_name])
        rounds_a = 0
        for _ in range(100000):
            srv.step()
            if srv.state(ta) == ibim.REQ_ACTIVE:
                rounds_a += 1
                if rounds_a == 3:
                    break
        assert srv.state(ta) == ibim.REQ_ACTIVE, "first request finished within three rounds"
        tb = srv.submit_workload(wls[b_name])
        # the second request's host setup, then its device setup, run on the
        # server's threads (a round hands it from one to the other, and the
        # first round after its device setup picks it up); wait for each
        # without stepping, so the first request advances only one round per wait
        for waited in range(1, 6):
            time.sleep(1.0)
            srv.step()
            sa, sb = srv.state(ta), srv.state(tb)
            _say(f"[serving] after {waited} wait(s): first {sa}, second {sb}")
            if sb != ibim.REQ_WAITING:
                break
        assert sa == ibim.REQ_ACTIVE and sb == ibim.REQ_ACTIVE
        shared = 1
        while True:
            a, w = srv.step()
            if srv.state(ta) == ibim.REQ_ACTIVE and srv.state(tb) == ibim.REQ_ACTIVE:
                shared += 1
            if a == 0 and w == 0:
                break
        _say(f"[serving] rounds shared by both requests: {shared}")
        out = {}
        for n, t in ((a_name, ta), (b_name, tb)):
            st, g, info = srv.poll(t)
            assert st == ibim.REQ_DONE, n
            out[n] = (g, srv.solution(t), info)
    finally:
        srv.close()
    for n in (a_name, b_name):
        alone, _ = _serve(wls, [n], slots=1, **opt)
        _same(alone[n], out[n], f"{n} alone vs admitted mid-solve")


@pytest.mark.parametrize("precision", [ibim.FP64, ibim.MIXED])
def test_footprint_estimates_bound_the_device_bytes(wls, precision):
    """Admission reserves each request's footprint estimate; it must bound the
    device bytes the request holds at the peak of its setup (temporaries
    included) and after it, for molecules of the serving stream's kind (the
    mixed near list included) and spheres."""
    pool = dict(wls)
    pool["ses_60_h0.5"] = workloads.ses_molecule(60, 12.0, 0.5, 2.0, seed=21, tol=1e-6)
    pool["ses_150_h0.3"] = workloads.ses_molecule(150, 17.0, 0.3, 2.0, seed=22, tol=1e-6)
    _, stats = _serve(pool, list(pool), precision=precision)
    _say(f"[serving] precision={precision}: estimate shortfall {stats['estimate_shortfall']} B, "
         f"peak {stats['bytes_peak']} B")
    assert stats["finished"] == len(pool) and stats["failed"] == 0
    assert stats["estimate_shortfall"] == 0


@pytest.mark.parametrize("precision", [ibim.FP64, ibim.MIXED])
def test_tree_requests_in_the_mix(wls, precision):
    """With IBIM_SUM_TREE and a size threshold, requests of at least
    tree_min_nodes nodes run the treecode in rounds of their own (a second
    stream, concurrent with the direct solves' rounds) and the others the
    batched direct kernel.  Every result is the same bits alone, in
    the mix and through ibim_solve with the same options, and the treecode's
    energies are within the treecode's error of the float64 direct solve."""
    pool = dict(wls)
    pool["kirkwood_r6"] = workloads.kirkwood_sphere(h=0.25, radius=6.0, r_charges=4.5,
                                                    n_charges=8, seed=3, tol=1e-8)
    sizes = {}
    for n, w in pool.items():
        p = ibim.Problem.from_workload(w, device=-1)
        sizes[n] = p.M
        p.close()
    thr = sorted(sizes.values())[len(sizes) // 2]
    opt = dict(precision=precision, summation=ibim.SUM_TREE, tree_min_nodes=thr)
    names = list(pool)
    _say(f"[serving] tree threshold {thr}: sizes {sizes}")
    mixed, stats = _serve(pool, names, **opt)
    assert stats["finished"] == len(names) and stats["failed"] == 0
    assert stats["bytes_in_use"] == 0
    n_tree = 0
    for n in names:
        p = ibim.Problem.from_workload(pool[n], device=-1, **opt)
        tree = p.summation == ibim.SUM_TREE
        p.close()
        assert tree == (sizes[n] >= thr), n
        n_tree += tree
        alone, _ = _serve(pool, [n], slots=1, **opt)
        _same(alone[n], mixed[n], f"{n} alone vs mix (tree={tree})")
        _same(_direct(pool[n], **opt), mixed[n], f"{n} ibim_solve vs server (tree={tree})")
        assert mixed[n][2]["converged"], n
        if tree:
            g64 = _direct(pool[n])[0]
            _say(f"[serving] {n}: treecode G={mixed[n][0]:.12e} direct fp64 G={g64:.12e}")
            assert abs(mixed[n][0] - g64) <= 1e-6 * abs(g64), n
    assert 0 < n_tree < len(names)


@pytest.mark.parametrize("precision", [ibim.FP64, ibim.MIXED])
def test_one_directional_requests_in_the_mix(wls, precision):
    """With a scratch cap that sends the larger requests to the one-directional
    kernels, both batched pair launches run in the same rounds; every result
    is still the same bits alone, in the mix and through ibim_solve."""
    names = list(MIX)
    sizes = {}
    for n in names:
        p = ibim.Problem.from_workload(wls[n], device=-1)
        sizes[n] = p.M
        p.close()
    # the symmetric partial sums take about T^2 (1 + 1/(2 rows)) x 4 KiB for T
    # tiles of 256 nodes: half of the largest problem's T^2 x 4 KiB sends it
    # (and only the larger problems) to the one-directional kernels
    cap = 4096 * (max(sizes.values()) // 256 + 1) ** 2 // 2
    opt = dict(precision=precision, pair_scratch_max=cap)
    onedir = {}
    for n in names:
        p = ibim.Problem.from_workload(wls[n], device=0, **opt)
        pairs, flops = p.pair_work()
        onedir[n] = flops == 60.0 * pairs  # (a one-tile problem counts 60 on either path)
        p.close()
    assert any(onedir.values()) and not all(onedir.values()), onedir
    mixed, stats = _serve(wls, names, **opt)
    _say(f"[serving one-directional cap={cap}] sizes {sizes} one-directional {onedir}")
    assert stats["finished"] == len(names) and stats["failed"] == 0
    for n in names:
        alone, _ = _serve(wls, [n], slots=1, **opt)
        _same(alone[n], mixed[n], f"{n} alone vs mix")
        _same(_direct(wls[n], **opt), mixed[n], f"{n} ibim_solve vs server")


def test_energy_matches_oracle(wls):
    wl = wls["kirkwood_small"]
    out, _ = _serve(wls, ["kirkwood_small", "born_h0.4"])
    orc = oracle.Oracle.from_workload(wl)
    _, info_o = orc.solve_energy(wl.charge_xyz, wl.charge_q, wl.tol)
    g = out["kirkwood_small"][0]
    assert abs(g - info_o["g_pol"]) <= 1e-10 * abs(info_o["g_pol"])


def test_budget_admission(wls):
    names = list(MIX)
    free, _ = _serve(wls, names)
    # the budget of the two largest footprints measured alone
    held = {}
    for n in names:
        _, st = _serve(wls, [n], slots=1)
        held[n] = st["bytes_peak"]
    budget = int(sum(sorted(held.values())[-2:]) * 1.05)
    out, st = _serve(wls, names, budget=budget)
    _say(f"[serving] budget={budget} peak={st['bytes_peak']} "
         f"max_active={st['max_active_seen']}")
    assert st["bytes_peak"] <= budget
    assert 1 <= st["max_active_seen"] < len(names)
    assert st["finished"] == len(names)
    for n in names:
        _same(out[n], free[n], f"{n} budgeted vs free")


def test_bad_requests_fail_alone(wls):
    srv = ibim.Server(8 * GiB, max_slots=4, host_threads=2)
    try:
        good = srv.submit_workload(wls["born_h0.4"])
        # no tube: the distance function never changes sign near zero
        far = wls["born_h0.4"]
        flat = np.full_like(far.sdf, 5.0)
        bad_geom = srv.submit(flat, far.origin, far.h, far.eps_tube, far.eps_in, far.eps_out,
                              far.kappa, far.charge_xyz, far.charge_q, tol=1e-8)
        bad_eps = srv.submit(far.sdf, far.origin, far.h, far.eps_tube, -1.0, far.eps_out,
                             far.kappa, far.charge_xyz, far.charge_q, tol=1e-8)
        good2 = srv.submit_workload(wls["tiny_sphere"])
        srv.run_until_idle()
        assert srv.state(bad_geom) == ibim.REQ_FAILED
        assert srv.state(bad_eps) == ibim.REQ_FAILED
        with pytest.raises(ibim.IbimError):
            srv.poll(bad_eps)
        for t, n in ((good, "born_h0.4"), (good2, "tiny_sphere")):
            st, g, info = srv.poll(t)
            assert st == ibim.REQ_DONE
            _same((g, srv.solution(t), info), _direct(wls[n]), n)
        s = srv.stats()
        assert s["failed"] == 2 and s["finished"] == 2
        srv.release(bad_geom)
        with pytest.raises(ibim.IbimError):
            srv.poll(bad_geom)
    finally:
        srv.close()
    # a request larger than the whole budget is refused, not left waiting
    srv = ibim.Server(1 << 20, max_slots=2, host_threads=1)
    try:
        t = srv.submit_workload(wls["offset_sphere"])
        srv.run_until_idle()
        assert srv.state(t) == ibim.REQ_FAILED
        with pytest.raises(ibim.IbimError) as ei:
            srv.poll(t)
        assert ei.value.code == -3
    finally:
        srv.close()
