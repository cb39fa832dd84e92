#!/usr/bin/env python
"""Benchmark of the CTR-IBIM solve on one MI355X.

One step = one complete solve on a device-resident problem: right-hand side,
GMRES to the workload's tolerance (every iteration one application of the
discrete operator: the dense pair kernel plus the sparse correction), the
explicit residual check, and the polarisation energy.  The problem setup
(signed distance on the host -> geometry, correction sets and weights on the
device) is timed separately because it consumes host buffers.

Default workload: the 2000-atom random-walk molecule (SES, 40 A box) at
h = 0.35, eps = 2h, float64 pairs, GMRES tol 1e-6.

value = pair interactions evaluated in all operator applications of the timed
steps / wall time of those steps (one pair = the four kernels for one
(target, source)).  Also reported: solves/s, per-solve latency, the dominant
kernel's roofline (60 algorithmic flops per ordered pair against the FP64
vector peak; the flops as evaluated and the VALU-counter flops beside it), a
mixed-precision leg on the same problem (solves/s, G_pol and solution error
against the FP64 solve), the oracle check of the coarsened h = 0.7 twin and
the oracle's own rates on the host.

Prints ONE JSON line.  ``--gpus`` above 1 is refused: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s in IBIM matvec; solves/s + p50/p99 latency at fixed error"
PEAK_FP64_VECTOR_TFLOPS = 78.6  # MI355X vector FP64
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X vector FP32 (counts packed float32 issue)


FLOPS_PER_PAIR = 60  # algorithmic flops of the four kernels for one ordered pair (FMA = 2)

# Counter figures of the dominant pair kernel, per (precision, workload), from
# the rocprofv3 summaries under profiles/: HBM bytes per launch (FETCH_SIZE and
# WRITE_SIZE, KiB per dispatch, scaled by what they read for a plain 256 MiB
# copy: 2.0 and 1.0), VALU flops per launch (SQ_INSTS_VALU_FLOPS_FP64 or _FP32
# x 64 lanes) and the average duration of the counted dispatches.  Valid only
# while the kernel sources' code (kernel_digest) hashes to the recorded digest;
# otherwise null.
MEASURED_COUNTERS = {
    ("fp64", "ses2000"): {"digest": "f5d34556",
                          "traffic_bytes": 1292402 * 1024 * 2.0 + 893624 * 1024,
                          "valu_flops": 71854568164 * 64, "ms": 107.57,
                          "source": "profiles/pair_sym_fp64_ses2000_h0.35.md"},
    ("mixed", "ses2000"): {"digest": "cc6f608c",
                           "traffic_bytes": 674207 * 1024 * 2.0 + 893624 * 1024,
                           "valu_flops": 50425253732 * 64, "ms": 56.84,
                           "source": "profiles/pair_sym_mixed_ses2000_h0.35.md"},
}
# stored oracle results (tests/golden/make_golden.py) per workload
GOLDEN = {"kirkwood": "kirkwood_R10_h0.25.json", "ses500": "ses500_h0.3.json",
          "ses2000": "ses2000_h0.35.json"}
KERNEL_SOURCES = {
    "fp64": ["operator.h", "symmetric.hip", "symmetric.h", "sym_core.h", "pair_math.h",
             "fastmath.h"],
    "mixed": ["operator.h", "symmetric_mixed.hip", "symmetric.h", "sym_core.h", "pair_math.h",
              "fastmath.h"],
}


def kernel_digest(precision):
    """Hash of the kernel sources' code: comments removed and whitespace runs
    collapsed, so that a comment edit keeps the counters of unchanged code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[precision]:
        with open(os.path.join(ROOT, "paper_2210_03699_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:8]


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(wl, M, seconds):
    """The FP64 oracle on a bounded, seeded sample of rows of the same operator."""
    import numpy as np

    import oracle
    import workloads

    rng = np.random.Generator(np.random.PCG64(4242))
    # probe with a small sample, then size the timed sample to ~`seconds`
    probe_rows = np.sort(rng.choice(M, size=min(M, 64), replace=False))
    orc = oracle.Oracle.from_workload(wl, weight_rows=probe_rows)
    u = workloads.random_vector(2 * M, 4243)
    t = time.perf_counter()
    orc.apply_rows(u, probe_rows)
    rate = len(probe_rows) * M / max(time.perf_counter() - t, 1e-6)
    n = int(min(M, max(64, seconds * rate / M)))
    rows = np.sort(rng.choice(M, size=n, replace=False))
    orc = oracle.Oracle.from_workload(wl, weight_rows=rows)
    t = time.perf_counter()
    orc.apply_rows(u, rows)
    dt = time.perf_counter() - t
    return {
        "value": n * M / dt,
        "unit": "pair-interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"operator rows: {n} seeded target rows x all {M} sources "
                  f"({n * M:.3e} pairs, {dt:.1f} s)",
    }


def serve_bench(args):
    """Serving benchmark: a seeded stream of independent solve requests
    (spheres and random-walk molecules at several grid spacings) through the
    continuous-batching server.  First a closed batch measures the capacity
    (solves/s); then the same requests arrive as a Poisson stream at 0.9x
    that rate and the latency arrival -> G_pol available is recorded."""
    import numpy as np

    import workloads
    from paper_2210_03699_amd import (FP64, MIXED, REQ_DONE, REQ_FAILED, SUM_DIRECT, SUM_TREE,
                                      Server)

    mode = FP64 if args.precision == "fp64" else MIXED
    summation = SUM_TREE if args.summation == "tree" else SUM_DIRECT
    hs = tuple(float(v) for v in args.hs.split(","))
    atoms = tuple(int(v) for v in args.ses_atoms.split(","))
    t = time.perf_counter()
    def progress(i, wl):
        if i % 16 == 15 or i + 1 == args.requests:
            print(f"[serve] made {i + 1}/{args.requests} requests "
                  f"({time.perf_counter() - t:.0f}s)", file=sys.stderr, flush=True)

    reqs = workloads.serving_stream(args.requests, seed=4, hs=hs, ses_atoms=atoms,
                                    progress=progress)
    t_gen = time.perf_counter() - t
    print(f"[serve] generated {len(reqs)} requests in {t_gen:.1f}s", file=sys.stderr, flush=True)
    budget = int(args.hbm_budget_gib * (1 << 30))

    def run(arrivals):
        srv = Server(budget, max_slots=args.slots, host_threads=args.host_threads,
                     precision=mode, summation=summation, tree_order=args.tree_order,
                     tree_theta=args.tree_theta, tree_min_nodes=args.tree_min_nodes)
        order = np.argsort(arrivals, kind="stable")
        tickets, t_arr, t_done = {}, {}, {}
        nxt = 0
        t0 = time.perf_counter()
        t_report = t0
        while nxt < len(order) or len(t_done) < len(order):
            if time.perf_counter() - t_report > 15.0:
                t_report = time.perf_counter()
                print(f"[serve] {t_report - t0:.0f}s: {nxt} submitted, {len(t_done)} done",
                      file=sys.stderr, flush=True)
            now = time.perf_counter() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                tickets[i] = srv.submit_workload(reqs[i])
                t_arr[i] = t0 + arrivals[i]
                nxt += 1
            active, waiting = srv.step() if tickets else (0, 0)
            now_abs = time.perf_counter()
            for i, tk in tickets.items():
                if i not in t_done and srv.state(tk) in (REQ_DONE, REQ_FAILED):
                    t_done[i] = now_abs
            if active == 0 and waiting == 0 and nxt < len(order):
                time.sleep(max(0.0, arrivals[order[nxt]] - (time.perf_counter() - t0)))
        makespan = max(t_done.values()) - t0
        res = []
        for i, tk in tickets.items():
            st, g, info = srv.poll(tk)
            assert st == REQ_DONE, f"request {i} did not finish"
            M = len(srv.solution(tk)) // 2
            res.append({"i": i, "M": M, "applies": info["applies"], "iters": info["iters"],
                        "latency": t_done[i] - t_arr[i], "g_pol": g})
        stats = srv.stats()
        srv.close()
        return makespan, res, stats

    # closed batch: capacity
    mk, res, st = run(np.zeros(len(reqs)))
    capacity = len(reqs) / mk
    print(f"[serve] closed batch: {len(reqs)} solves in {mk:.2f}s -> {capacity:.2f} solves/s, "
          f"max active {st['max_active_seen']}", file=sys.stderr, flush=True)
    # open loop at 0.9x capacity
    rate = 0.9 * capacity
    rng = np.random.Generator(np.random.PCG64(4))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    arrivals -= arrivals[0]
    mk2, res2, st2 = run(arrivals)
    lat = [r["latency"] for r in res2]
    pairs = sum(float(r["applies"]) * r["M"] * r["M"] for r in res2)
    Ms = sorted(r["M"] for r in res2)
    n_tree = sum(1 for m in Ms if summation == SUM_TREE and m >= args.tree_min_nodes)
    out = {
        "metric": METRIC,
        "value": pairs / mk2,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": mk2 / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"serving_stream_{len(reqs)}", "seed": 4, "tol": 1e-6,
            "spheres": "R~U[2,10], 1..30 charges", "ses": f"{atoms[0]}..{atoms[1]} atoms",
            "h": list(hs), "eps_tube": "2h", "slots": args.slots,
            "hbm_budget_gib": args.hbm_budget_gib, "pair_kernel": args.precision,
            "summation": args.summation,
            **({"tree_min_nodes": args.tree_min_nodes, "tree_order": args.tree_order,
                "tree_theta": args.tree_theta, "tree_requests": n_tree,
                "pairs": "M^2 per application whichever summation"}
               if summation == SUM_TREE else {}),
            "M_min": Ms[0], "M_median": Ms[len(Ms) // 2], "M_max": Ms[-1],
            "M_p10_p90": [percentile(Ms, 10), percentile(Ms, 90)],
            "requests_by_h": {str(hh): sum(1 for w in reqs if w.h == hh) for hh in hs},
            "ses_requests": sum(1 for w in reqs if w.meta.get("geometry") == "ses"),
            "input_generation_s": t_gen,
        },
        "solves_per_s": len(reqs) / mk2,
        "capacity_solves_per_s": capacity,
        "arrival_rate_per_s": rate,
        "latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3},
        "closed_batch_latency_ms": {
            "p50": percentile([r["latency"] for r in res], 50) * 1e3,
            "p99": percentile([r["latency"] for r in res], 99) * 1e3},
        "rounds": st2["rounds"],
        "max_active": st2["max_active_seen"],
        "bytes_peak": st2["bytes_peak"],
        # admission passes that held a set-up request back (closed batch, Poisson run)
        "held_for_slot": [st["held_for_slot"], st2["held_for_slot"]],
        "held_for_budget": [st["held_for_budget"], st2["held_for_budget"]],
        "bytes_peak_closed_batch": st["bytes_peak"],
    }
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_solve_baseline():
    """One complete oracle solve (setup + GMRES + G_pol) of the Born ion, the
    smallest configuration (sphere R = 2, h = 0.2, tol 1e-10, M = 5,020)."""
    import oracle
    import workloads

    wl = workloads.born_sphere()
    t = time.perf_counter()
    orc = oracle.Oracle.from_workload(wl)
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    _, info = orc.solve_energy(wl.charge_xyz, wl.charge_q, wl.tol)
    t_solve = time.perf_counter() - t
    return wl, {"workload": wl.name, "M": orc.M, "setup_s": t_setup, "solve_s": t_solve,
                "solves_per_s": 1.0 / t_solve, "iters": info["iters"], "g_pol": info["g_pol"]}


def measured_profile(precision, workload):
    """Counter figures of the dominant pair kernel from profiles/, valid while
    the kernel sources' code hashes to the digest they were taken with."""
    rec = MEASURED_COUNTERS.get((precision, workload))
    if rec is None or kernel_digest(precision) != rec["digest"]:
        return None
    return rec


def timed_solves(prob, tol, steps, warmup, label):
    """warmup + steps complete solves (rhs, GMRES, explicit residual, G_pol)."""
    import torch

    def step():
        g = prob.rhs()
        x, info = prob.solve(g, tol)
        G = prob.energy(x)  # synchronises the stream
        return x, info, G

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    prob.pair_timing(True)
    lat, applies, iters, x, G = [], 0, [], None, None
    t_start = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        x, info, G = step()
        lat.append(time.perf_counter() - ts)
        applies += info["applies"]
        iters.append(info["iters"])
        print(f"[bench] {label} step {i}: {lat[-1] * 1e3:.1f} ms iters={info['iters']} "
              f"G_pol={G:.12e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_launch, pair_ms = prob.pair_timing_read()
    prob.pair_timing(False)
    return {"elapsed": elapsed, "lat": lat, "applies": applies, "iters": iters, "x": x, "G": G,
            "pair_ms": pair_ms / max(n_launch, 1), "n_launch": n_launch}


def block_errors(x, ref, M):
    """Max and RMS error of the psi and psi_n blocks relative to the largest
    entry of the reference block."""
    out = {}
    for name, sl in (("psi", slice(0, M)), ("psi_n", slice(M, 2 * M))):
        d = x[sl] - ref[sl]
        s = max(float(abs(ref[sl]).max()), 1e-300)
        out[name] = {"max_rel": float(abs(d).max()) / s,
                     "rms_rel": float((d * d).mean() ** 0.5) / s}
    return out


def twin_check(args):
    """FP64 and mixed solves of the 2000-atom molecule on the coarsened
    h = 0.7 grid against the stored oracle solve (G_pol, sampled solution rows)."""
    import numpy as np

    import workloads
    from paper_2210_03699_amd import FP64, MIXED, Problem

    path = os.path.join(ROOT, "tests", "golden", "ses2000_twin_h0.7.json")
    gold = json.load(open(path))
    wl = workloads.by_name("ses2000_twin")
    rows = np.asarray(gold["rows"], dtype=np.int64)
    xr1, xr2 = np.asarray(gold["x_rows_1"]), np.asarray(gold["x_rows_2"])
    out = {"workload": wl.name, "M": gold["M"], "oracle_g_pol": gold["g_pol"],
           "oracle_iters": gold["gmres"]["iters"]}
    for label, mode in (("fp64", FP64), ("mixed", MIXED)):
        prob = Problem.from_workload(wl, device=0, precision=mode)
        x, info = prob.solve_energy(wl.tol)
        xh = x.cpu().numpy()
        M = prob.M
        out[label] = {
            "iters": info["iters"],
            "g_pol": info["g_pol"],
            "g_pol_rel_err_vs_oracle": abs(info["g_pol"] - gold["g_pol"]) / abs(gold["g_pol"]),
            "psi_rows_max_rel_err_vs_oracle":
                float(np.max(np.abs(xh[rows] - xr1)) / np.max(np.abs(xr1))),
            "psi_n_rows_max_rel_err_vs_oracle":
                float(np.max(np.abs(xh[M + rows] - xr2)) / np.max(np.abs(xr2))),
        }
        prob.close()
    return out


def rnear_sweep(args):
    """Mixed form: G_pol and surface-potential error against the stored oracle
    solves and time per solve, for near radii r_near = 1h, 2h, 3h, 4h (and the
    FP64 solve for reference), on the 500-atom molecule and the 2000-atom
    molecule's h = 0.7 twin."""
    import numpy as np
    import torch

    import workloads
    from paper_2210_03699_amd import FP64, MIXED, Problem

    out = {"metric": "mixed-form error and time per solve against r_near", "cases": []}
    for name, gname in (("ses500", "ses500_h0.3.json"), ("ses2000_twin", "ses2000_twin_h0.7.json")):
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", gname)))
        wl = workloads.by_name(name)
        rows = np.asarray(gold["rows"], dtype=np.int64)
        xr1, xr2 = np.asarray(gold["x_rows_1"]), np.asarray(gold["x_rows_2"])
        for f in (0.0, 1.0, 2.0, 3.0, 4.0):
            prec = FP64 if f == 0.0 else MIXED
            t0 = time.perf_counter()
            prob = Problem.from_workload(wl, device=0, precision=prec, r_near=f * wl.h)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            times = []
            for rep in range(3):
                t0 = time.perf_counter()
                x, info = prob.solve_energy(wl.tol)
                times.append(time.perf_counter() - t0)
            xh = x.cpu().numpy()
            M = prob.M
            rec = {"workload": wl.name, "M": M, "precision": "fp64" if f == 0.0 else "mixed",
                   "r_near_over_h": f, "setup_s": t_setup, "solve_s": min(times),
                   "iters": info["iters"],
                   "g_pol_rel_err_vs_oracle":
                       abs(info["g_pol"] - gold["g_pol"]) / abs(gold["g_pol"]),
                   "psi_rows_max_rel_err":
                       float(np.max(np.abs(xh[rows] - xr1)) / np.max(np.abs(xr1))),
                   "psi_n_rows_max_rel_err":
                       float(np.max(np.abs(xh[M + rows] - xr2)) / np.max(np.abs(xr2)))}
            print(f"[rnear] {json.dumps(rec)}", file=sys.stderr, flush=True)
            out["cases"].append(rec)
            prob.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ses2000",
                    help="named workload (workloads.by_name); default: the 2000-atom SES "
                         "molecule at h = 0.35, the largest single-GPU configuration")
    ap.add_argument("--rows", default="ctr2", choices=["ctr2", "hyb", "kreg"],
                    help="quadrature of the rows: CTR2 everywhere, HYB-IBIM (K-reg rows at "
                         "bad nodes), or K-reg everywhere")
    ap.add_argument("--unscaled", action="store_true",
                    help="GMRES on A x = b as written instead of the row-scaled system")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64: float64 pairs; mixed: float32 pairs with float64 sums, "
                         "float64 near pairs, weights and Krylov")
    ap.add_argument("--summation", default="direct", choices=["direct", "tree"],
                    help="dense pair sum: every pair (default) or the treecode (with --precision "
                         "mixed its far field in float32; value then counts the M^2 pairs each "
                         "application stands for)")
    ap.add_argument("--tree-order", type=int, default=8)
    ap.add_argument("--tree-theta", type=float, default=0.7)
    ap.add_argument("--mixed-steps", type=int, default=5,
                    help="timed solves of the mixed-precision leg (after one warm-up solve)")
    ap.add_argument("--no-mixed-leg", action="store_true")
    ap.add_argument("--no-twin", action="store_true",
                    help="skip the oracle check on the h = 0.7 twin of the 2000-atom molecule")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: 3 operator applications and one plain "
                         "256 MiB device copy (the reference for the HBM byte counters)")
    ap.add_argument("--rnear-sweep", action="store_true",
                    help="mixed form: error against the stored oracle solves and time per solve "
                         "for r_near = h, 2h, 3h, 4h on the 500-atom molecule and the h = 0.7 twin")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: a seeded stream of independent requests through "
                         "the continuous-batching server (p50/p99 latency, solves/s)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--host-threads", type=int, default=8)
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0)
    ap.add_argument("--hs", default="0.2,0.3,0.5",
                    help="--serve: grid spacings the stream draws from (comma list)")
    ap.add_argument("--ses-atoms", default="50,2000",
                    help="--serve: atom-count range of the stream's molecules")
    ap.add_argument("--tree-min-nodes", type=int, default=0,
                    help="with --summation tree: requests below this many nodes keep the "
                         "direct sum (and --precision)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.rnear_sweep:
        rnear_sweep(args)
        return

    import numpy as np
    import torch

    import workloads
    from paper_2210_03699_amd import (CTR2, FP64, HYB, KREG, MIXED, PRECOND_DIAG, PRECOND_NONE,
                                      SUM_DIRECT, SUM_TREE, Problem)

    t0 = time.perf_counter()
    wl = workloads.by_name(args.workload)
    input_s = time.perf_counter() - t0
    dev = "cuda:0"
    torch.cuda.synchronize()
    mode = FP64 if args.precision == "fp64" else MIXED
    rows = {"ctr2": CTR2, "hyb": HYB, "kreg": KREG}[args.rows]
    precond = PRECOND_NONE if args.unscaled else PRECOND_DIAG
    tree = args.summation == "tree"
    kw = dict(device=0, hybrid=rows, precond=precond,
              summation=SUM_TREE if tree else SUM_DIRECT, tree_order=args.tree_order,
              tree_theta=args.tree_theta)
    t0 = time.perf_counter()
    prob = Problem.from_workload(wl, precision=mode, **kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    M = prob.M
    print(f"[bench] {wl.name}: M={M} nnz={prob.nnz} input {input_s:.1f}s setup {setup_s:.2f}s",
          file=sys.stderr, flush=True)

    if args.profile:
        u = torch.from_numpy(workloads.random_vector(2 * M, 1)).to(dev)
        for _ in range(3):
            prob.apply(u)
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": True, "M": M, "copy_bytes": src.numel() * 8}), flush=True)
        return

    r = timed_solves(prob, wl.tol, args.steps, args.warmup, args.precision)
    elapsed, lat = r["elapsed"], r["lat"]
    pairs = float(r["applies"]) * M * M
    avg_pair_ms = r["pair_ms"]
    peak = PEAK_FP64_VECTOR_TFLOPS if args.precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    _, performed_flops = prob.pair_work()
    alg_flops = FLOPS_PER_PAIR * float(M) * M
    achieved = alg_flops / (avg_pair_ms * 1e-3) / 1e12
    prof = None if tree else measured_profile(args.precision, args.workload)
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": prof["traffic_bytes"] if prof else None,
        "kernel": "pair_sym_fp64_kernel" if args.precision == "fp64" else "pair_sym_mixed_kernel",
        "flops_per_launch": alg_flops,
        "flop_count": f"algorithmic: {FLOPS_PER_PAIR} flops per ordered pair x M^2 ordered pairs",
        "launch_ms": avg_pair_ms,
        "performed": {
            "flops_per_launch": performed_flops,
            "achieved": performed_flops / (avg_pair_ms * 1e-3) / 1e12,
            "frac": performed_flops / (avg_pair_ms * 1e-3) / 1e12 / peak,
            "flop_count": "as evaluated: 68 per shared evaluation of both directions of a pair "
                          "(66 in Debye units), "
                          "60 per one-directional pair (diagonal, corrected and ragged tiles)"},
        "valu_counter": None if prof is None else {
            "flops_per_launch": prof["valu_flops"],
            "launch_ms": prof["ms"],
            "achieved": prof["valu_flops"] / (prof["ms"] * 1e-3) / 1e12,
            "frac": prof["valu_flops"] / (prof["ms"] * 1e-3) / 1e12 / peak,
            "source": prof["source"]},
    }
    out = {
        "metric": METRIC,
        "value": pairs / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "M": M, "unknowns": 2 * M, "h": wl.h, "eps_tube": wl.eps_tube,
            "tol": wl.tol, "n_charges": int(wl.charge_q.shape[0]), "gmres_restart": 60,
            "gmres_system": "A x = b" if args.unscaled else "Lambda^-1 A x = Lambda^-1 b",
            "rows": args.rows,
            "pair_kernel": args.precision,
            "summation": args.summation,
        },
        "solves_per_s": args.steps / elapsed,
        "latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3},
        "gmres_iters": r["iters"],
        "applies_per_solve": r["applies"] / args.steps,
        "pair_kernel_ms": avg_pair_ms,
        "pair_kernel_pairs_per_s": float(M) * M / (avg_pair_ms * 1e-3),
        "input_s": input_s,
        "setup_s": setup_s,
        "g_pol": r["G"],
        "roofline": roofline,
    }
    if tree:
        tc = prob.tree_counts()
        out["config"]["tree"] = {"order": args.tree_order, "theta": args.tree_theta,
                                 "batches": tc["batches"], "proxy_clusters": tc["proxy_clusters"]}
        ev = tc["far_evals"] + tc["near_evals"]
        out["tree_evaluations_per_apply"] = {k: tc[k] for k in ("far_evals", "near_evals",
                                                                "proxy_terms")}
        out["tree_evaluations_per_s"] = ev / (avg_pair_ms * 1e-3)
    golden = os.path.join(ROOT, "tests", "golden", GOLDEN.get(args.workload, "-"))
    if os.path.exists(golden):
        gold = json.load(open(golden))
        if "g_pol" in gold:
            out["g_pol_rel_err_vs_oracle"] = abs(r["G"] - gold["g_pol"]) / abs(gold["g_pol"])
        else:
            # sampled operator rows of the stored oracle values (no full oracle solve)
            grows = np.asarray(gold["rows"], dtype=np.int64)
            u = torch.from_numpy(workloads.random_vector(2 * M, gold["u_seed"])).to(dev)
            Au = prob.apply(u).cpu().numpy()
            a1, a2 = np.asarray(gold["apply_rows_1"]), np.asarray(gold["apply_rows_2"])
            out["apply_rows_rel_err_vs_oracle"] = max(
                float(np.max(np.abs(Au[grows] - a1)) / np.max(np.abs(a1))),
                float(np.max(np.abs(Au[M + grows] - a2)) / np.max(np.abs(a2))))
    x64 = r["x"].cpu().numpy()

    if args.precision == "fp64" and not tree and not args.no_mixed_leg:
        # the mixed form on the same problem: speed and its error against FP64
        prob.close()
        del prob
        torch.cuda.empty_cache()
        pm = Problem.from_workload(wl, precision=MIXED, **kw)
        rm = timed_solves(pm, wl.tol, args.mixed_steps, 1, "mixed")
        xm = rm["x"].cpu().numpy()
        mixed = {
            "solves_per_s": args.mixed_steps / rm["elapsed"],
            "ms_per_solve": rm["elapsed"] / args.mixed_steps * 1e3,
            "speedup_vs_fp64_solves": (args.mixed_steps / rm["elapsed"]) / out["solves_per_s"],
            "gmres_iters": rm["iters"],
            "pair_kernel_ms": rm["pair_ms"],
            "pair_kernel_pairs_per_s": float(M) * M / (rm["pair_ms"] * 1e-3),
            "frac_fp32_vector_peak": FLOPS_PER_PAIR * float(M) * M / (rm["pair_ms"] * 1e-3)
                                     / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
            "g_pol": rm["G"],
            "g_pol_rel_err_vs_fp64": abs(rm["G"] - r["G"]) / abs(r["G"]),
            "solution_err_vs_fp64": block_errors(xm, x64, M),
        }
        mp = measured_profile("mixed", args.workload)
        if mp is not None:
            mixed["valu_counter_fp32_tflops"] = mp["valu_flops"] / (mp["ms"] * 1e-3) / 1e12
            mixed["traffic"] = mp["traffic_bytes"]
        out["mixed"] = mixed
        pm.close()
        del pm
        torch.cuda.empty_cache()
    if args.workload == "ses2000" and not args.no_twin:
        print("[bench] twin h = 0.7 against the stored oracle solve", file=sys.stderr, flush=True)
        out["twin_h0.7"] = twin_check(args)
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        cb = cpu_baseline(wl, M, args.cpu_seconds)
        cb["cpu_model"] = cpu_model()
        # the oracle's solve rate on this workload, from its measured pair rate
        cb["oracle_solve_s_estimated"] = r["applies"] / args.steps * M * M / cb["value"]
        bwl, ob = oracle_solve_baseline()
        # the same Born-ion solve on the GPU, for the solves/s comparison
        pb = Problem.from_workload(bwl, device=0)
        rb = timed_solves(pb, bwl.tol, 20, 2, "born")
        ob["gpu_solves_per_s"] = 20 / rb["elapsed"]
        ob["gpu_g_pol"] = rb["G"]
        cb["oracle_solve_born"] = ob
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
