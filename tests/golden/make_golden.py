"""Write the stored oracle values for the full-size workloads.

Calls only ``oracle`` and ``workloads``.  Outputs beside this script:
``kirkwood_R10_h0.25.json`` (Kirkwood sphere), ``ses500_h0.3.json``
(500-atom molecule), ``ses2000_twin_h0.7.json`` (the 2000-atom molecule on
the coarsened h = 0.7 grid) and, with --no-solve, ``ses2000_h0.35.json``
(sampled rows only).  A full oracle solve at these sizes (1.2e5-1.3e5 tube nodes,
~1.5e10 pair evaluations per operator application) takes 30-60 minutes on
eight cores, so the results are stored instead of recomputed in every test.

Usage: python tests/golden/make_golden.py [kirkwood|ses500|ses2000|ses2000_twin] [--no-solve]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

N_SAMPLE = 256
SEED_ROWS = 77
SEED_U = 78


OUTPUT = {"kirkwood": "kirkwood_R10_h0.25.json", "ses500": "ses500_h0.3.json",
          "ses2000": "ses2000_h0.35.json", "ses2000_twin": "ses2000_twin_h0.7.json"}


def main():
    name = sys.argv[1] if len(sys.argv) > 1 and not sys.argv[1].startswith("-") else "kirkwood"
    solve = "--no-solve" not in sys.argv
    wl = workloads.by_name(name)
    t0 = time.time()
    rng = np.random.Generator(np.random.PCG64(SEED_ROWS))
    if solve:
        o = oracle.Oracle.from_workload(wl)
    else:
        # weights only at the sampled rows (the other rows are never applied)
        o0 = oracle.Oracle.from_workload(wl, weight_rows=np.zeros(1, dtype=np.int64))
        rows0 = np.sort(rng.choice(o0.M, size=N_SAMPLE, replace=False))
        rng = np.random.Generator(np.random.PCG64(SEED_ROWS))
        o = oracle.Oracle.from_workload(wl, weight_rows=rows0)
    t_setup = time.time() - t0
    M = o.M
    print(f"M={M} nnz={o.nnz} setup {t_setup:.1f}s threads={oracle.num_threads()}", flush=True)
    rng = np.random.Generator(np.random.PCG64(SEED_ROWS))
    rows = np.sort(rng.choice(M, size=N_SAMPLE, replace=False))
    u = workloads_random_vector(2 * M, SEED_U)
    t0 = time.time()
    a1, a2 = o.apply_rows(u, rows)
    t_rows = time.time() - t0
    print(f"sampled apply {t_rows:.1f}s", flush=True)
    g = o.rhs(wl.charge_xyz, wl.charge_q)
    corr = o.corrections()
    sel = []
    for r in rows[:64]:
        for e in range(corr["row"][r], corr["row"][r + 1]):
            sel.append(e)
    sel = np.array(sel, dtype=np.int64)
    out = {
        "workload": wl.describe(),
        "M": M,
        "nnz": o.nnz,
        "area": o.area(),
        "rows": rows.tolist(),
        "u_seed": SEED_U,
        "apply_rows_1": a1.tolist(),
        "apply_rows_2": a2.tolist(),
        "rhs_rows_1": g[rows].tolist(),
        "rhs_rows_2": g[M + rows].tolist(),
        "corr_entries": sel.tolist(),
        "corr_col": corr["col"][sel].tolist(),
        "corr_om11": corr["om11"][sel].tolist(),
        "corr_om21": corr["om21"][sel].tolist(),
        "oracle_seconds": {"setup": t_setup, "sampled_apply": t_rows,
                           "threads": oracle.num_threads()},
    }
    if solve:
        t0 = time.time()
        x, info = o.gmres(g, wl.tol, restart=60, maxit=300, precond=1)
        t_solve = time.time() - t0
        gpol = o.energy(x, wl.charge_xyz, wl.charge_q)
        print(f"solve {t_solve:.1f}s info={info} gpol={gpol!r}", flush=True)
        out["gmres"] = {"tol": wl.tol, "restart": 60, "precond": 1, **info}
        out["g_pol"] = gpol
        out["x_rows_1"] = x[rows].tolist()
        out["x_rows_2"] = x[M + rows].tolist()
        out["oracle_seconds"]["solve"] = t_solve
    path = os.path.join(HERE, OUTPUT[name])
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print("wrote", path)


def workloads_random_vector(n, seed):
    return workloads.random_vector(n, seed)


if __name__ == "__main__":
    main()
