"""Write the stored oracle values for the full-size Kirkwood workload.

Calls only ``oracle`` and ``workloads``.  Output: ``kirkwood_R10_h0.25.json``
beside this script.  The full oracle solve at this size (~1.2e5 tube nodes,
1.45e10 pair evaluations per operator application) takes about an hour on
eight cores, so its results are stored instead of recomputed in every test.

Usage: python tests/golden/make_golden.py
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


def main():
    wl = workloads.by_name("kirkwood")
    t0 = time.time()
    o = oracle.Oracle.from_workload(wl)
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
    t0 = time.time()
    x, info = o.gmres(g, wl.tol, restart=60, maxit=300)
    t_solve = time.time() - t0
    gpol = o.energy(x, wl.charge_xyz, wl.charge_q)
    print(f"solve {t_solve:.1f}s info={info} gpol={gpol!r}", flush=True)
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
        "gmres": {"tol": wl.tol, "restart": 60, **info},
        "g_pol": gpol,
        "x_rows_1": x[rows].tolist(),
        "x_rows_2": x[M + rows].tolist(),
        "oracle_seconds": {"setup": t_setup, "sampled_apply": t_rows, "solve": t_solve,
                           "threads": oracle.num_threads()},
    }
    path = os.path.join(HERE, "kirkwood_R10_h0.25.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print("wrote", path)


def workloads_random_vector(n, seed):
    return workloads.random_vector(n, seed)


if __name__ == "__main__":
    main()
