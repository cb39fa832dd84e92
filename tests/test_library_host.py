"""Host-side checks of the HIP library (no GPU needed).

* the shared library loads and exports every function ``include/ibim.h``
  declares;
* the host part of the setup (tube nodes, geometry, correction sets) agrees
  with the oracle: the sets N_h(y_k) and their shifts exactly, the weights w
  to rounding;
* argument and geometry errors come back as the documented codes.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from paper_2210_03699_amd import ibim


def test_library_exports_every_header_function():
    lib = ibim.load()
    names = ibim.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def _compare(wl, hybrid=ibim.CTR2):
    lib = ibim.Problem.from_workload(wl, device=-1, hybrid=hybrid)
    orc = oracle.Oracle.from_workload(wl, hybrid=hybrid)
    assert lib.M == orc.M and lib.nnz == orc.nnz
    assert np.array_equal(lib.node_flags(), orc.bad_nodes())
    nd = orc.nodes()
    gi = lib.node_grid_index()
    ny, nz = wl.sdf.shape[1], wl.sdf.shape[2]
    assert np.array_equal(gi, (nd["ijk"][:, 0].astype(np.int64) * ny + nd["ijk"][:, 1]) * nz
                          + nd["ijk"][:, 2])
    P, n, w = lib.node_geometry()
    assert np.array_equal(P, nd["P"])          # same IEEE expression order
    assert np.array_equal(n, nd["n"])
    assert np.max(np.abs(w - nd["w"])) <= 1e-13 * np.max(nd["w"])
    cl, co = lib.corrections(), orc.corrections()
    assert np.array_equal(cl["row"], co["row"])
    for k in range(lib.M):
        a, b = slice(cl["row"][k], cl["row"][k + 1]), slice(co["row"][k], co["row"][k + 1])
        order = np.argsort(co["col"][b], kind="stable")
        assert np.array_equal(cl["col"][a], co["col"][b][order])
        for key in ("axis", "alpha", "beta", "eta"):
            assert np.array_equal(cl[key][a], co[key][b][order]), (k, key)
    return lib, orc


def test_host_setup_matches_oracle_centered_sphere():
    _compare(workloads.born_sphere(h=0.2))


def test_host_setup_matches_oracle_offset_sphere():
    _compare(workloads.born_sphere(h=0.25, radius=1.7, offset=(0.37, 0.11, -0.23)))


def test_host_setup_matches_oracle_torus():
    _compare(workloads.torus_case(h=0.1))


def test_host_setup_matches_oracle_wide_tube():
    _compare(workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0, n_charges=3))


def test_host_setup_matches_oracle_ses_molecule():
    _compare(workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11))


def test_hybrid_sets_match_oracle_ses_molecule():
    """HYB-IBIM: bad-node flags, K-reg sets (axis -1) and J = 1 weights agree."""
    lib, orc = _compare(workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11), hybrid=ibim.HYB)
    bad = orc.bad_nodes()
    assert 0 < bad.sum() < 0.2 * lib.M
    cl = lib.corrections()
    rows = np.repeat(np.arange(lib.M), np.diff(cl["row"]))
    assert np.all((cl["axis"] < 0) == bad[rows])


def test_kreg_everywhere_matches_oracle_sphere():
    lib, orc = _compare(workloads.born_sphere(h=0.4), hybrid=ibim.KREG)
    assert lib.node_flags().all()
    assert np.all(lib.corrections()["axis"] == -1)


def test_hybrid_flags_no_node_on_smooth_surfaces():
    for wl in (workloads.born_sphere(h=0.2), workloads.torus_case(h=0.1),
               workloads.kirkwood_sphere(h=0.3, radius=3.0, r_charges=2.0, n_charges=5, seed=7)):
        p = ibim.Problem.from_workload(wl, device=-1, hybrid=ibim.HYB)
        assert not p.node_flags().any(), wl.name


def test_every_row_corrects_its_own_node():
    lib = ibim.Problem.from_workload(workloads.born_sphere(h=0.2), device=-1)
    c = lib.corrections()
    for k in range(lib.M):
        assert k in set(c["col"][c["row"][k]:c["row"][k + 1]])


def _raw_setup(sdf, origin, h, eps, kappa=0.1, device=-1):
    lib = ibim.load()
    opt = ibim._Options()
    lib.ibim_default_options(ctypes.byref(opt))
    opt.device = device
    ctx = ctypes.c_void_p()
    sdf = np.ascontiguousarray(sdf)
    origin = np.ascontiguousarray(origin, dtype=np.float64)
    zq = np.zeros(3)
    q = np.ones(1)
    code = lib.ibim_setup(ibim._dp(sdf), sdf.shape[0], sdf.shape[1], sdf.shape[2],
                          ibim._dp(origin), h, eps, 1.0, 80.0, kappa, ibim._dp(zq), ibim._dp(q), 1,
                          ctypes.byref(opt), None, ctypes.byref(ctx))
    return code, ctx


def test_error_codes():
    lib = ibim.load()
    sdf, org = workloads.sphere_sdf(2.0, 0.2, 0.4)
    bad = sdf.copy()
    bad[5, 5, 5] = np.nan
    assert _raw_setup(bad, org, 0.2, 0.4)[0] == -2          # NaN
    assert _raw_setup(sdf, org, 0.2, 50.0)[0] == -2         # tube reaches the grid edge
    assert _raw_setup(sdf, org, -0.2, 0.4)[0] == -1         # h <= 0
    assert _raw_setup(sdf, org, 0.2, 0.4, kappa=-1.0)[0] == -1
    assert _raw_setup(np.full((9, 9, 9), 5.0), org, 0.2, 0.4)[0] == -2  # empty tube
    code, ctx = _raw_setup(sdf, org, 0.2, 0.4)
    assert code == 0
    # device entry points on a host-only context fail without touching HIP
    assert lib.ibim_apply(ctx, None, None, None) == -6
    assert lib.ibim_rhs(ctx, None, None) == -6
    assert b"host-only" in lib.ibim_last_error()
    lib.ibim_destroy(ctx)
    lib.ibim_destroy(None)


def test_python_binding_rejects_bad_arguments():
    sdf, org = workloads.sphere_sdf(2.0, 0.2, 0.4)
    with pytest.raises(ibim.IbimError):
        ibim.Problem(sdf, org, 0.2, 0.4, 1.0, 80.0, 0.1, np.zeros((1, 3)), np.ones(1),
                     device=-1, restart=0)
    with pytest.raises(ValueError):
        ibim.Problem(sdf, org, 0.2, 0.4, 1.0, 80.0, 0.1, np.zeros((2, 3)), np.ones(1), device=-1)
    with pytest.raises(ibim.IbimError):
        ibim.Problem(sdf, org, 0.2, 0.4, 1.0, 80.0, 0.1, np.zeros((1, 3)), np.ones(1),
                     device=-1, pair_scratch_max=-1)
