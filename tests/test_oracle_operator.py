"""Pins for the oracle's discrete operator, solve and energy.

Each check compares the oracle with something the paper or the mathematics
fixes, not with the oracle itself:

* surface area h^3 sum w -> exact area (eq. surface-integral-IBIM, f = 1);
* every 2x2 block applied to a constant density on a sphere -> the exact
  layer-potential integrals (second order at fixed tube width);
* the double-layer identity int dG0/dn_y = -1/2 on a rotated torus;
* Born ion and Kirkwood sphere energies -> closed forms (eq. pol-energy);
* GMRES -> dense LU of the explicitly assembled matrix;
* apply -> the operator written out entry by entry on a tiny grid.
"""
import math

import numpy as np
import pytest

import analytic
import oracle
import workloads

EI, EE, KAP = 1.0, 80.0, 0.1257


def _sphere_oracle(R, h, eps, kappa=KAP, ei=EI, ee=EE):
    sdf, org = workloads.sphere_sdf(R, h, eps)
    return oracle.Oracle(sdf, org, h, eps, ei, ee, kappa)


def test_sphere_area_second_order():
    """h^3 sum w -> 4 pi R^2 at fixed tube width: the observed order, fitted
    over four grids, is about two (grid alignment makes single ratios erratic)."""
    hs = (0.2, 0.15, 0.1, 0.075)
    errs = []
    for h in hs:
        sdf, org = workloads.sphere_sdf(2.0, h, 0.6)
        o = oracle.Oracle(sdf, org, h, 0.6, EI, EE, KAP, weight_rows=np.zeros(1, dtype=np.int64))
        errs.append(abs(o.area() - 16 * math.pi) / (16 * math.pi))
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    print(f"sphere area errors {errs}, fitted order {order:.2f}")
    assert 1.7 < order < 3.5
    assert max(errs) < 5e-4 and errs[-1] < 5e-5


def test_torus_area():
    wl = workloads.torus_case(h=0.1)
    o = oracle.Oracle.from_workload(wl)
    exact = 4 * math.pi ** 2 * 1.0 * 0.5
    assert abs(o.area() - exact) / exact < 1e-3


def test_torus_area_study_against_table_1():
    """Area of the rotated torus (radii 1 and 1/2, the angles of Section 2.6)
    with eps = 2h and the finite-difference Jacobian J_h, as in the torus
    table of Section 2.6, whose relative errors lie between 9.5e-7 and 8.5e-6
    on grids of 103 to 512 nodes per side.  The table does not state the box
    those grids cover, so the spacing of each row, and so its exact value, is
    unknown (parity unpinned); what is checked is that the error falls from
    h = 0.1 into the table's range at the finest spacings here."""
    exact = 4 * math.pi ** 2 * 1.0 * 0.5
    errs = {}
    for h in (0.1, 0.05, 0.025, 0.02):
        wl = workloads.torus_case(h=h)
        o = oracle.Oracle.from_workload(wl, weight_rows=np.zeros(1, dtype=np.int64))
        errs[h] = abs(o.area() - exact) / exact
    print("torus area relative errors:", errs)
    assert errs[0.05] < errs[0.1] / 4
    assert errs[0.025] < 1.5e-5 and errs[0.02] < 1.5e-5


def test_sphere_geometry_exact_quantities():
    R, h = 2.0, 0.2
    o = _sphere_oracle(R, h, 0.4)
    nd = o.nodes()
    rad = np.linalg.norm(nd["P"], axis=1)
    assert np.max(np.abs(rad - R)) < 2e-3                      # projection onto the sphere
    radial = nd["y"] / np.linalg.norm(nd["y"], axis=1)[:, None]
    assert np.min(np.sum(nd["n"] * radial, axis=1)) > 1 - 1e-4  # outward normals
    assert np.max(np.abs(nd["kappa"] - 1.0 / R)) < 1.5e-2 / R  # principal curvatures 1/R, O(h^2)
    Jex = (R / (R - nd["d"])) ** 2                              # level-set Jacobian
    assert np.max(np.abs(nd["J"] / Jex - 1)) < 1e-2            # O(h^2) from the Hessian


def _block_errors(R, h, eps):
    o = _sphere_oracle(R, h, eps)
    M = o.M
    one, zero = np.ones(M), np.zeros(M)
    a1 = o.apply(np.r_[one, zero])
    a2 = o.apply(np.r_[zero, one])
    S0, Sk, D0, Dk = analytic.sphere_layer_integrals(R, KAP)
    H = analytic.sphere_hyper_difference(R, KAP)
    lam1, lam2 = 0.5 * (1 + EE / EI), 0.5 * (1 + EI / EE)
    # integrals of K11, K21, K12, K22 (eq. Kij-kernels) against density 1
    I11 = D0 - (EE / EI) * Dk
    I12 = S0 - Sk
    I21 = H
    I22 = D0 - (EI / EE) * Dk     # adjoint double layers equal the double layers on a sphere
    got = [a1[:M] - lam1, a1[M:], -a2[:M], a2[M:] - lam2]
    ex = [I11, I21, I12, -I22]
    return [float(np.max(np.abs(g - e)) / abs(e)) for g, e in zip(got, ex)]


def test_blocks_on_sphere_second_order_at_fixed_width():
    coarse = _block_errors(1.0, 0.2, 0.4)
    fine = _block_errors(1.0, 0.1, 0.4)
    for c, f in zip(coarse, fine):
        assert f < 0.02
        assert c / f > 3.0, (coarse, fine)  # order >= ~1.6 on a 2x refinement


def test_double_layer_identity_on_torus():
    # kappa = 0, eps_E/eps_I = 2: K11 = -dG0/dn_y; row 1 of A [1; 0] is
    # lambda_1 + 1/2 = eps_E/eps_I wherever the double layer integrates to -1/2.
    errs = []
    for h in (0.1, 0.07):
        wl = workloads.torus_case(h=h, eps_factor=0.3 / h, kappa=0.0, eps_in=1.0, eps_out=2.0)
        o = oracle.Oracle.from_workload(wl)
        a = o.apply(np.r_[np.ones(o.M), np.zeros(o.M)])
        errs.append(float(np.sqrt(np.mean((a[:o.M] - 2.0) ** 2))))
    assert errs[1] < 2e-3
    assert errs[0] / errs[1] > 1.5, errs  # (0.1/0.07)^2 = 2.04 for second order


def test_born_energy_converges_to_closed_form():
    exact = analytic.born_energy(1.0, 2.0, EI, EE, KAP)
    rel = []
    for h in (0.4, 0.2):
        wl = workloads.born_sphere(h=h)
        o = oracle.Oracle.from_workload(wl)
        x, info = o.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10)
        assert info["status"] == 0 and info["true_relres"] < 1e-9
        rel.append(abs(info["g_pol"] - exact) / abs(exact))
    assert rel[1] < 1e-4, rel
    assert rel[0] / rel[1] > 4.0, rel


def test_born_surface_solution():
    wl = workloads.born_sphere(h=0.2)
    o = oracle.Oracle.from_workload(wl)
    x, info = o.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10)
    psi, psin = analytic.born_psi_surface(1.0, 2.0, EI, EE, KAP)
    M = o.M
    assert np.max(np.abs(x[:M] - psi)) / abs(psi) < 5e-3
    assert np.max(np.abs(x[M:] - psin)) / abs(psin) < 5e-3


def test_kirkwood_series_born_limit_and_interface():
    from scipy import special
    a = 10.0
    # single central charge -> Born
    gk = analytic.kirkwood_energy(np.zeros((1, 3)), np.ones(1), a, EI, EE, KAP)
    assert abs(gk - analytic.born_energy(1.0, a, EI, EE, KAP)) < 1e-15
    # interface conditions mode by mode with k_n from scipy (independent of
    # the ratio recurrence): eps_I d_r phi_in = eps_E d_r phi_out at r = a.
    b, q = 6.5, 1.0
    c = analytic.kirkwood_coeffs(30, a, EI, EE, KAP)
    for n in range(30):
        An = q * c[n] * b ** n
        coul = q * b ** n / (4 * math.pi * EI * a ** (n + 1))
        T = An * a ** n + coul
        D = n * An * a ** (n - 1) - (n + 1) * coul / a if n > 0 else -(n + 1) * coul / a
        x = KAP * a
        ratio = KAP * special.spherical_kn(n, x, derivative=True) / special.spherical_kn(n, x)
        assert abs(EI * D - EE * ratio * T) < 1e-12 * abs(EE * ratio * T)


def test_kirkwood_small_sphere_energy():
    rng = np.random.default_rng(5)
    R = 2.0
    zq, q = workloads.ball_charges(4, 1.2, seed=11)
    wl = workloads.born_sphere(h=0.2, radius=R)
    o = oracle.Oracle.from_workload(wl)
    x, info = o.solve_energy(zq, q, 1e-10)
    exact = analytic.kirkwood_energy(zq, q, R, EI, EE, KAP)
    assert abs(info["g_pol"] - exact) / abs(exact) < 2e-3, (info["g_pol"], exact)


def test_gmres_matches_dense_lu():
    o = _sphere_oracle(1.0, 0.3, 0.6)
    M = o.M
    N = 2 * M
    A = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = o.apply(e)
    b = o.rhs(np.zeros((1, 3)), np.ones(1))
    xd = np.linalg.solve(A, b)
    xg, info = o.gmres(b, 1e-13, restart=120, maxit=400)
    assert info["status"] == 0
    assert np.max(np.abs(xg - xd)) < 1e-9 * np.max(np.abs(xd))
    # restarted GMRES reaches the same solution
    xr, info_r = o.gmres(b, 1e-13, restart=5, maxit=2000)
    assert np.max(np.abs(xr - xd)) < 1e-9 * np.max(np.abs(xd))
    # the matrix has the 2x2 block structure: diagonal blocks carry lambda
    lam1, lam2 = 0.5 * (1 + EE / EI), 0.5 * (1 + EI / EE)
    assert abs(np.mean(np.diag(A)[:M]) - lam1) < 0.2 * lam1
    assert abs(np.mean(np.diag(A)[M:]) - lam2) < 0.2 * lam2


def test_rhs_is_coulomb_field():
    o = _sphere_oracle(2.0, 0.2, 0.4)
    nd = o.nodes()
    zq = np.array([[0.3, -0.2, 0.1]])
    g = o.rhs(zq, np.array([0.7]))
    r = nd["P"] - zq
    R = np.linalg.norm(r, axis=1)
    assert np.allclose(g[:o.M], 0.7 / (4 * math.pi * EI * R), rtol=1e-14, atol=0)
    g2 = -0.7 * np.sum(r * nd["n"], axis=1) / (4 * math.pi * EI * R ** 3)
    assert np.allclose(g[o.M:], g2, rtol=1e-13, atol=0)


def test_setup_rejects_bad_inputs():
    sdf, org = workloads.sphere_sdf(2.0, 0.2, 0.4)
    bad = sdf.copy()
    bad[3, 3, 3] = np.nan
    with pytest.raises(ValueError):
        oracle.Oracle(bad, org, 0.2, 0.4, EI, EE, KAP)
    with pytest.raises(ValueError):
        oracle.Oracle(sdf, org, 0.2, 100.0, EI, EE, KAP)  # tube reaches the grid edge
    with pytest.raises(ValueError):
        oracle.Oracle(sdf, org, -0.2, 0.4, EI, EE, KAP)


def test_apply_equals_its_definition_on_a_tiny_grid():
    """Brute force: the operator assembled entry by entry from eq.
    (corr-trapz-rule-sys1/2) -- Lambda, h^3 K w off the correction sets, and the
    correction blocks [h^2 om11, -h^3 kappa/(4 pi); h^2 om21, h^2 (eps_I/eps_E) om11]
    times w on them -- applied to a random vector equals the oracle's apply.
    Catches a dropped term, a sign, or a pair skipped or counted twice."""
    wl = workloads.born_sphere(h=0.3, radius=0.6, eps_factor=1.5,
                               offset=(0.07, -0.05, 0.11))
    o = oracle.Oracle.from_workload(wl)
    M, h = o.M, wl.h
    nd, c = o.nodes(), o.corrections()
    P, n, w = nd["P"], nd["n"], nd["w"]
    u = workloads.random_vector(2 * M, 31)
    a1, a2 = w * u[:M], w * u[M:]
    lam1, lam2 = 0.5 * (1 + wl.eps_out / wl.eps_in), 0.5 * (1 + wl.eps_in / wl.eps_out)
    out = np.concatenate([lam1 * u[:M], lam2 * u[M:]])
    for k in range(M):
        corr = {int(c["col"][e]): e for e in range(c["row"][k], c["row"][k + 1])}
        assert k in corr  # a node is always in its own correction set
        for m in range(M):
            if m in corr:
                e = corr[m]
                out[k] += h * h * c["om11"][e] * a1[m] - h ** 3 * wl.kappa / (4 * math.pi) * a2[m]
                out[M + k] += (h * h * c["om21"][e] * a1[m]
                               + h * h * (wl.eps_in / wl.eps_out) * c["om11"][e] * a2[m])
            else:
                K = oracle.kernels(P[k], n[k], P[m], n[m], wl.eps_in, wl.eps_out, wl.kappa)
                out[k] += h ** 3 * (K[0] * a1[m] - K[1] * a2[m])
                out[M + k] += h ** 3 * (K[2] * a1[m] - K[3] * a2[m])
    ref = o.apply(u)
    assert M < 400
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
