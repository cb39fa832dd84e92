"""Pins of the oracle's K-reg and HYB-IBIM rows (Section 2.3, Section 3.2).

* the K-reg constant of K12 equals the mean of K12 over the tangent disc of
  radius tau, computed by quadrature of the kernel itself;
* the regularised sets are exactly the tube nodes within tangential distance
  tau (and normal distance eps + h) of P(y_k), found by brute force;
* K-reg everywhere (J = 1) on the Born ion converges to the closed form, with
  a larger error than CTR2, as Fig. 2 of the paper reports;
* HYB on a smooth sphere flags no node and reproduces CTR2 bit for bit;
* on a molecular surface HYB flags a small fraction of the nodes, and the
  flagged rows carry exactly the K-reg constants.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import analytic
import oracle
import workloads

KAP = workloads.KAPPA
EI, EE = workloads.EPS_IN, workloads.EPS_OUT


@pytest.mark.parametrize("kappa,tau", [(0.1257, 0.4), (0.1257, 0.8), (2.0, 0.3), (1e-5, 0.5)])
def test_kreg_constant_is_the_disc_mean_of_k12(kappa, tau):
    # K12(r) = (1 - e^{-kappa r}) / (4 pi r) on the tangent plane (x = P(y))
    def k12(r):
        return -math.expm1(-kappa * r) / (4.0 * math.pi * r)
    mean = integrate.quad(lambda r: k12(r) * 2.0 * math.pi * r, 0.0, tau, epsabs=0,
                          epsrel=1e-13)[0] / (math.pi * tau * tau)
    assert abs(oracle.kreg_c12(kappa, tau) - mean) <= 1e-12 * mean
    assert oracle.kreg_c12(0.0, tau) == 0.0


def test_kreg_sets_by_brute_force():
    wl = workloads.born_sphere(h=0.4, offset=(0.13, -0.07, 0.21))
    o = oracle.Oracle.from_workload(wl, hybrid=2)
    nd = o.nodes()
    c = o.corrections()
    tau, reach = 2.0 * wl.h, wl.eps_tube + wl.h
    rng = np.random.default_rng(3)
    for k in rng.choice(o.M, size=25, replace=False):
        v = nd["y"] - nd["P"][k]
        vn = v @ nd["n"][k]
        t = v - vn[:, None] * nd["n"][k][None, :]
        tt = np.einsum("ij,ij->i", t, t)
        # brute force with a margin: decisions closer than 1e-12 to the
        # thresholds are left to the oracle's own rounding
        inside = np.nonzero((tt < tau * tau - 1e-12) & (np.abs(vn) <= reach - 1e-12))[0]
        maybe = np.nonzero((tt < tau * tau + 1e-12) & (np.abs(vn) <= reach + 1e-12))[0]
        got = c["col"][c["row"][k]:c["row"][k + 1]]
        assert np.all(np.diff(got) > 0)
        assert set(inside) <= set(got) <= set(maybe), k
        assert np.all(c["axis"][c["row"][k]:c["row"][k + 1]] == -1)


def test_kreg_born_ion_converges_with_larger_error_than_ctr2():
    exact = analytic.born_energy(1.0, 2.0, EI, EE, KAP)
    err = {}
    for hybrid in (0, 2):
        for h in (0.4, 0.2):
            wl = workloads.born_sphere(h=h)
            o = oracle.Oracle.from_workload(wl, hybrid=hybrid)
            _, info = o.solve_energy(wl.charge_xyz, wl.charge_q, 1e-10)
            err[hybrid, h] = abs(info["g_pol"] - exact) / abs(exact)
    print({k: f"{v:.3e}" for k, v in err.items()})
    # first order for K-reg at eps = 2h (the area with J = 1 alone is O(h))
    assert err[2, 0.2] < 0.6 * err[2, 0.4] and err[2, 0.4] < 0.15
    assert err[0, 0.2] < err[2, 0.2] and err[0, 0.4] < err[2, 0.4]


def test_hybrid_on_smooth_sphere_is_ctr2():
    wl = workloads.born_sphere(h=0.3, offset=(0.11, 0.05, -0.17))
    a = oracle.Oracle.from_workload(wl, hybrid=0)
    b = oracle.Oracle.from_workload(wl, hybrid=1)
    assert not b.bad_nodes().any()
    u = workloads.random_vector(2 * a.M, 9)
    assert np.array_equal(a.apply(u), b.apply(u))


def test_hybrid_rows_on_molecular_surface():
    wl = workloads.ses_molecule(20, 9.0, 0.35, 2.0, seed=11)
    o = oracle.Oracle.from_workload(wl, hybrid=1)
    bad = o.bad_nodes()
    assert 0 < bad.sum() < 0.1 * o.M
    nd = o.nodes()
    assert np.all(nd["J"][bad] == 1.0)
    # one bad row by hand: only the K12 constant acts on its regularised set
    k = int(np.nonzero(bad)[0][0])
    c = o.corrections()
    e = slice(c["row"][k], c["row"][k + 1])
    cols = c["col"][e]
    u = workloads.random_vector(2 * o.M, 4)
    out1, out2 = o.apply_rows(u, np.array([k]))
    excl = np.zeros(o.M, bool)
    excl[cols] = True
    h3 = wl.h ** 3
    s1 = s2 = 0.0
    for m in range(o.M):
        if excl[m]:
            continue
        K = oracle.kernels(nd["P"][k], nd["n"][k], nd["P"][m], nd["n"][m], EI, EE, KAP)
        a1, a2 = u[m] * nd["w"][m], u[o.M + m] * nd["w"][m]
        s1 += K[0] * a1 - K[1] * a2
        s2 += K[2] * a1 - K[3] * a2
    c12 = oracle.kreg_c12(KAP, 2.0 * wl.h)
    a2 = u[o.M + cols] * nd["w"][cols]
    lam1, lam2 = 0.5 * (1 + EE / EI), 0.5 * (1 + EI / EE)
    ref1 = lam1 * u[k] + h3 * s1 - h3 * c12 * a2.sum()
    ref2 = lam2 * u[o.M + k] + h3 * s2
    assert abs(out1[0] - ref1) <= 1e-11 * abs(ref1)
    assert abs(out2[0] - ref2) <= 1e-11 * max(abs(ref2), 1e-300)
