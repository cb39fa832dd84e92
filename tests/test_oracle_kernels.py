"""Pins for the oracle's pair kernels and for the Theorem 2.1 leading terms.

* The four kernels of eq. (Kij-kernels) are checked against finite
  differences (40-digit arithmetic) of the fundamental solutions G0 and
  G_kappa of eq. (layer-kernels) themselves.
* The leading terms l^(ij) used for the correction weights are checked
  against the limit |u| K(x*, P(u0(t) + u)) -> l(theta) on a rotated torus,
  whose closest-point projection and curvatures are known exactly.  This pins
  the sign of s0^(11), s0^(22) and the factor kappa^2 of s0^(21).
"""
import math

import mpmath
import numpy as np
import pytest

import oracle

mpmath.mp.dps = 40

EI, EE, KAP = 1.0, 80.0, 0.1257


def _G(kappa):
    def g(x, y):
        r = mpmath.sqrt(sum((x[i] - y[i]) ** 2 for i in range(3)))
        return mpmath.exp(-kappa * r) / (4 * mpmath.pi * r)
    return g


def _fd_kernels(x, nx, y, ny, ei, ee, kappa):
    x = [mpmath.mpf(v) for v in x]
    y = [mpmath.mpf(v) for v in y]
    nx = [mpmath.mpf(v) for v in nx]
    ny = [mpmath.mpf(v) for v in ny]
    G0, Gk = _G(0), _G(mpmath.mpf(kappa))
    s = mpmath.mpf("1e-12")

    def sh(p, n, t):
        return [p[i] + t * n[i] for i in range(3)]

    def dny(G):
        return (G(x, sh(y, ny, s)) - G(x, sh(y, ny, -s))) / (2 * s)

    def dnx(G):
        return (G(sh(x, nx, s), y) - G(sh(x, nx, -s), y)) / (2 * s)

    def dnxny(G):
        return (G(sh(x, nx, s), sh(y, ny, s)) - G(sh(x, nx, s), sh(y, ny, -s))
                - G(sh(x, nx, -s), sh(y, ny, s)) + G(sh(x, nx, -s), sh(y, ny, -s))) / (4 * s * s)

    r = mpmath.mpf(ee) / ei
    K11 = dny(G0) - r * dny(Gk)
    K12 = G0(x, y) - Gk(x, y)
    K21 = dnxny(G0) - dnxny(Gk)
    K22 = dnx(G0) - (1 / r) * dnx(Gk)
    return np.array([float(K11), float(K12), float(K21), float(K22)])


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("seed", range(6))
def test_kernels_match_fundamental_solution_derivatives(seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-3, 3, 3)
    R = [0.05, 0.4, 2.0, 9.0, 25.0, 0.2][seed]
    y = x + R * _unit(rng.normal(size=3))
    nx = _unit(rng.normal(size=3))
    ny = _unit(rng.normal(size=3))
    K = oracle.kernels(x, nx, y, ny, EI, EE, KAP)
    ref = _fd_kernels(x, nx, y, ny, EI, EE, KAP)
    scale = np.abs(ref) + 1e-300
    assert np.all(np.abs(K - ref) <= 1e-11 * scale + 1e-15), (K, ref)


def test_kernels_laplace_limit():
    rng = np.random.default_rng(7)
    x = rng.normal(size=3)
    y = x + 0.7 * _unit(rng.normal(size=3))
    nx, ny = _unit(rng.normal(size=3)), _unit(rng.normal(size=3))
    K = oracle.kernels(x, nx, y, ny, 2.0, 5.0, 0.0)
    # kappa = 0: K12 = K21 = 0, K11 = (1 - eps_E/eps_I) dG0/dn_y
    assert K[1] == 0.0 and K[2] == 0.0
    r = x - y
    R = np.linalg.norm(r)
    assert abs(K[0] - (1 - 5.0 / 2.0) * np.dot(r, ny) / (4 * math.pi * R ** 3)) < 1e-14


# -------------------------------------------------------------------------
# exact rotated torus
R1, R2 = 1.0, 0.5
ANG = (1.99487, 2.54097947651017, 4.219760487439292)


def _rot(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    rz = np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]])
    return rz @ ry @ rx


ROT = _rot(*ANG)


def torus_point(u, v):
    """surface point, outward normal, (tau_v, k_v), (tau_u, k_u) in world frame"""
    nb = np.array([math.cos(v) * math.cos(u), math.cos(v) * math.sin(u), math.sin(v)])
    cb = R1 * np.array([math.cos(u), math.sin(u), 0.0])
    xb = cb + R2 * nb
    tv = np.array([-math.sin(v) * math.cos(u), -math.sin(v) * math.sin(u), math.cos(v)])
    tu = np.array([-math.sin(u), math.cos(u), 0.0])
    kv = 1.0 / R2
    ku = math.cos(v) / (R1 + R2 * math.cos(v))
    return ROT @ xb, ROT @ nb, (ROT @ tv, kv), (ROT @ tu, ku)


def torus_project(p):
    b = ROT.T @ p
    rho = math.hypot(b[0], b[1])
    c = R1 * np.array([b[0] / rho, b[1] / rho, 0.0])
    dv = b - c
    nb = dv / np.linalg.norm(dv)
    return ROT @ (c + R2 * nb), ROT @ nb


@pytest.mark.parametrize("uv,eta", [((0.3, 0.4), 0.0), ((1.2, 2.5), 0.12), ((4.0, -1.0), -0.15),
                                    ((2.2, 3.0), 0.2)])
def test_leading_terms_are_the_kernel_limits(uv, eta):
    xs, n, (t1, k1), (t2, k2) = torus_point(*uv)
    ia = int(np.argmax(np.abs(n)))
    a, b = (ia + 1) % 3, (ia + 2) % 3
    L = xs - eta * n  # line point at signed distance eta (eta > 0 inside)
    thetas = np.linspace(0.1, 2 * math.pi, 7, endpoint=False)
    ells = [oracle.ell(t1, t2, k1, k2, eta, a, b, EI, EE, KAP, th) for th in thetas]
    s11 = max(abs(e[0]) for e in ells)
    s21 = max(abs(e[1]) for e in ells)
    for theta in thetas:
        def f(rho):
            dlt = np.zeros(3)
            dlt[a] = rho * math.cos(theta)
            dlt[b] = rho * math.sin(theta)
            Py, ny = torus_project(L + dlt)
            K = oracle.kernels(xs, n, Py, ny, EI, EE, KAP)
            return rho * K

        f1, f2, f4 = f(1e-3), f(2e-3), f(4e-3)
        lim = (8 * f1 - 6 * f2 + f4) / 3.0
        l11, l21 = oracle.ell(t1, t2, k1, k2, eta, a, b, EI, EE, KAP, theta)
        l22 = -(EI / EE) * l11
        assert abs(lim[0] - l11) < 1e-6 * s11, (lim[0], l11)
        assert abs(lim[2] - l21) < 1e-6 * s21, (lim[2], l21)
        assert abs(lim[3] - l22) < 1e-6 * (EI / EE) * s11, (lim[3], l22)
        assert abs(lim[1]) < 1e-9  # K12 is bounded: s0^(12) = 0
        # s1^(12): K12 itself tends to kappa / (4 pi)
        assert abs(f1[1] / 1e-3 - KAP / (4 * math.pi)) < 1e-4 * KAP


def test_leading_term_printed_sign_would_fail():
    """The printed (1 - eps_E/eps_I) prefactor has the opposite sign of the limit."""
    xs, n, (t1, k1), (t2, k2) = torus_point(0.3, 0.4)
    ia = int(np.argmax(np.abs(n)))
    a, b = (ia + 1) % 3, (ia + 2) % 3
    l11, _ = oracle.ell(t1, t2, k1, k2, 0.0, a, b, EI, EE, KAP, 0.7)
    dlt = np.zeros(3)
    dlt[a], dlt[b] = 1e-3 * math.cos(0.7), 1e-3 * math.sin(0.7)
    Py, ny = torus_project(xs + dlt)
    K = oracle.kernels(xs, n, Py, ny, EI, EE, KAP)
    assert np.sign(K[0]) == np.sign(l11)
    assert np.sign(K[0]) != np.sign((1 - EE / EI))  # printed prefactor sign
