"""Pins for the oracle's correction weights (Section 2.4.2).

The weight of eq. (single_correction_weight) is *defined* as a limit h -> 0
of a punctured trapezoidal sum.  These tests check the oracle's closed Ewald
evaluation against that definition computed by brute force, against the
known lattice constant for 1/|y| at alpha = beta = 0, and against the
symmetries of the square lattice.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle


def omega_limit_bruteforce(k, alpha, beta, part, q=0):
    """omega_h of the paper's definition with g(y) = exp(-|y|^2), Richardson in h.

    s(y) = |y|^(q-1) e^{ik psi(y)}; q = 0 gives the 1/|y| modes, q = 1 with
    k = 0 the constant function.
    """
    def om_h(h):
        L = int(7.0 / h) + 2
        n = np.arange(-L, L + 1)
        N1, N2 = np.meshgrid(n, n, indexing="ij")
        Y1 = h * (N1 - alpha)
        Y2 = h * (N2 - beta)
        keep = ~((N1 == 0) & (N2 == 0))
        r = np.hypot(Y1, Y2)
        r = np.where(keep, r, 1.0)  # the punctured node is dropped below
        s = ((Y1 + 1j * Y2) / r) ** k * r ** (q - 1)
        g = np.exp(-r * r)
        lattice = (h * h * s * g)[keep].sum()
        if q == 0:
            integral = math.pi ** 1.5 if k == 0 else 0.0
        else:
            integral = math.pi if k == 0 else 0.0
        g0 = math.exp(-h * h * (alpha * alpha + beta * beta))
        val = (integral - lattice) / (h ** (q + 1) * g0)
        return val.real if part == "c" else val.imag

    v1, v2, v3 = om_h(1 / 16), om_h(1 / 32), om_h(1 / 64)
    r1 = (4 * v2 - v1) / 3
    r2 = (4 * v3 - v2) / 3
    return r2, abs(r2 - r1)


def test_w0_origin_equals_epstein_constant():
    # sum' 1/|n| over Z^2 continues to 4 zeta(1/2) beta(1/2) (Epstein zeta of the
    # square lattice); the weight is minus it.
    ref = float(-4 * mpmath.zeta(0.5) * mpmath.dirichlet(0.5, [0, 1, 0, -1]))
    z = oracle.lattice_sums(0.0, 0.0, 3)
    assert abs(-z[0].real - ref) < 1e-13
    assert abs(ref - 3.900264920001956) < 1e-12


def test_w2_origin_vanishes_by_lattice_symmetry():
    z = oracle.lattice_sums(0.0, 0.0, 3)
    assert abs(z[1]) < 1e-14  # cos 2psi / |y| and sin 2psi / |y| at the origin


@pytest.mark.parametrize("alpha,beta", [(0.31, -0.17), (-0.45, 0.38), (0.05, 0.49)])
@pytest.mark.parametrize("k,part", [(0, "c"), (2, "c"), (2, "s"), (4, "c"), (4, "s"), (6, "s")])
def test_ewald_matches_limit_definition(alpha, beta, k, part):
    z = oracle.lattice_sums(alpha, beta, 4)
    ew = -(z[k // 2].real if part == "c" else z[k // 2].imag)
    bf, spread = omega_limit_bruteforce(k, alpha, beta, part)
    assert abs(ew - bf) < 5e-8 + 10 * spread, (ew, bf, spread)


def test_constant_function_weight_is_one():
    # omega[1; alpha, beta] = 1: the punctured rule misses exactly one node.
    for al, be in [(0.0, 0.0), (0.3, -0.2), (-0.5, 0.49)]:
        bf, _ = omega_limit_bruteforce(0, al, be, "c", q=1)
        assert abs(bf - 1.0) < 1e-9


def test_even_modes_are_even_in_the_shift():
    rng = np.random.default_rng(1)
    for _ in range(5):
        al, be = rng.uniform(-0.5, 0.5, 2)
        z1 = oracle.lattice_sums(al, be, 12)
        z2 = oracle.lattice_sums(-al, -be, 12)
        assert np.max(np.abs(z1 - z2)) < 1e-12


def test_axis_swap_symmetry():
    # Swapping lattice axes maps e^{ik psi} to e^{ik(pi/2 - psi)}:
    # Z_k(b, a) = i^k conj(Z_k(a, b)).
    al, be = 0.21, -0.34
    z1 = oracle.lattice_sums(al, be, 10)
    z2 = oracle.lattice_sums(be, al, 10)
    for j in range(10):
        k = 2 * j
        assert abs(z2[j] - (1j ** k) * np.conj(z1[j])) < 1e-12


def test_weights_continuous_at_zero_shift():
    z0 = oracle.lattice_sums(0.0, 0.0, 8)
    z1 = oracle.lattice_sums(1e-9, -2e-9, 8)
    assert np.max(np.abs(z0 - z1)) < 1e-7
    z2 = oracle.lattice_sums(1e-15, 0.0, 8)  # rounding-size shift of a diagonal entry
    assert np.max(np.abs(z0 - z2)) < 1e-12


def test_plane_weight_isotropic_reduces_to_w0():
    # On a locally flat-tangent, isotropic frame (normal along the plane axis,
    # equal curvatures, eta = 0) l11 and l21 are constant in theta, so the
    # weights are a0 * W0.
    tau1 = np.array([1.0, 0.0, 0.0])
    tau2 = np.array([0.0, 1.0, 0.0])
    k = 0.3
    ei, ee, kap = 1.0, 80.0, 0.1257
    o11, o21 = oracle.plane_weights(tau1, tau2, k, k, 0.0, 0, 1, 0.0, 0.0, ei, ee, kap)
    w0 = 3.900264920001956
    l11 = (ee / ei - 1) * k / (8 * math.pi)
    l21 = kap * kap / (8 * math.pi)
    assert abs(o11 - l11 * w0) < 1e-12 * abs(l11 * w0)
    assert abs(o21 - l21 * w0) < 1e-12 * abs(l21 * w0)
