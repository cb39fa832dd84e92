"""Closed-form solutions used to pin the oracle (independent of it).

* Born ion (Section 2.6, exact sphere solution, with the two misprints of the
  printed formula corrected: the interior Coulomb term carries eps_I, and the
  reaction potential is linear in q).
* Kirkwood series for off-centre charges in a dielectric sphere with an
  ionic exterior (standard separation of variables; derived in the design
  notes and checked here against the interface conditions).
* Layer-potential integrals of a constant density over a sphere, used to pin
  each block of the operator separately.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
from scipy import special


# --------------------------------------------------------------------------
# Born ion
def born_psi_surface(q, R, eps_in, eps_out, kappa):
    """(psi, interior psi_n) on the sphere |x| = R for a charge q at the centre."""
    psi = q / (4 * math.pi * eps_out * R * (1 + kappa * R))
    psi_n = -q / (4 * math.pi * eps_in * R * R)
    return psi, psi_n


def born_energy(q, R, eps_in, eps_out, kappa):
    """G_pol = q^2/(8 pi R) (1/(eps_E (1 + kappa R)) - 1/eps_I)."""
    return q * q / (8 * math.pi * R) * (1.0 / (eps_out * (1 + kappa * R)) - 1.0 / eps_in)


# --------------------------------------------------------------------------
# Kirkwood sphere
def _gamma_n(nmax, x):
    """gamma_n = x k_n'(x)/k_n(x) for the decaying modified spherical Bessel k_n.

    With R_n = k_{n-1}/k_n: R_0 = 1, R_n = 1/(R_{n-1} + (2n-1)/x),
    gamma_n = -x R_n - (n+1).  For x = 0 the Laplace limit -(n+1).
    """
    g = np.empty(nmax + 1)
    if x == 0.0:
        return -(np.arange(nmax + 1) + 1.0)
    Rn = 1.0
    g[0] = -x * Rn - 1.0
    for n in range(1, nmax + 1):
        Rn = 1.0 / (Rn + (2 * n - 1) / x)
        g[n] = -x * Rn - (n + 1.0)
    return g


def kirkwood_coeffs(nmax, a, eps_in, eps_out, kappa):
    """c_n with phi_rxn(x) = sum_j q_j sum_n c_n |z_j|^n |x|^n P_n(cos theta_j)."""
    g = _gamma_n(nmax, kappa * a)
    n = np.arange(nmax + 1, dtype=np.float64)
    c = (eps_out * g + (n + 1) * eps_in) / (n * eps_in - eps_out * g)
    return c / (4 * math.pi * eps_in * a ** (2 * n + 1))


def kirkwood_phi_rxn(x, zq, q, a, eps_in, eps_out, kappa, nmax=120):
    """Reaction potential at interior points x (k, 3) of the sphere radius a."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    zq = np.atleast_2d(np.asarray(zq, dtype=np.float64))
    c = kirkwood_coeffs(nmax, a, eps_in, eps_out, kappa)
    out = np.zeros(x.shape[0])
    for i in range(x.shape[0]):
        rx = np.linalg.norm(x[i])
        for j in range(zq.shape[0]):
            rz = np.linalg.norm(zq[j])
            if rx == 0.0 or rz == 0.0:
                out[i] += q[j] * c[0]
                continue
            ct = float(np.dot(x[i], zq[j]) / (rx * rz))
            ct = max(-1.0, min(1.0, ct))
            n = np.arange(nmax + 1)
            terms = c * (rz * rx) ** n * special.eval_legendre(n, ct)
            out[i] += q[j] * terms.sum()
    return out


def kirkwood_energy(zq, q, a, eps_in, eps_out, kappa, nmax=120):
    phi = kirkwood_phi_rxn(zq, zq, q, a, eps_in, eps_out, kappa, nmax)
    return 0.5 * float(np.dot(q, phi))


# --------------------------------------------------------------------------
# Layer potentials of the density 1 on a sphere of radius R, evaluated on it.
def sphere_layer_integrals(R, kappa):
    """Exact surface integrals (x on the sphere, outward normals):

    S0 = int G0,   Sk = int Gk,
    D0 = int dG0/dn_y = -1/2,   Dk = int dGk/dn_y  (= int dGk/dn_x on a sphere).
    """
    S0 = R
    Sk = (1 - math.exp(-2 * kappa * R)) / (2 * kappa) if kappa > 0 else R
    D0 = -0.5
    if kappa > 0:
        Dk = -(1 - math.exp(-2 * kappa * R) * (1 + kappa * R)) / (2 * kappa * R)
    else:
        Dk = -0.5
    return S0, Sk, D0, Dk


def sphere_hyper_difference(R, kappa, dps=30):
    """int over the sphere of d^2(G0 - Gk)/dn_x dn_y, by 1-D quadrature.

    The mixed normal derivative of G0 - Gk is formed by central finite
    differences of the fundamental solutions themselves (``dps``-digit
    arithmetic), not from a closed-form kernel.  For points on the sphere at
    chord rho the integrand depends on rho only, and dsigma = 2 pi rho drho.
    """
    old = mpmath.mp.dps
    mpmath.mp.dps = dps
    try:
        kap = mpmath.mpf(kappa)
        Rm = mpmath.mpf(R)
        step = mpmath.mpf(10) ** (-(dps // 3))

        def G(rr):
            return -mpmath.expm1(-kap * rr) / (4 * mpmath.pi * rr)

        def integrand(rho):
            t = 2 * mpmath.asin(rho / (2 * Rm))
            x = (mpmath.mpf(0), mpmath.mpf(0), Rm)
            y = (Rm * mpmath.sin(t), mpmath.mpf(0), Rm * mpmath.cos(t))
            nx = (0, 0, 1)
            ny = (y[0] / Rm, y[1] / Rm, y[2] / Rm)
            s = step * rho

            def Gat(a, b):
                d = [(x[i] + a * nx[i]) - (y[i] + b * ny[i]) for i in range(3)]
                return G(mpmath.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2))

            d2 = (Gat(s, s) - Gat(s, -s) - Gat(-s, s) + Gat(-s, -s)) / (4 * s * s)
            return d2 * 2 * mpmath.pi * rho

        val = mpmath.quad(integrand, [0, Rm / 4, Rm, 2 * Rm])
        return float(val)
    finally:
        mpmath.mp.dps = old
