"""Seeded synthetic inputs for the CTR-IBIM solver and its oracle.

This module only *generates inputs*: a signed-distance grid (positive inside
the molecule, Section 2.1, signed-distance definition) and point charges.  It
holds none of the method's arithmetic (no kernels, no projections, no
quadrature weights), so both the HIP library and the CPU oracle may consume
what it returns.

Every generator is deterministic given its arguments (seeded ``numpy``
generators, ``PCG64``).

Grid convention shared by every consumer: ``sdf`` is a C-ordered float64
array of shape ``(nx, ny, nz)`` (z fastest); node ``(i, j, k)`` sits at
``origin + h * (i, j, k)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload",
    "sphere_sdf",
    "torus_sdf",
    "ball_charges",
    "born_sphere",
    "kirkwood_sphere",
    "torus_case",
    "by_name",
    "ses_molecule",
    "random_vector",
]

# Dielectrics and Debye parameter used by every named workload.
EPS_IN = 1.0
EPS_OUT = 80.0
KAPPA = 0.1257

# Grid nodes kept between the tube and the grid edge.  The second-derivative
# stencil reaches two nodes, so the tube must stay at least two nodes inside.
PAD_NODES = 4


@dataclasses.dataclass
class Workload:
    name: str
    sdf: np.ndarray          # (nx, ny, nz) float64, positive inside
    origin: np.ndarray       # (3,) float64
    h: float
    eps_tube: float
    eps_in: float
    eps_out: float
    kappa: float
    charge_xyz: np.ndarray   # (nc, 3) float64
    charge_q: np.ndarray     # (nc,) float64
    tol: float
    meta: dict

    @property
    def dims(self):
        return tuple(int(s) for s in self.sdf.shape)

    def describe(self) -> dict:
        return {
            "workload": self.name,
            "grid": list(self.dims),
            "h": self.h,
            "eps_tube": self.eps_tube,
            "eps_in": self.eps_in,
            "eps_out": self.eps_out,
            "kappa": self.kappa,
            "n_charges": int(self.charge_q.shape[0]),
            "tol": self.tol,
            **{k: v for k, v in self.meta.items() if isinstance(v, (int, float, str))},
        }


def _grid_around(center, half_extent: float, h: float, offset=(0.0, 0.0, 0.0)):
    """Node coordinates (three 1-D axes) covering ``center +- half_extent``.

    With ``offset == 0`` the centre is itself a grid node.
    """
    n_half = int(math.ceil(half_extent / h))
    axes = []
    origin = np.empty(3)
    for a in range(3):
        o = center[a] + offset[a] * h - n_half * h
        origin[a] = o
        axes.append(o + h * np.arange(2 * n_half + 1, dtype=np.float64))
    return origin, axes


def sphere_sdf(radius: float, h: float, eps_tube: float, center=(0.0, 0.0, 0.0),
               offset=(0.0, 0.0, 0.0)):
    """Exact signed distance ``R - |x - c|`` of a sphere on a uniform grid."""
    c = np.asarray(center, dtype=np.float64)
    half = radius + eps_tube + PAD_NODES * h
    origin, (xs, ys, zs) = _grid_around(c, half, h, offset)
    X, Y, Z = np.meshgrid(xs - c[0], ys - c[1], zs - c[2], indexing="ij")
    sdf = radius - np.sqrt(X * X + Y * Y + Z * Z)
    return np.ascontiguousarray(sdf), origin


def _rotation(a: float, b: float, c: float) -> np.ndarray:
    ca, sa = math.cos(a), math.sin(a)
    cb, sb = math.cos(b), math.sin(b)
    cc, sc = math.cos(c), math.sin(c)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    rz = np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]])
    return rz @ ry @ rx


def torus_sdf(r_major: float, r_minor: float, h: float, eps_tube: float,
              angles=(0.0, 0.0, 0.0), offset=(0.0, 0.0, 0.0)):
    """Exact signed distance of a torus (positive inside its tube).

    The torus lies in the plane z = 0 before the rotation ``Rz(c) Ry(b) Rx(a)``
    (rotation angles about x, y, z as in the torus test of Section 2.6).
    """
    half = r_major + r_minor + eps_tube + PAD_NODES * h
    origin, (xs, ys, zs) = _grid_around(np.zeros(3), half, h, offset)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    rot = _rotation(*angles)
    pts = np.stack([X, Y, Z], axis=-1) @ rot  # body coordinates = R^T x
    rho = np.sqrt(pts[..., 0] ** 2 + pts[..., 1] ** 2)
    sdf = r_minor - np.sqrt((rho - r_major) ** 2 + pts[..., 2] ** 2)
    return np.ascontiguousarray(sdf), origin


def ball_charges(n: int, r_max: float, seed: int, q_lo=-1.0, q_hi=1.0):
    """``n`` charges uniform in the ball ``|z| <= r_max``; ``q ~ U[q_lo, q_hi]``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = r_max * rng.random(n) ** (1.0 / 3.0)
    xyz = v * r[:, None]
    q = rng.uniform(q_lo, q_hi, size=n)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(q)


def born_sphere(h=0.2, radius=2.0, eps_factor=2.0, offset=(0.0, 0.0, 0.0), tol=1e-10,
                kappa=KAPPA, eps_in=EPS_IN, eps_out=EPS_OUT) -> Workload:
    """Sphere with one +1 charge at its centre (Born ion)."""
    eps_tube = eps_factor * h
    sdf, origin = sphere_sdf(radius, h, eps_tube, offset=offset)
    return Workload(
        name=f"born_sphere_R{radius:g}_h{h:g}_eps{eps_factor:g}h",
        sdf=sdf, origin=origin, h=h, eps_tube=eps_tube, eps_in=eps_in,
        eps_out=eps_out, kappa=kappa,
        charge_xyz=np.zeros((1, 3)), charge_q=np.ones(1), tol=tol,
        meta={"radius": radius, "geometry": "sphere"},
    )


def kirkwood_sphere(h=0.25, radius=10.0, eps_factor=3.0, n_charges=20, r_charges=8.0,
                    seed=2210, tol=1e-8, offset=(0.0, 0.0, 0.0)) -> Workload:
    """Sphere with ``n_charges`` seeded charges inside ``r <= r_charges``."""
    eps_tube = eps_factor * h
    sdf, origin = sphere_sdf(radius, h, eps_tube, offset=offset)
    xyz, q = ball_charges(n_charges, r_charges, seed)
    return Workload(
        name=f"kirkwood_sphere_R{radius:g}_nc{n_charges}_h{h:g}_eps{eps_factor:g}h",
        sdf=sdf, origin=origin, h=h, eps_tube=eps_tube, eps_in=EPS_IN,
        eps_out=EPS_OUT, kappa=KAPPA, charge_xyz=xyz, charge_q=q, tol=tol,
        meta={"radius": radius, "geometry": "sphere", "seed": seed},
    )


def torus_case(h=0.1, r_major=1.0, r_minor=0.5, eps_factor=2.0, kappa=KAPPA,
               angles=(1.99487, 2.54097947651017, 4.219760487439292),
               eps_in=EPS_IN, eps_out=EPS_OUT, tol=1e-10) -> Workload:
    """Rotated torus (radii and rotation angles of the torus test, Section 2.6)."""
    eps_tube = eps_factor * h
    sdf, origin = torus_sdf(r_major, r_minor, h, eps_tube, angles=angles)
    rot = _rotation(*angles)
    # one unit charge on the core circle of the torus tube (inside the body)
    z = rot @ np.array([r_major, 0.0, 0.0])
    return Workload(
        name=f"torus_R{r_major:g}_r{r_minor:g}_h{h:g}",
        sdf=sdf, origin=origin, h=h, eps_tube=eps_tube, eps_in=eps_in,
        eps_out=eps_out, kappa=kappa, charge_xyz=z[None, :].copy(),
        charge_q=np.ones(1), tol=tol,
        meta={"geometry": "torus", "r_major": r_major, "r_minor": r_minor},
    )


def ses_molecule(n_atoms=500, box=25.0, h=0.3, eps_factor=2.0, seed=3, probe=1.4,
                 tol=1e-6) -> Workload:
    """Random-walk molecule (see ``workloads.ses``) with its SES signed distance."""
    from . import ses
    xyz, radii, q = ses.random_walk_molecule(n_atoms, box, seed)
    eps_tube = eps_factor * h
    sdf, origin = ses.ses_grid(xyz, radii, h, eps_tube, probe=probe, pad_nodes=PAD_NODES)
    return Workload(
        name=f"ses_molecule_{n_atoms}at_box{box:g}_h{h:g}_eps{eps_factor:g}h",
        sdf=sdf, origin=origin, h=h, eps_tube=eps_tube, eps_in=EPS_IN, eps_out=EPS_OUT,
        kappa=KAPPA, charge_xyz=xyz, charge_q=q, tol=tol,
        meta={"geometry": "ses", "n_atoms": n_atoms, "box": box, "seed": seed, "probe": probe},
    )


def by_name(name: str) -> Workload:
    """Named workloads.

    ``born``      Born ion: sphere R = 2 A, +1e at the centre, h = 0.2, eps = 2h.
    ``kirkwood``  Kirkwood sphere R = 10 A, 20 charges in r <= 8 A, h = 0.25, eps = 3h.
    ``ses500``    500-atom random-walk molecule, 25 A box, SES (probe 1.4 A), h = 0.3,
                  eps = 2h, tol 1e-6.
    ``ses2000``   2000 atoms, 40 A box, h = 0.35, eps = 2h, tol 1e-6.
    ``ses2000_twin`` the same molecule at h = 0.7 with eps = 1.5h (within the
                  re-entrant reach of the 1.4 A probe).
    ``kirkwood_h0.1`` the Kirkwood sphere at h = 0.1 (eps = 3h, M ~ 7.5e5).
    ``kirkwood_h0.07`` the Kirkwood sphere at h = 0.07 (M ~ 1.5e6).
    """
    if name == "born":
        return born_sphere()
    if name == "kirkwood":
        return kirkwood_sphere()
    if name == "ses500":
        return ses_molecule(500, 25.0, 0.3, 2.0, seed=3)
    if name == "ses2000":
        return ses_molecule(2000, 40.0, 0.35, 2.0, seed=5)
    if name == "ses2000_twin":
        return ses_molecule(2000, 40.0, 0.7, 1.5, seed=5)
    if name == "kirkwood_h0.1":
        return kirkwood_sphere(h=0.1)
    if name == "kirkwood_h0.07":
        return kirkwood_sphere(h=0.07)
    raise KeyError(name)


def serving_stream(n_requests=256, seed=4, sphere_radius=(2.0, 10.0), max_charges=30,
                   ses_atoms=(50, 2000), hs=(0.2, 0.3, 0.5), tol=1e-6, progress=None) -> list:
    """Seeded mix of solve requests for the serving benchmark.

    Half spheres (radius uniform in ``sphere_radius``, 1..``max_charges``
    charges in r <= 0.8 R), half random-walk SES molecules (atom count uniform
    in ``ses_atoms``, box scaled as 25 A * (n/500)^(1/3)); grid spacing drawn
    from ``hs``, tube half-width 2h, GMRES tolerance ``tol``.  ``progress``,
    if given, is called with (index, workload) after each request is made.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_requests):
        h = float(rng.choice(np.asarray(hs, dtype=np.float64)))
        sub_seed = int(rng.integers(1, 2**31 - 1))
        if rng.random() < 0.5:
            R = float(rng.uniform(*sphere_radius))
            nq = int(rng.integers(1, max_charges + 1))
            wl = kirkwood_sphere(h=h, radius=R, eps_factor=2.0, n_charges=nq, r_charges=0.8 * R,
                                 seed=sub_seed, tol=tol)
        else:
            n = int(rng.integers(ses_atoms[0], ses_atoms[1] + 1))
            box = 25.0 * (n / 500.0) ** (1.0 / 3.0)
            wl = ses_molecule(n, box, h, 2.0, seed=sub_seed, tol=tol)
        out.append(wl)
        if progress is not None:
            progress(i, wl)
    return out


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal test vector (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)
