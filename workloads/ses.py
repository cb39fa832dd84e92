"""Synthetic molecules and their solvent-excluded-surface signed distance.

Input generation only (no quantity of the solver's method is computed here).

* ``random_walk_molecule``: a seeded random-walk chain of atoms (bond length
  1.5 A, isotropic steps) confined to a cubic box; a step is redrawn when it
  would leave the box or land closer than ``min_sep`` to a non-adjacent atom;
  after 200 failed draws the walk restarts from a random earlier atom (a
  branch).  Radii uniform in [r_lo, r_hi]; charges uniform in [q_lo, q_hi],
  shifted by a common constant so that the net charge is the nearest integer.
* ``ses_grid``: the signed distance (positive inside) to the solvent-excluded
  surface for a probe radius, computed by ``ses.c`` (exact in a band around
  the surface, a bound with the right sign elsewhere).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ses.c")
_LIB = os.path.join(_HERE, "libses.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", _LIB + ".tmp",
           _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        lib.ses_sdf.argtypes = [D, D, ctypes.c_int, ctypes.c_double, D, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, D]
        lib.ses_sdf.restype = ctypes.c_int
        _lib = lib
    return _lib


def random_walk_molecule(n_atoms: int, box: float, seed: int, bond=1.5, min_sep=1.0, r_lo=1.2,
                         r_hi=2.0, q_lo=-0.8, q_hi=0.8):
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = np.empty((n_atoms, 3))
    xyz[0] = box / 2.0
    cur = 0
    i = 1
    while i < n_atoms:
        placed = False
        for _ in range(200):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            cand = xyz[cur] + bond * v
            if np.any(cand < 0.0) or np.any(cand > box):
                continue
            d = np.linalg.norm(xyz[:i] - cand, axis=1)
            d[cur] = np.inf  # the atom it bonds to
            if np.min(d) < min_sep:
                continue
            xyz[i] = cand
            cur = i
            i += 1
            placed = True
            break
        if not placed:
            cur = int(rng.integers(0, i))
    radii = rng.uniform(r_lo, r_hi, size=n_atoms)
    q = rng.uniform(q_lo, q_hi, size=n_atoms)
    q += (round(float(q.sum())) - q.sum()) / n_atoms
    return xyz, radii, q


def ses_grid(xyz, radii, h: float, eps_tube: float, probe=1.4, pad_nodes=4):
    """Grid and signed distance to the SES; the tube plus padding fits inside."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    margin = float(np.max(radii)) + eps_tube + (pad_nodes + 2) * h
    lo = xyz.min(axis=0) - margin
    hi = xyz.max(axis=0) + margin
    dims = [int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3)]
    origin = np.ascontiguousarray(lo)
    out = np.empty(dims, dtype=np.float64)
    band = eps_tube + (pad_nodes + 1) * h
    lib = _load()
    D = ctypes.POINTER(ctypes.c_double)
    rc = lib.ses_sdf(xyz.ctypes.data_as(D), radii.ctypes.data_as(D), xyz.shape[0], float(probe),
                     origin.ctypes.data_as(D), dims[0], dims[1], dims[2], float(h), float(band),
                     out.ctypes.data_as(D))
    if rc != 0:
        raise ValueError("ses_sdf: needs at least one atom")
    return out, origin
