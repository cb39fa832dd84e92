"""Checks of the synthetic SES signed distance (input generation).

Pinned against the definition: for a single atom the SES is the atom's own
sphere (exact distance); for two atoms the distance is 1-Lipschitz and equals
the brute-force distance to the exposed part of the probe-centre surface;
on the 500-atom molecule the finite-difference gradient has unit length on
almost every tube node.
"""
import numpy as np

import workloads
from workloads import ses


def test_single_atom_is_exact_sphere():
    xyz = np.array([[0.0, 0.0, 0.0]])
    r = np.array([1.7])
    sdf, origin = ses.ses_grid(xyz, r, 0.25, 0.5)
    n = sdf.shape
    X = origin[:, None, None, None] + 0.25 * np.indices(n)
    rad = np.sqrt((X ** 2).sum(axis=0))
    near = np.abs(1.7 - rad) < 1.2
    assert np.max(np.abs(sdf[near] - (1.7 - rad[near]))) < 1e-12


def _brute_force(x, xyz, R, probe, n=40000, seed=0):
    rng = np.random.default_rng(seed)
    best = np.inf
    for i in range(len(R)):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        P = xyz[i] + R[i] * v
        dd = np.linalg.norm(P[:, None, :] - xyz[None, :, :], axis=2) - R[None, :]
        dd[:, i] = 1.0
        ok = np.all(dd >= 0.0, axis=1)
        if ok.any():
            best = min(best, np.min(np.linalg.norm(P[ok] - x, axis=1)))
    return best - probe


def test_two_atoms_match_brute_force():
    xyz = np.array([[0.0, 0.0, 0.0], [2.6, 0.3, 0.0]])
    r = np.array([1.6, 1.4])
    sdf, origin = ses.ses_grid(xyz, r, 0.3, 0.6)
    rng = np.random.default_rng(1)
    idx = np.argwhere(np.abs(sdf) < 0.6)
    for t in rng.choice(len(idx), size=12, replace=False):
        i, j, k = idx[t]
        x = origin + 0.3 * np.array([i, j, k])
        ref = _brute_force(x, xyz, r + 1.4, 1.4)
        assert abs(sdf[i, j, k] - ref) < 5e-3, (x, sdf[i, j, k], ref)  # sampling resolution


def test_molecule_gradient_unit_length():
    wl = workloads.ses_molecule(60, 12.0, 0.3, 2.0, seed=4)
    d, h = wl.sdf, wl.h
    tube = np.abs(d) < wl.eps_tube
    g = np.gradient(d, h)
    gn = np.sqrt(sum(c * c for c in g))
    dev = np.abs(gn[tube] - 1.0)
    assert np.percentile(dev, 90) < 0.05
    assert np.max(dev) < 1.0  # kinks at ridges only, no jumps
    # the distance is 1-Lipschitz between grid neighbours inside the band where
    # the generator computes it exactly (outside it returns a bound)
    band = wl.eps_tube + 4 * h
    for a in range(3):
        lo = np.take(d, range(d.shape[a] - 1), axis=a)
        hi = np.take(d, range(1, d.shape[a]), axis=a)
        inb = (np.abs(lo) < band) & (np.abs(hi) < band)
        assert np.max(np.abs(hi - lo)[inb]) <= h * (1 + 1e-9)
    # every charge sits inside the molecule
    from scipy import ndimage
    vals = ndimage.map_coordinates(d, ((wl.charge_xyz - wl.origin) / h).T, order=1)
    assert np.all(vals > 0)
    assert abs(wl.charge_q.sum() - round(wl.charge_q.sum())) < 1e-12
