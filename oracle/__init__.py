"""FP64 CPU oracle for the CTR-IBIM discretisation (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
built by :func:`build`) with ``ctypes`` and ``numpy``; it shares no code with
the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (no FMA contraction, OpenMP rows)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
        "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oc_build.restype = ctypes.c_void_p
    lib.oc_build.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oc_build_rows.restype = ctypes.c_void_p
    lib.oc_build_rows.argtypes = lib.oc_build.argtypes + [_I64, ctypes.c_int64]
    lib.oc_build_hyb.restype = ctypes.c_void_p
    lib.oc_build_hyb.argtypes = lib.oc_build.argtypes + [ctypes.c_int, _I64, ctypes.c_int64]
    lib.oc_get_bad.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8)]
    lib.oc_kreg_c12.restype = ctypes.c_double
    lib.oc_kreg_c12.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oc_free.argtypes = [ctypes.c_void_p]
    lib.oc_last_error.restype = ctypes.c_char_p
    lib.oc_num_nodes.restype = ctypes.c_int64
    lib.oc_num_nodes.argtypes = [ctypes.c_void_p]
    lib.oc_num_corrections.restype = ctypes.c_int64
    lib.oc_num_corrections.argtypes = [ctypes.c_void_p]
    lib.oc_get_nodes.argtypes = [ctypes.c_void_p, _I32] + [_D] * 8
    lib.oc_get_corrections.argtypes = [ctypes.c_void_p, _I64, _I64, _I32] + [_D] * 5
    lib.oc_apply.argtypes = [ctypes.c_void_p, _D, _D]
    lib.oc_apply_rows.argtypes = [ctypes.c_void_p, _D, _I64, ctypes.c_int64, _D, _D]
    lib.oc_rhs.argtypes = [ctypes.c_void_p, _D, _D, ctypes.c_int, _D]
    lib.oc_energy.restype = ctypes.c_double
    lib.oc_energy.argtypes = [ctypes.c_void_p, _D, _D, _D, ctypes.c_int]
    lib.oc_psi_rxn.restype = ctypes.c_double
    lib.oc_psi_rxn.argtypes = [ctypes.c_void_p, _D, _D]
    lib.oc_area.restype = ctypes.c_double
    lib.oc_area.argtypes = [ctypes.c_void_p]
    lib.oc_gmres.restype = ctypes.c_int
    lib.oc_gmres.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int), _D, _D]
    lib.oc_lattice_sums.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D]
    lib.oc_ell.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                           ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, _D, _D]
    lib.oc_plane_weights.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
    lib.oc_kernels.argtypes = [_D, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               _D]
    lib.oc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oc_num_threads())


class Oracle:
    """One discretised problem: tube nodes, geometry, correction sets, weights."""

    def __init__(self, sdf, origin, h, eps_tube, eps_in, eps_out, kappa, weight_rows=None,
                 hybrid=0):
        """``weight_rows``: build correction weights only for these rows (the
        others hold NaN, so only ``apply_rows`` on listed rows is meaningful).
        ``hybrid``: 0 CTR2 rows everywhere, 1 HYB-IBIM (K-reg rows and J = 1
        at bad nodes), 2 every node bad (K-reg everywhere, J = 1)."""
        lib = _load()
        self._lib = lib
        sdf = _f64(sdf)
        assert sdf.ndim == 3
        origin = _f64(origin)
        self.h, self.eps, self.eps_in, self.eps_out, self.kappa = (
            float(h), float(eps_tube), float(eps_in), float(eps_out), float(kappa))
        self._sdf = sdf
        self.hybrid = int(hybrid)
        if weight_rows is None:
            ptr = lib.oc_build_hyb(_dp(sdf), sdf.shape[0], sdf.shape[1], sdf.shape[2],
                                   _dp(origin), self.h, self.eps, self.eps_in, self.eps_out,
                                   self.kappa, self.hybrid, None, 0)
        else:
            wr = np.ascontiguousarray(weight_rows, dtype=np.int64)
            ptr = lib.oc_build_hyb(_dp(sdf), sdf.shape[0], sdf.shape[1], sdf.shape[2],
                                   _dp(origin), self.h, self.eps, self.eps_in, self.eps_out,
                                   self.kappa, self.hybrid, wr.ctypes.data_as(_I64), wr.shape[0])
        if not ptr:
            raise ValueError("oracle setup failed: " + lib.oc_last_error().decode())
        self._c = ctypes.c_void_p(ptr)
        self.M = int(lib.oc_num_nodes(self._c))
        self.nnz = int(lib.oc_num_corrections(self._c))

    @classmethod
    def from_workload(cls, wl, weight_rows=None, hybrid=0):
        return cls(wl.sdf, wl.origin, wl.h, wl.eps_tube, wl.eps_in, wl.eps_out, wl.kappa,
                   weight_rows=weight_rows, hybrid=hybrid)

    def bad_nodes(self) -> np.ndarray:
        """Boolean per node: in M_B (K-reg row, J = 1)."""
        out = np.empty(self.M, np.uint8)
        self._lib.oc_get_bad(self._c, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return out.astype(bool)

    def __del__(self):
        c = getattr(self, "_c", None)
        if c is not None and c.value:
            self._lib.oc_free(c)
            self._c = None

    # -- geometry and corrections ------------------------------------------
    def nodes(self) -> dict:
        M = self.M
        out = {
            "ijk": np.empty((M, 3), np.int32), "y": np.empty((M, 3)), "d": np.empty(M),
            "P": np.empty((M, 3)), "n": np.empty((M, 3)), "J": np.empty(M), "w": np.empty(M),
            "kappa": np.empty((M, 2)), "tau": np.empty((M, 2, 3)),
        }
        self._lib.oc_get_nodes(self._c, out["ijk"].ctypes.data_as(_I32), _dp(out["y"]),
                               _dp(out["d"]), _dp(out["P"]), _dp(out["n"]), _dp(out["J"]),
                               _dp(out["w"]), _dp(out["kappa"]), _dp(out["tau"]))
        return out

    def corrections(self) -> dict:
        n = self.nnz
        out = {
            "row": np.empty(self.M + 1, np.int64), "col": np.empty(n, np.int64),
            "axis": np.empty(n, np.int32), "alpha": np.empty(n), "beta": np.empty(n),
            "eta": np.empty(n), "om11": np.empty(n), "om21": np.empty(n),
        }
        self._lib.oc_get_corrections(self._c, out["row"].ctypes.data_as(_I64),
                                     out["col"].ctypes.data_as(_I64),
                                     out["axis"].ctypes.data_as(_I32), _dp(out["alpha"]),
                                     _dp(out["beta"]), _dp(out["eta"]), _dp(out["om11"]),
                                     _dp(out["om21"]))
        return out

    def area(self) -> float:
        return float(self._lib.oc_area(self._c))

    # -- operator ------------------------------------------------------------
    def apply(self, u) -> np.ndarray:
        u = _f64(u)
        assert u.shape == (2 * self.M,)
        out = np.empty(2 * self.M)
        self._lib.oc_apply(self._c, _dp(u), _dp(out))
        return out

    def apply_rows(self, u, rows):
        u = _f64(u)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        o1 = np.empty(rows.shape[0])
        o2 = np.empty(rows.shape[0])
        self._lib.oc_apply_rows(self._c, _dp(u), rows.ctypes.data_as(_I64), rows.shape[0],
                                _dp(o1), _dp(o2))
        return o1, o2

    def rhs(self, charge_xyz, charge_q) -> np.ndarray:
        z = _f64(charge_xyz).reshape(-1, 3)
        q = _f64(charge_q)
        g = np.empty(2 * self.M)
        self._lib.oc_rhs(self._c, _dp(z), _dp(q), int(q.shape[0]), _dp(g))
        return g

    def energy(self, x, charge_xyz, charge_q) -> float:
        x = _f64(x)
        z = _f64(charge_xyz).reshape(-1, 3)
        q = _f64(charge_q)
        return float(self._lib.oc_energy(self._c, _dp(x), _dp(z), _dp(q), int(q.shape[0])))

    def psi_rxn(self, x, z) -> float:
        return float(self._lib.oc_psi_rxn(self._c, _dp(_f64(x)), _dp(_f64(z))))

    def gmres(self, b, tol, restart=60, maxit=300, precond=1):
        """GMRES(restart) from x0 = 0; precond 1: on D^-1 A x = D^-1 b (D = Lambda)."""
        b = _f64(b)
        x = np.empty(2 * self.M)
        it = ctypes.c_int(0)
        est = np.zeros(1)
        true = np.zeros(1)
        status = self._lib.oc_gmres(self._c, _dp(b), float(tol), int(restart), int(maxit),
                                    int(precond), _dp(x), ctypes.byref(it), _dp(est), _dp(true))
        return x, {"status": int(status), "iters": int(it.value), "est_relres": float(est[0]),
                   "true_relres": float(true[0])}

    def solve_energy(self, charge_xyz, charge_q, tol, restart=60, maxit=300, precond=1):
        g = self.rhs(charge_xyz, charge_q)
        x, info = self.gmres(g, tol, restart, maxit, precond)
        info["g_pol"] = self.energy(x, charge_xyz, charge_q)
        return x, info


# -- free functions used by the weight and expansion pins -------------------
def kreg_c12(kappa: float, tau: float) -> float:
    """K-reg constant of K12 for radius tau (Section 2.3)."""
    return float(_load().oc_kreg_c12(float(kappa), float(tau)))


def lattice_sums(alpha: float, beta: float, nmode: int = 41):
    """Z_{2j}(alpha, beta), j < nmode (complex), the regularised lattice sums."""
    lib = _load()
    zr = np.empty(nmode)
    zi = np.empty(nmode)
    lib.oc_lattice_sums(float(alpha), float(beta), int(nmode), _dp(zr), _dp(zi))
    return zr + 1j * zi


def ell(tau1, tau2, k1, k2, eta, ax_a, ax_b, eps_in, eps_out, kappa, theta):
    lib = _load()
    l11 = ctypes.c_double()
    l21 = ctypes.c_double()
    lib.oc_ell(_dp(_f64(tau1)), _dp(_f64(tau2)), k1, k2, eta, ax_a, ax_b, eps_in, eps_out, kappa,
               theta, ctypes.byref(l11), ctypes.byref(l21))
    return l11.value, l21.value


def plane_weights(tau1, tau2, k1, k2, eta, ax_a, ax_b, alpha, beta, eps_in, eps_out, kappa):
    lib = _load()
    o11 = ctypes.c_double()
    o21 = ctypes.c_double()
    lib.oc_plane_weights(_dp(_f64(tau1)), _dp(_f64(tau2)), k1, k2, eta, ax_a, ax_b, alpha, beta,
                         eps_in, eps_out, kappa, ctypes.byref(o11), ctypes.byref(o21))
    return o11.value, o21.value


def kernels(x, nx, y, ny, eps_in, eps_out, kappa):
    lib = _load()
    K = np.empty(4)
    lib.oc_kernels(_dp(_f64(x)), _dp(_f64(nx)), _dp(_f64(y)), _dp(_f64(ny)), eps_in, eps_out,
                   kappa, _dp(K))
    return K
