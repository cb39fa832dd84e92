"""Python binding of ``libibim.so`` (the C ABI declared in ``include/ibim.h``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device vectors are ``torch`` float64 CUDA tensors (HIP on ROCm);
the current torch stream is passed to the library unless a stream is given.
The library is loaded from the package directory; if it is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libibim.so")
HEADER = os.path.join(ROOT, "include", "ibim.h")

FP64 = 0
MIXED = 1
CTR2, HYB, KREG = 0, 1, 2  # quadrature of the rows (ibim_options.hybrid)
PRECOND_NONE, PRECOND_DIAG = 0, 1  # system handed to GMRES (ibim_options.precond)
SUM_DIRECT, SUM_TREE = 0, 1  # evaluation of the dense pair sum (ibim_options.summation)

_ERRORS = {
    -1: "IBIM_EINVAL", -2: "IBIM_EGEOM", -3: "IBIM_ENOMEM", -4: "IBIM_EHIP", -5: "IBIM_ENAN",
    -6: "IBIM_ENODEV",
}


class IbimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("check_residual", ctypes.c_int), ("device", ctypes.c_int),
                ("r_near", ctypes.c_double), ("hybrid", ctypes.c_int),
                ("precond", ctypes.c_int), ("summation", ctypes.c_int),
                ("tree_order", ctypes.c_int), ("tree_theta", ctypes.c_double),
                ("tree_min_nodes", ctypes.c_int64), ("pair_scratch_max", ctypes.c_int64)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("applies", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_resid", ctypes.c_double), ("explicit_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("finished", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("batched_items", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t), ("active", ctypes.c_int),
                ("waiting", ctypes.c_int), ("max_active_seen", ctypes.c_int),
                ("held_for_slot", ctypes.c_int64), ("held_for_budget", ctypes.c_int64),
                ("estimate_shortfall", ctypes.c_size_t)]


REQ_WAITING, REQ_ACTIVE, REQ_DONE, REQ_FAILED = 0, 1, 2, -1

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_VP = ctypes.c_void_p


def header_functions() -> list[str]:
    """Names of the functions declared in ``include/ibim.h``."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ibim_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load ``libibim.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_03699_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7) and opens it by
    # an unversioned name; loading torch first makes this library bind to that
    # same runtime, so torch streams and device pointers are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    lib.ibim_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.ibim_default_options.restype = None
    lib.ibim_last_error.restype = ctypes.c_char_p
    lib.ibim_setup.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               _D, _D, ctypes.c_int, ctypes.POINTER(_Options), _VP,
                               ctypes.POINTER(_VP)]
    lib.ibim_destroy.argtypes = [_VP]
    lib.ibim_destroy.restype = None
    lib.ibim_num_nodes.argtypes = [_VP, _I64]
    lib.ibim_context_options.argtypes = [_VP, ctypes.POINTER(_Options)]
    lib.ibim_node_grid_index.argtypes = [_VP, _I64]
    lib.ibim_node_geometry.argtypes = [_VP, _D, _D, _D]
    lib.ibim_num_corrections.argtypes = [_VP, _I64]
    lib.ibim_node_flags.argtypes = [_VP, ctypes.POINTER(ctypes.c_uint8), _I64]
    lib.ibim_corrections.argtypes = [_VP, _I64, _I64, _I32, _D, _D, _D]
    lib.ibim_correction_weights.argtypes = [_VP, _D, _D, _VP]
    lib.ibim_rhs.argtypes = [_VP, _VP, _VP]
    lib.ibim_apply.argtypes = [_VP, _VP, _VP, _VP]
    lib.ibim_apply_noalloc.argtypes = [_VP, _VP, _VP, _VP]
    lib.ibim_solve.argtypes = [_VP, _VP, ctypes.c_double, _VP, ctypes.POINTER(_SolveInfo), _VP]
    lib.ibim_solve_guess.argtypes = lib.ibim_solve.argtypes
    lib.ibim_energy.argtypes = [_VP, _VP, _D, _VP]
    lib.ibim_pair_timing.argtypes = [_VP, ctypes.c_int]
    lib.ibim_pair_timing_read.argtypes = [_VP, _I64, _D]
    lib.ibim_pair_work.argtypes = [_VP, _D, _D]
    lib.ibim_tree_counts.argtypes = [_VP, _D]
    lib.ibim_tree_plan.argtypes = [_VP, _I64] + [_I32] * 4 + [_D] + [_I32] * 8 + [_D]
    lib.ibim_tree_pairs.argtypes = [_VP, _I64, _I32, _I32]
    lib.ibim_server_create.argtypes = [ctypes.POINTER(_Options), ctypes.c_size_t, ctypes.c_int,
                                       ctypes.c_int, _VP, ctypes.POINTER(_VP)]
    lib.ibim_server_submit.argtypes = [_VP, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_int,
                                       ctypes.c_double, _I64]
    lib.ibim_server_step.argtypes = [_VP, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int)]
    lib.ibim_server_poll.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_int), _D,
                                     ctypes.POINTER(_SolveInfo)]
    lib.ibim_server_solution.argtypes = [_VP, ctypes.c_int64, _D, _I64]
    lib.ibim_server_release.argtypes = [_VP, ctypes.c_int64]
    lib.ibim_server_get_stats.argtypes = [_VP, ctypes.POINTER(_ServerStats)]
    lib.ibim_server_destroy.argtypes = [_VP]
    lib.ibim_server_destroy.restype = None
    _lib = lib
    return lib


def _check(code):
    if code < 0:
        raise IbimError(code, load().ibim_last_error().decode())
    return code


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _stream_ptr(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def _dev_ptr(t, n=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 device tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """One discretised problem (``ibim_setup``) and its solve entry points."""

    def __init__(self, sdf, origin, h, eps_tube, eps_in, eps_out, kappa, charge_xyz=None,
                 charge_q=None, precision=FP64, restart=60, max_iter=300, check_residual=True,
                 device=0, r_near=0.0, hybrid=CTR2, precond=PRECOND_DIAG, summation=SUM_DIRECT,
                 tree_order=8, tree_theta=0.7, tree_min_nodes=0, pair_scratch_max=0, stream=None):
        lib = load()
        self._lib = lib
        sdf = np.ascontiguousarray(sdf, dtype=np.float64)
        if sdf.ndim != 3:
            raise ValueError("sdf must be a 3-D array")
        origin = np.ascontiguousarray(origin, dtype=np.float64).reshape(3)
        zq = np.ascontiguousarray(np.zeros((0, 3)) if charge_xyz is None else charge_xyz,
                                  dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(np.zeros(0) if charge_q is None else charge_q, dtype=np.float64)
        if q.shape[0] != zq.shape[0]:
            raise ValueError("charge_xyz and charge_q disagree")
        opt = _Options()
        lib.ibim_default_options(ctypes.byref(opt))
        opt.precision = int(precision)
        opt.restart = int(restart)
        opt.max_iter = int(max_iter)
        opt.check_residual = int(bool(check_residual))
        opt.device = int(device)
        opt.r_near = float(r_near)
        opt.hybrid = int(hybrid)
        opt.precond = int(precond)
        opt.summation = int(summation)
        opt.tree_order = int(tree_order)
        opt.tree_theta = float(tree_theta)
        opt.tree_min_nodes = int(tree_min_nodes)
        opt.pair_scratch_max = int(pair_scratch_max)
        self.device = int(device)
        self.h = float(h)
        ctx = ctypes.c_void_p()
        st = ctypes.c_void_p(0) if device < 0 else _stream_ptr(stream)
        _check(lib.ibim_setup(_dp(sdf), sdf.shape[0], sdf.shape[1], sdf.shape[2], _dp(origin),
                              float(h), float(eps_tube), float(eps_in), float(eps_out),
                              float(kappa), _dp(zq), _dp(q), int(q.shape[0]), ctypes.byref(opt),
                              st, ctypes.byref(ctx)))
        self._ctx = ctx
        M = ctypes.c_int64()
        _check(lib.ibim_num_nodes(ctx, ctypes.byref(M)))
        self.M = int(M.value)
        nnz = ctypes.c_int64()
        _check(lib.ibim_num_corrections(ctx, ctypes.byref(nnz)))
        self.nnz = int(nnz.value)
        eff = _Options()
        _check(lib.ibim_context_options(ctx, ctypes.byref(eff)))
        #: summation and precision this problem runs with (IBIM_SUM_TREE is
        #: resolved by size: direct below tree_min_nodes, the treecode above)
        self.summation = int(eff.summation)
        self.precision = int(eff.precision)

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.sdf, wl.origin, wl.h, wl.eps_tube, wl.eps_in, wl.eps_out, wl.kappa,
                   wl.charge_xyz, wl.charge_q, **kw)

    def close(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            self._lib.ibim_destroy(ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host inspection ----------------------------------------------------
    def node_grid_index(self) -> np.ndarray:
        out = np.empty(self.M, np.int64)
        _check(self._lib.ibim_node_grid_index(self._ctx, out.ctypes.data_as(_I64)))
        return out

    def node_geometry(self):
        P = np.empty((self.M, 3))
        n = np.empty((self.M, 3))
        w = np.empty(self.M)
        _check(self._lib.ibim_node_geometry(self._ctx, _dp(P), _dp(n), _dp(w)))
        return P, n, w

    def node_flags(self) -> np.ndarray:
        """Boolean per node: in M_B (K-reg row, J = 1)."""
        out = np.empty(self.M, np.uint8)
        _check(self._lib.ibim_node_flags(self._ctx, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_uint8)), None))
        return out.astype(bool)

    def corrections(self) -> dict:
        out = {"row": np.empty(self.M + 1, np.int64), "col": np.empty(self.nnz, np.int64),
               "axis": np.empty(self.nnz, np.int32), "alpha": np.empty(self.nnz),
               "beta": np.empty(self.nnz), "eta": np.empty(self.nnz)}
        _check(self._lib.ibim_corrections(self._ctx, out["row"].ctypes.data_as(_I64),
                                          out["col"].ctypes.data_as(_I64),
                                          out["axis"].ctypes.data_as(_I32), _dp(out["alpha"]),
                                          _dp(out["beta"]), _dp(out["eta"])))
        return out

    def correction_weights(self, stream=None):
        om11 = np.empty(self.nnz)
        om21 = np.empty(self.nnz)
        _check(self._lib.ibim_correction_weights(self._ctx, _dp(om11), _dp(om21),
                                                 _stream_ptr(stream)))
        return om11, om21

    # -- device entry points ------------------------------------------------
    def new_vector(self):
        import torch
        return torch.empty(2 * self.M, dtype=torch.float64, device=f"cuda:{self.device}")

    def rhs(self, out=None, stream=None):
        g = self.new_vector() if out is None else out
        _check(self._lib.ibim_rhs(self._ctx, _dev_ptr(g, 2 * self.M), _stream_ptr(stream)))
        return g

    def apply(self, u, out=None, stream=None):
        out = self.new_vector() if out is None else out
        _check(self._lib.ibim_apply(self._ctx, _dev_ptr(u, 2 * self.M),
                                    _dev_ptr(out, 2 * self.M), _stream_ptr(stream)))
        return out

    def apply_noalloc(self, u, out, stream=None):
        """``ibim_apply_noalloc``: as :meth:`apply` into a caller-supplied
        ``out``, with the pair sum's partial sums in the library's static
        device scratch (no device allocation)."""
        _check(self._lib.ibim_apply_noalloc(self._ctx, _dev_ptr(u, 2 * self.M),
                                            _dev_ptr(out, 2 * self.M), _stream_ptr(stream)))
        return out

    def solve(self, rhs, tol, x=None, stream=None, warm=False):
        """GMRES from x0 = 0, or (warm=True) from the given x, which is updated in place."""
        if warm and x is None:
            raise ValueError("a warm start needs x")
        x = self.new_vector() if x is None else x
        info = _SolveInfo()
        fn = self._lib.ibim_solve_guess if warm else self._lib.ibim_solve
        code = _check(fn(self._ctx, _dev_ptr(rhs, 2 * self.M), float(tol),
                         _dev_ptr(x, 2 * self.M), ctypes.byref(info), _stream_ptr(stream)))
        return x, {"status": int(code), "iters": info.iters, "applies": info.applies,
                   "converged": bool(info.converged),
                   "rel_resid": info.rel_resid, "explicit_rel_resid": info.explicit_rel_resid,
                   "seconds": info.seconds}

    def energy(self, x, stream=None) -> float:
        g = ctypes.c_double()
        _check(self._lib.ibim_energy(self._ctx, _dev_ptr(x, 2 * self.M), ctypes.byref(g),
                                     _stream_ptr(stream)))
        return float(g.value)

    def pair_timing(self, enable: bool):
        _check(self._lib.ibim_pair_timing(self._ctx, int(bool(enable))))

    def pair_timing_read(self):
        """(launches, total milliseconds) of the pair kernels timed so far."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(self._lib.ibim_pair_timing_read(self._ctx, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def pair_work(self):
        """(ordered pairs, flops) of one dense pair-sum launch (``ibim_pair_work``)."""
        p = ctypes.c_double()
        f = ctypes.c_double()
        _check(self._lib.ibim_pair_work(self._ctx, ctypes.byref(p), ctypes.byref(f)))
        return float(p.value), float(f.value)

    def tree_counts(self):
        """Work of one treecode pair sum (``ibim_tree_counts``)."""
        out = np.zeros(6)
        _check(self._lib.ibim_tree_counts(self._ctx, _dp(out)))
        return {"far_evals": out[0], "near_evals": out[1], "proxy_terms": out[2],
                "batches": int(out[3]), "proxy_clusters": int(out[4]),
                "transfers": int(out[5])}

    def tree_pairs(self):
        """Two-way pairs of the treecode plan (``ibim_tree_pairs``): (lower, upper) batches."""
        n = np.zeros(1, dtype=np.int64)
        nul = ctypes.POINTER(ctypes.c_int32)()
        _check(self._lib.ibim_tree_pairs(self._ctx, n.ctypes.data_as(_I64), nul, nul))
        lo = np.zeros(int(n[0]), dtype=np.int32)
        hi = np.zeros(int(n[0]), dtype=np.int32)
        _check(self._lib.ibim_tree_pairs(self._ctx, n.ctypes.data_as(_I64),
                                         lo.ctypes.data_as(_I32), hi.ctypes.data_as(_I32)))
        return lo, hi

    def tree_plan(self):
        """The treecode plan (``ibim_tree_plan``) as numpy arrays."""
        cnt = np.zeros(8, dtype=np.int64)
        nul = ctypes.POINTER(ctypes.c_int32)()
        dnul = ctypes.POINTER(ctypes.c_double)()
        _check(self._lib.ibim_tree_plan(self._ctx, cnt.ctypes.data_as(_I64), *([nul] * 4), dnul,
                                        *([nul] * 8), dnul))
        M, B, C, F, R = (int(v) for v in cnt[:5])
        i32 = lambda n: np.zeros(max(n, 0), dtype=np.int32)
        out = {"perm": i32(M), "bstart": i32(B + 1), "cstart": i32(C), "cend": i32(C),
               "cbox": np.zeros(6 * C), "kid": i32(2 * C), "dstart": i32(C), "dend": i32(C),
               "frow": i32(B + 1), "fcol": i32(F), "nrow": i32(B + 1), "nlo": i32(R),
               "nhi": i32(R)}
        gap = np.zeros(1)
        p = lambda a: a.ctypes.data_as(_I32)
        _check(self._lib.ibim_tree_plan(
            self._ctx, cnt.ctypes.data_as(_I64), p(out["perm"]), p(out["bstart"]),
            p(out["cstart"]), p(out["cend"]), _dp(out["cbox"]), p(out["kid"]), p(out["dstart"]),
            p(out["dend"]), p(out["frow"]), p(out["fcol"]), p(out["nrow"]), p(out["nlo"]),
            p(out["nhi"]), _dp(gap)))
        out["cbox"] = out["cbox"].reshape(-1, 6)
        out["gap"] = float(gap[0])
        out["items"] = int(cnt[5])
        out["order"] = int(cnt[6])
        return out

    def solve_energy(self, tol, stream=None):
        g = self.rhs(stream=stream)
        x, info = self.solve(g, tol, stream=stream)
        info["g_pol"] = self.energy(x, stream=stream)
        return x, info


def _info_dict(info):
    return {"iters": info.iters, "applies": info.applies, "converged": bool(info.converged),
            "rel_resid": info.rel_resid, "explicit_rel_resid": info.explicit_rel_resid,
            "seconds": info.seconds}


class Server:
    """Continuous-batching solve server (``ibim_server_*``): many independent
    problems share one persistent batched pair-kernel launch per round."""

    def __init__(self, hbm_budget_bytes, max_slots=16, host_threads=4, precision=FP64,
                 restart=60, max_iter=300, check_residual=True, device=0, r_near=0.0,
                 hybrid=CTR2, precond=PRECOND_DIAG, summation=SUM_DIRECT, tree_order=8,
                 tree_theta=0.7, tree_min_nodes=0, pair_scratch_max=0, stream=None):
        lib = load()
        self._lib = lib
        opt = _Options()
        lib.ibim_default_options(ctypes.byref(opt))
        opt.precision = int(precision)
        opt.restart = int(restart)
        opt.max_iter = int(max_iter)
        opt.check_residual = int(bool(check_residual))
        opt.device = int(device)
        opt.r_near = float(r_near)
        opt.hybrid = int(hybrid)
        opt.precond = int(precond)
        opt.summation = int(summation)
        opt.tree_order = int(tree_order)
        opt.tree_theta = float(tree_theta)
        opt.tree_min_nodes = int(tree_min_nodes)
        opt.pair_scratch_max = int(pair_scratch_max)
        srv = ctypes.c_void_p()
        _check(lib.ibim_server_create(ctypes.byref(opt), int(hbm_budget_bytes), int(max_slots),
                                      int(host_threads), _stream_ptr(stream), ctypes.byref(srv)))
        self._srv = srv

    def submit(self, sdf, origin, h, eps_tube, eps_in, eps_out, kappa, charge_xyz=None,
               charge_q=None, tol=1e-8) -> int:
        sdf = np.ascontiguousarray(sdf, dtype=np.float64)
        if sdf.ndim != 3:
            raise ValueError("sdf must be a 3-D array")
        origin = np.ascontiguousarray(origin, dtype=np.float64).reshape(3)
        zq = np.ascontiguousarray(np.zeros((0, 3)) if charge_xyz is None else charge_xyz,
                                  dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(np.zeros(0) if charge_q is None else charge_q, dtype=np.float64)
        if q.shape[0] != zq.shape[0]:
            raise ValueError("charge_xyz and charge_q disagree")
        t = ctypes.c_int64()
        _check(self._lib.ibim_server_submit(self._srv, _dp(sdf), sdf.shape[0], sdf.shape[1],
                                            sdf.shape[2], _dp(origin), float(h), float(eps_tube),
                                            float(eps_in), float(eps_out), float(kappa), _dp(zq),
                                            _dp(q), int(q.shape[0]), float(tol), ctypes.byref(t)))
        return int(t.value)

    def submit_workload(self, wl, tol=None) -> int:
        return self.submit(wl.sdf, wl.origin, wl.h, wl.eps_tube, wl.eps_in, wl.eps_out, wl.kappa,
                           wl.charge_xyz, wl.charge_q, tol=wl.tol if tol is None else tol)

    def step(self):
        """One round; returns (active, waiting)."""
        a = ctypes.c_int()
        w = ctypes.c_int()
        _check(self._lib.ibim_server_step(self._srv, ctypes.byref(a), ctypes.byref(w)))
        return int(a.value), int(w.value)

    def poll(self, ticket):
        """(state, g_pol or None, info dict or None); raises IbimError for a failed request."""
        st = ctypes.c_int()
        g = ctypes.c_double()
        info = _SolveInfo()
        _check(self._lib.ibim_server_poll(self._srv, int(ticket), ctypes.byref(st),
                                          ctypes.byref(g), ctypes.byref(info)))
        if st.value == REQ_DONE:
            return REQ_DONE, float(g.value), _info_dict(info)
        return int(st.value), None, None

    def state(self, ticket) -> int:
        st = ctypes.c_int()
        code = self._lib.ibim_server_poll(self._srv, int(ticket), ctypes.byref(st), None, None)
        if code < 0 and st.value != REQ_FAILED:
            _check(code)
        return int(st.value)

    def solution(self, ticket) -> np.ndarray:
        M = ctypes.c_int64()
        _check(self._lib.ibim_server_solution(self._srv, int(ticket), None, ctypes.byref(M)))
        x = np.empty(2 * M.value)
        _check(self._lib.ibim_server_solution(self._srv, int(ticket), _dp(x), ctypes.byref(M)))
        return x

    def release(self, ticket):
        _check(self._lib.ibim_server_release(self._srv, int(ticket)))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(self._lib.ibim_server_get_stats(self._srv, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def run_until_idle(self, max_rounds=1_000_000):
        for _ in range(max_rounds):
            a, w = self.step()
            if a == 0 and w == 0:
                return
        raise RuntimeError("server did not drain")

    def close(self):
        srv = getattr(self, "_srv", None)
        if srv is not None and srv.value:
            self._lib.ibim_server_destroy(srv)
        self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
