"""Python binding of libfct (ctypes).

Argument marshalling only: every step of the transform runs in the HIP
library.  Device buffers are PyTorch tensors on the current HIP device and
work is enqueued on PyTorch's current stream.  Importing this module loads
``libfct.so``; if it has not been built, the import fails with an error that
says how to build it (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfct.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libfct is not built ({LIB_PATH} missing); build it with "
        "`python -m paper_2309_14584_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# status codes (include/fct.h)
FCT_OK, FCT_EINVAL, FCT_ENOMEM, FCT_EDEVICE, FCT_ERANK, FCT_ENOCONV, FCT_ENONFINITE = range(7)
FCT_PLAN_ALLOW_RANK_DEFICIENT = 1
FCT_PLAN_GAUSS = 2
FCT_PLAN_ROWS_BY_MEMBER = 4

FAMILY_PLANTED, FAMILY_EXPCOS, FAMILY_GAUSS, FAMILY_RUNGE, FAMILY_OSC = range(5)
DCT_F64, DCT_F32, DCT_BF16X3 = 0, 1, 2
ENGINE_VECTOR, ENGINE_MATRIX = 0, 1
ABI_VERSION = 3          # FCT_ABI_VERSION of the header this binding follows
SOLVE_F64, SOLVE_F32_REFINE, SOLVE_F32 = 0, 1, 2

_vp = ctypes.c_void_p
_i32, _i64, _u32, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double


class PlanInfo(ctypes.Structure):
    _fields_ = [("D", _i32), ("K", _i32), ("n_support", _i64), ("total_points", _i64),
                ("total_rows", _i64), ("max_points", _i64), ("max_degree", _i32),
                ("dct_levels", _i32), ("device_bytes", _i64), ("problems", _i32),
                ("reserved", _i32), ("entries", _i64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", _i32), ("maxit", _i32), ("check_every", _i32),
                ("warm_start", _i32), ("use_graph", _i32), ("timing", _i32),
                ("tol", _dbl), ("max_refine", _i32), ("restart_rounds", _i32),
                ("inner_tol", _dbl), ("single_kernel", _i32), ("one_reduction", _i32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("converged", _i32),
                ("rel_normal_residual", _dbl), ("normal_residual0", _dbl),
                ("rows_kernel_us", _dbl), ("cols_kernel_us", _dbl),
                ("problems", _i32), ("problems_converged", _i32),
                ("refinements", _i32), ("reserved", _i32)]


class CondInfo(ctypes.Structure):
    _fields_ = [("lambda_min", _dbl), ("lambda_max", _dbl), ("kappa", _dbl),
                ("steps", _i32), ("full_rank", _i32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("dct_tile", _i32), ("unit_rows", _i32), ("dct_us", _dbl * 3),
                ("rows_us", _dbl * 4), ("dct_engine", _i32), ("reserved", _i32),
                ("dct_matrix_us", _dbl * 3)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_last_error = _sig("fct_last_error", ctypes.c_char_p)
_status_string = _sig("fct_status_string", ctypes.c_char_p, ctypes.c_int)
abi_version = _sig("fct_abi_version", _i32)
_plan_create = _sig("fct_plan_create", ctypes.c_int, _i32, _i64, _vp, _i32, _vp, _u32, _vp,
                    ctypes.POINTER(_vp))
_plan_destroy = _sig("fct_plan_destroy", None, _vp)
_plan_get_info = _sig("fct_plan_get_info", ctypes.c_int, _vp, ctypes.POINTER(PlanInfo))
_plan_grid = _sig("fct_plan_grid", ctypes.c_int, _vp, _i32, ctypes.POINTER(_i64),
                  ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_plan_export = _sig("fct_plan_export", ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_plan_weights = _sig("fct_plan_weights", ctypes.c_int, _vp, _vp, _vp)
_grid_nodes = _sig("fct_grid_nodes", ctypes.c_int, _vp, _i32, _i32, _vp)
_ws_create = _sig("fct_ws_create", ctypes.c_int, _vp, ctypes.POINTER(_vp))
_ws_destroy = _sig("fct_ws_destroy", None, _vp)
_sample = _sig("fct_sample", ctypes.c_int, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp)
_dct = _sig("fct_dct", ctypes.c_int, _vp, _vp, _vp, _i32, _vp, _vp)
_dct_full = _sig("fct_dct_full", ctypes.c_int, _vp, _vp, _vp, _i32, _vp, _vp)
_apply_A = _sig("fct_apply_A", ctypes.c_int, _vp, _vp, _vp, _vp)
_apply_AT = _sig("fct_apply_AT", ctypes.c_int, _vp, _vp, _vp, _vp)
_batch_create = _sig("fct_batch_create", ctypes.c_int, _i32, ctypes.POINTER(_vp), _vp,
                     ctypes.POINTER(_vp))
_plan_problem = _sig("fct_plan_problem", ctypes.c_int, _vp, _i32, *[ctypes.POINTER(_i64)] * 6)
_ws_problem_info = _sig("fct_ws_problem_info", ctypes.c_int, _vp, _i32, ctypes.POINTER(SolveInfo))
_plan_tune = _sig("fct_plan_tune", ctypes.c_int, _vp, _vp, _i32, _vp, ctypes.POINTER(TuneInfo))
_plan_set_dct_engine = _sig("fct_plan_set_dct_engine", ctypes.c_int, _vp, _i32, _i32)
_eval = _sig("fct_eval", ctypes.c_int, _vp, _vp, _i64, _vp, _vp, _vp, _vp)
_plan_condition = _sig("fct_plan_condition", ctypes.c_int, _vp, _vp, _i32, _dbl, _dbl, _vp,
                       ctypes.POINTER(CondInfo))
_select_grids = _sig("fct_select_grids", ctypes.c_int, _i32, _i64, _vp, _i32, _vp, _dbl, _vp,
                     _i32, _dbl, _dbl, _vp, ctypes.POINTER(_i32), ctypes.POINTER(CondInfo))
_solve = _sig("fct_solve", ctypes.c_int, _vp, _vp, _vp, ctypes.POINTER(SolveOpts),
              ctypes.POINTER(SolveInfo), _vp, _vp)

EXPORTED = ["fct_last_error", "fct_status_string", "fct_abi_version", "fct_plan_create",
            "fct_plan_destroy", "fct_plan_get_info", "fct_plan_grid", "fct_plan_export",
            "fct_grid_nodes", "fct_ws_create", "fct_ws_destroy", "fct_sample", "fct_dct",
            "fct_dct_full", "fct_apply_A", "fct_apply_AT", "fct_solve", "fct_batch_create",
            "fct_plan_problem", "fct_ws_problem_info", "fct_plan_tune",
            "fct_plan_set_dct_engine", "fct_eval", "fct_plan_condition", "fct_select_grids",
            "fct_plan_weights"]


def _cond_dict(info):
    return {"lambda_min": info.lambda_min, "lambda_max": info.lambda_max, "kappa": info.kappa,
            "steps": info.steps, "full_rank": bool(info.full_rank)}


def select_grids(support, candidates, kappa0, v0, max_steps=200, tol=1e-10, rank_tol=1e-10,
                 stream=None):
    """Alg. 2 on the GPU (fct_select_grids): the first L such that the plan
    of candidates[:L] is full rank with kappa(A) <= kappa0.  support int32
    [n, D], candidates int32 [n_cand, D] (host), v0 device double [n].
    Returns (L, estimate dict); L = 0 if no prefix qualifies."""
    torch = _torch()
    S = np.ascontiguousarray(support, dtype=np.int32)
    C = np.ascontiguousarray(candidates, dtype=np.int32)
    n, D = S.shape
    L = _i32(0)
    info = CondInfo()
    st = _select_grids(D, n, S.ctypes.data_as(_vp), C.shape[0], C.ctypes.data_as(_vp),
                       float(kappa0), _ptr(v0, torch.float64, n, "v0"), int(max_steps),
                       float(tol), float(rank_tol), _stream(stream), ctypes.byref(L),
                       ctypes.byref(info))
    if st not in (FCT_OK, FCT_ENOCONV):
        _check(st)
    return L.value, _cond_dict(info)


class FctError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__(f"{_status_string(status).decode()}: {msg}")


def _check(status):
    if status != FCT_OK:
        raise FctError(status, _last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _ptr(t, dtype, numel, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return _vp(t.data_ptr())


@dataclass
class SolveResult:
    iterations: int
    converged: bool
    rel_normal_residual: float
    normal_residual0: float
    status: int
    rows_kernel_us: float = 0.0
    cols_kernel_us: float = 0.0
    problems: int = 1
    problems_converged: int = 0
    refinements: int = 0


class Workspace:
    """A workspace of its own for a plan (fct_ws_create): DCT scratch and
    solver state.  Calls on one plan that run at the same time, on different
    streams, each need one of these."""

    def __init__(self, plan):
        w = _vp()
        _check(_ws_create(plan._h, ctypes.byref(w)))
        self._w = w

    @property
    def handle(self):
        if self._w is None:
            raise ValueError("workspace is closed")
        return self._w

    def close(self):
        if getattr(self, "_w", None):
            _ws_destroy(self._w)
            self._w = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Alias structure of a support on K Lobatto grids, or with gauss=True on
    K Chebyshev-Gauss grids with the DCT-II (fct_plan_create)."""

    def __init__(self, support=None, grids=None, allow_rank_deficient=False, stream=None,
                 _handle=None, gauss=False, rows_by_member=False):
        if _handle is not None:
            self._h = _handle
            self.support = self.grids = None
            self._load_info()
            return
        S = np.ascontiguousarray(np.asarray(support, dtype=np.int32))
        G = np.ascontiguousarray(np.asarray(grids, dtype=np.int32))
        if S.ndim != 2 or G.ndim != 2 or S.shape[1] != G.shape[1]:
            raise ValueError("support [n, D] and grids [K, D] must share D")
        self.support, self.grids = S, G
        h = _vp()
        flags = FCT_PLAN_ALLOW_RANK_DEFICIENT if allow_rank_deficient else 0
        if gauss:
            flags |= FCT_PLAN_GAUSS
        if rows_by_member:
            flags |= FCT_PLAN_ROWS_BY_MEMBER
        _check(_plan_create(S.shape[1], S.shape[0], S.ctypes.data_as(_vp), G.shape[0],
                            G.ctypes.data_as(_vp), flags, _stream(stream), ctypes.byref(h)))
        self._h = h
        self._load_info()

    def _load_info(self):
        info = PlanInfo()
        _check(_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info
        self.D, self.K, self.n = info.D, info.K, info.n_support
        self.M, self.P = info.total_rows, info.total_points
        self.problems = info.problems
        self.entries = info.entries
        self._ws = None

    @classmethod
    def batch(cls, plans, stream=None):
        """Pack single-problem plans into one batch plan (fct_batch_create)."""
        arr = (_vp * len(plans))(*[p._h for p in plans])
        h = _vp()
        _check(_batch_create(len(plans), arr, _stream(stream), ctypes.byref(h)))
        return cls(_handle=h)

    def problem(self, q):
        """(n, rows, col_offset, row_offset, point_offset, points) of problem q."""
        vals = [_i64() for _ in range(6)]
        _check(_plan_problem(self._h, q, *[ctypes.byref(v) for v in vals]))
        return tuple(v.value for v in vals)

    def new_workspace(self):
        return Workspace(self)

    def tune(self, dct_mode=DCT_F64, stream=None, ws=None):
        """Pick the DCT tile size and (for a batch) the LDS unit size by
        timing them on this plan (fct_plan_tune); returns the choices and
        the timings in microseconds."""
        info = TuneInfo()
        _check(_plan_tune(self._h, self._wsh(ws), int(dct_mode), _stream(stream),
                          ctypes.byref(info)))
        pinfo = PlanInfo()
        _check(_plan_get_info(self._h, ctypes.byref(pinfo)))
        self.info = pinfo
        return {"dct_tile": info.dct_tile, "unit_rows": info.unit_rows,
                "dct_engine": info.dct_engine,
                "dct_us": dict(zip((1024, 2048, 4096), info.dct_us)),
                "dct_matrix_us": dict(zip((1024, 2048, 4096), info.dct_matrix_us)),
                "rows_us": dict(zip((4096, 8192, 16384, 32768), info.rows_us))}

    def set_dct_engine(self, dct_mode, engine):
        """Run dct_mode's contractions on ENGINE_VECTOR or ENGINE_MATRIX
        (fct_plan_set_dct_engine)."""
        _check(_plan_set_dct_engine(self._h, int(dct_mode), int(engine)))

    def _wsh(self, ws):
        return self.ws if ws is None else ws.handle

    def problem_result(self, q, ws=None):
        info = SolveInfo()
        _check(_ws_problem_info(self._wsh(ws), q, ctypes.byref(info)))
        return SolveResult(info.iterations, bool(info.converged), info.rel_normal_residual,
                           info.normal_residual0, FCT_OK, 0.0, 0.0, 1, info.problems_converged,
                           info.refinements)

    def close(self):
        if self._ws is not None:
            _ws_destroy(self._ws)
            self._ws = None
        if getattr(self, "_h", None):
            _plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ws(self):
        if self._ws is None:
            w = _vp()
            _check(_ws_create(self._h, ctypes.byref(w)))
            self._ws = w
        return self._ws

    def grid(self, l):
        vals = [_i64() for _ in range(4)]
        _check(_plan_grid(self._h, l, *[ctypes.byref(v) for v in vals]))
        return tuple(v.value for v in vals)   # points, rows, point_offset, row_offset

    def nodes(self, l, i):
        N = int(self.grids[l, i])
        out = np.empty(N + 1)
        _check(_grid_nodes(self._h, l, i, out.ctypes.data_as(_vp)))
        return out

    def export(self, stream=None):
        torch = _torch()
        L = self.K * self.n
        dev = torch.device("cuda", torch.cuda.current_device())
        alias = torch.empty(L, dtype=torch.int64, device=dev)
        perm = torch.empty(L, dtype=torch.int32, device=dev)
        seg = torch.empty(self.M + 1, dtype=torch.int32, device=dev)
        bins = torch.empty(max(self.M, 1), dtype=torch.int64, device=dev)
        rowmap = torch.empty(L, dtype=torch.int32, device=dev)
        _check(_plan_export(self._h, _vp(alias.data_ptr()), _vp(perm.data_ptr()),
                            _vp(seg.data_ptr()), _vp(bins.data_ptr()), _vp(rowmap.data_ptr()),
                            _stream(stream)))
        return dict(alias=alias.view(self.K, self.n), perm=perm.view(self.K, self.n),
                    seg_off=seg, bin_id=bins[: self.M], rowmap=rowmap.view(self.K, self.n))

    def weights(self, stream=None):
        """Entry weights of A, int8 [K, n] on the device (fct_plan_weights)."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        w = torch.empty(self.K * self.n, dtype=torch.int8, device=dev)
        _check(_plan_weights(self._h, _vp(w.data_ptr()), _stream(stream)))
        return w.view(self.K, self.n)

    def _empty(self, n):
        torch = _torch()
        return torch.empty(max(int(n), 1), dtype=torch.float64,
                           device=torch.device("cuda", torch.cuda.current_device()))[: int(n)]

    def sample(self, family, params=(), coeffs=None, out=None, stream=None, ws=None):
        torch = _torch()
        out = self._empty(self.P) if out is None else out
        prm = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
        cptr = _ptr(coeffs, torch.float64, self.n, "coeffs")
        _check(_sample(self._h, int(family), prm.ctypes.data_as(_vp) if prm.size else None,
                       int(prm.size), cptr, _ptr(out, torch.float64, self.P, "out"),
                       self._wsh(ws) if family == FAMILY_PLANTED else None, _stream(stream)))
        return out

    def dct(self, samples, out=None, mode=DCT_F64, stream=None, ws=None):
        torch = _torch()
        out = self._empty(self.M) if out is None else out
        _check(_dct(self._h, _ptr(samples, torch.float64, self.P, "samples"),
                    _ptr(out, torch.float64, self.M, "out"), mode, self._wsh(ws),
                    _stream(stream)))
        return out

    def dct_full(self, samples, out=None, mode=DCT_F64, stream=None, ws=None):
        torch = _torch()
        out = self._empty(self.P) if out is None else out
        _check(_dct_full(self._h, _ptr(samples, torch.float64, self.P, "samples"),
                         _ptr(out, torch.float64, self.P, "out"), mode, self._wsh(ws),
                         _stream(stream)))
        return out

    def eval(self, c, x, out=None, stream=None, ws=None):
        """The expansion with coefficients c (device double [n]) at the
        points x (device double [m, D]) -> device double [m] (fct_eval; the
        plan's workspace lets the support be sliced across the device,
        ws=False evaluates without one)."""
        torch = _torch()
        m = int(x.shape[0]) if x.dim() == 2 else 0
        if x.dim() != 2 or (m and int(x.shape[1]) != self.D):
            raise ValueError(f"x must have shape [m, {self.D}]")
        out = self._empty(m) if out is None else out
        if m == 0:
            return out
        _check(_eval(self._h, _ptr(c, torch.float64, self.n, "c"), m,
                     _ptr(x, torch.float64, m * self.D, "x"),
                     _ptr(out, torch.float64, m, "out"),
                     None if ws is False else self._wsh(ws), _stream(stream)))
        return out

    def condition(self, v0, max_steps=200, tol=1e-10, rank_tol=1e-10, stream=None):
        """Extreme eigenvalues of A^T A and kappa(A) by Lanczos from the
        device vector v0 (fct_plan_condition); returns a dict."""
        torch = _torch()
        info = CondInfo()
        _check(_plan_condition(self._h, _ptr(v0, torch.float64, self.n, "v0"), int(max_steps),
                               float(tol), float(rank_tol), _stream(stream), ctypes.byref(info)))
        return _cond_dict(info)

    def apply_A(self, c, out=None, stream=None):
        torch = _torch()
        out = self._empty(self.M) if out is None else out
        _check(_apply_A(self._h, _ptr(c, torch.float64, self.n, "c"),
                        _ptr(out, torch.float64, self.M, "out"), _stream(stream)))
        return out

    def apply_AT(self, r, out=None, stream=None):
        torch = _torch()
        out = self._empty(self.n) if out is None else out
        _check(_apply_AT(self._h, _ptr(r, torch.float64, self.M, "r"),
                         _ptr(out, torch.float64, self.n, "out"), _stream(stream)))
        return out

    def solve(self, b, out=None, tol=0.0, maxit=0, check_every=0, warm_start=False,
              use_graph=True, mode=SOLVE_F64, raise_on_noconv=True, timing=False,
              max_refine=0, inner_tol=0.0, restart_rounds=False, single_kernel=False,
              one_reduction=False, stream=None, ws=None):
        torch = _torch()
        out = self._empty(self.n) if out is None else out
        opts = SolveOpts(mode, int(maxit), int(check_every), 1 if warm_start else 0,
                         1 if use_graph else 0, 1 if timing else 0, float(tol),
                         int(max_refine), 1 if restart_rounds else 0, float(inner_tol),
                         1 if single_kernel else 0, 1 if one_reduction else 0)
        info = SolveInfo()
        st = _solve(self._h, _ptr(b, torch.float64, self.M, "b"),
                    _ptr(out, torch.float64, self.n, "out"), ctypes.byref(opts),
                    ctypes.byref(info), self._wsh(ws), _stream(stream))
        if st != FCT_OK and (raise_on_noconv or st != FCT_ENOCONV):
            _check(st)
        return out, SolveResult(info.iterations, bool(info.converged),
                                info.rel_normal_residual, info.normal_residual0, st,
                                info.rows_kernel_us, info.cols_kernel_us, info.problems,
                                info.problems_converged, info.refinements)
