"""Thin ctypes binding of libsscs (include/sscs.h).

Argument marshalling only: every step of the solve runs in the HIP library.
The library must have been built (``python -m paper_1903_06477_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsscs.so")

SOLVED, INFEASIBLE, UNBOUNDED, MAX_ITERS, TIME_LIMIT, NUMERICAL = 1, 2, 3, 4, 5, 6
STATUS_NAMES = {1: "solved", 2: "infeasible", 3: "unbounded", 4: "max_iters", 5: "time_limit",
                6: "numerical"}
LINSYS = {"cg": 0, "direct": 1}
DIRECTIONS = {"rb": 0, "aa": 1, "residual": 2, "none": 2, "zero": 3, "scs": 4, "aa_qr": 5}
PRECISIONS = {"fp64": 0, "mixed": 1}

_c_int_p = ctypes.POINTER(ctypes.c_int32)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)


class _Data(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", _c_int_p), ("colind", _c_int_p), ("val", _c_dbl_p),
                ("b", _c_dbl_p), ("c", _c_dbl_p)]


class _Cone(ctypes.Structure):
    _fields_ = [("z", ctypes.c_int32), ("l", ctypes.c_int32), ("nq", ctypes.c_int32), ("q", _c_int_p),
                ("ns", ctypes.c_int32), ("s", _c_int_p), ("ep", ctypes.c_int32)]


class _Settings(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("direction", ctypes.c_int32), ("mem", ctypes.c_int32),
                ("c0", ctypes.c_double), ("c1", ctypes.c_double), ("q", ctypes.c_double),
                ("sigma", ctypes.c_double), ("lambda_", ctypes.c_double), ("thetabar", ctypes.c_double),
                ("ls_max", ctypes.c_int32), ("max_iters", ctypes.c_int64), ("max_time_s", ctypes.c_double),
                ("precision", ctypes.c_int32), ("cg_tol", ctypes.c_double), ("cg_max", ctypes.c_int32),
                ("data_on_device", ctypes.c_int32), ("record_trace", ctypes.c_int32),
                ("aa_reg", ctypes.c_double), ("cg_adapt", ctypes.c_double), ("cg_d_match", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("workgroups", ctypes.c_int32), ("linsys", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64), ("k0", ctypes.c_int64),
                ("k1", ctypes.c_int64), ("k2", ctypes.c_int64), ("km", ctypes.c_int64),
                ("backtracks", ctypes.c_int64), ("cg_iters", ctypes.c_int64),
                ("pr", ctypes.c_double), ("dr", ctypes.c_double), ("gap", ctypes.c_double),
                ("ic", ctypes.c_double), ("uc", ctypes.c_double), ("pobj", ctypes.c_double),
                ("dobj", ctypes.c_double), ("res_fp", ctypes.c_double), ("setup_s", ctypes.c_double),
                ("solve_s", ctypes.c_double)]


EXPORTS = ["sscs_default_settings", "sscs_create", "sscs_solve", "sscs_update_settings", "sscs_update_bc",
           "sscs_destroy", "sscs_linear_step", "sscs_project_dual_cone", "sscs_residual", "sscs_spmv",
           "sscs_spmv_bench", "sscs_get_trace", "sscs_batch_create", "sscs_batch_update_bc",
           "sscs_batch_solve", "sscs_batch_destroy", "sscs_batch_autotune", "sscs_solve_noalloc", "sscs_error_string",
           "sscs_mlp_create", "sscs_mlp_destroy", "sscs_mlp_set_params", "sscs_mlp_get_params",
           "sscs_mlp_forward", "sscs_mlp_train_step", "sscs_mlp_gradients", "sscs_mlp_gemm_nt",
           "sscs_assemble_u0"]

_lib = None


def lib():
    """Loads libsscs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.sscs_error_string.restype = ctypes.c_char_p
        L.sscs_error_string.argtypes = [ctypes.c_int]
        L.sscs_default_settings.argtypes = [ctypes.POINTER(_Settings)]
        L.sscs_create.argtypes = [ctypes.POINTER(_Data), ctypes.POINTER(_Cone), ctypes.POINTER(_Settings), vp,
                                  ctypes.POINTER(vp)]
        L.sscs_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(_Info)]
        L.sscs_update_settings.argtypes = [vp, ctypes.POINTER(_Settings)]
        L.sscs_update_bc.argtypes = [vp, vp, vp]
        L.sscs_destroy.argtypes = [vp]
        L.sscs_linear_step.argtypes = [vp, vp, vp]
        L.sscs_project_dual_cone.argtypes = [vp, vp, vp]
        L.sscs_residual.argtypes = [vp, vp, vp, vp]
        L.sscs_spmv.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.sscs_spmv_bench.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.sscs_get_trace.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.sscs_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(_Data), ctypes.POINTER(_Cone),
                                        ctypes.POINTER(_Settings), vp, ctypes.POINTER(vp)]
        L.sscs_batch_update_bc.argtypes = [vp, vp, vp]
        L.sscs_batch_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(_Info)]
        L.sscs_batch_destroy.argtypes = [vp]
        L.sscs_batch_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp, vp,
                                          vp]
        L.sscs_solve_noalloc.argtypes = [ctypes.POINTER(_Data), ctypes.POINTER(_Cone), ctypes.POINTER(_Settings), vp,
                                         vp, vp, vp, vp, ctypes.POINTER(_Info)]
        _lib = L
    return _lib


class SSCSError(RuntimeError):
    pass


def _check(code: int):
    if code != 0:
        raise SSCSError(f"libsscs error {code}: {lib().sscs_error_string(code).decode()}")


@dataclasses.dataclass
class Settings:
    eps: float = 1e-6
    direction: str = "aa"
    mem: int = 5
    c0: Optional[float] = None       # default: 0.1 for "rb", 0.99 otherwise
    c1: float = 0.9999
    q: float = 0.999
    sigma: float = 0.01
    lam: float = 1.5
    thetabar: float = 0.1
    ls_max: int = 10
    max_iters: int = 10000
    max_time: float = 0.0
    precision: str = "fp64"
    cg_tol: float = 1e-10
    cg_max: int = 500
    data_on_device: bool = False
    record_trace: bool = False
    aa_reg: float = 1e-12
    cg_adapt: float = 0.0
    cg_d_match: bool = True
    check_every: int = 1
    workgroups: int = 0
    linsys: str = "cg"             # "cg" (iterative) or "direct" (dense Cholesky of I + A^T A)

    def to_c(self) -> _Settings:
        st = _Settings()
        st.eps = self.eps
        st.direction = DIRECTIONS[self.direction]
        st.mem = self.mem
        st.c0 = self.c0 if self.c0 is not None else (0.1 if self.direction == "rb" else 0.99)
        st.c1, st.q, st.sigma, st.lambda_, st.thetabar = self.c1, self.q, self.sigma, self.lam, self.thetabar
        st.ls_max = self.ls_max
        st.max_iters = self.max_iters
        st.max_time_s = self.max_time
        st.precision = PRECISIONS[self.precision]
        st.cg_tol = self.cg_tol
        st.cg_max = self.cg_max
        st.data_on_device = int(self.data_on_device)
        st.record_trace = int(self.record_trace)
        st.aa_reg = self.aa_reg
        st.cg_adapt = self.cg_adapt
        st.cg_d_match = int(self.cg_d_match)
        st.check_every = int(self.check_every)
        st.workgroups = int(self.workgroups)
        st.linsys = LINSYS[self.linsys]
        return st


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class _Marshal:
    """Keeps the host arrays of one problem alive while C reads them."""

    def __init__(self, A, b, c, cone):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        A.sort_indices()
        self.rp, self.ci, self.v = _i32(A.indptr), _i32(A.indices), _f64(A.data)
        self.b, self.c = _f64(b), _f64(c)
        self.q = _i32(cone.q if len(cone.q) else [0])
        self.s = _i32(cone.s if len(cone.s) else [0])
        self.data = _Data(A.shape[0], A.shape[1], int(self.v.size), _ptr(self.rp, ctypes.c_int32),
                          _ptr(self.ci, ctypes.c_int32), _ptr(self.v, ctypes.c_double),
                          _ptr(self.b, ctypes.c_double), _ptr(self.c, ctypes.c_double))
        self.cone = _Cone(cone.z, cone.l, len(cone.q), _ptr(self.q, ctypes.c_int32), len(cone.s),
                          _ptr(self.s, ctypes.c_int32), cone.ep)


def _vptr(a) -> int:
    """Address of a numpy array or a torch tensor."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _info_dict(inf: _Info) -> dict:
    d = {k: getattr(inf, k) for k, _ in _Info._fields_}
    d["status_name"] = STATUS_NAMES.get(d["status"], "?")
    return d


class Solver:
    """One instance (A, b, c, K) resident on the GPU."""

    def __init__(self, prob, settings: Optional[Settings] = None, stream=None):
        self.settings = settings or Settings()
        m = _Marshal(prob.A, prob.b, prob.c, prob.cone)
        self.m, self.n = prob.A.shape
        self.N = self.n + self.m + 1
        st = self.settings.to_c()
        h = ctypes.c_void_p()
        _check(lib().sscs_create(ctypes.byref(m.data), ctypes.byref(m.cone), ctypes.byref(st),
                                 ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sscs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def update_settings(self, settings: Settings):
        st = settings.to_c()
        _check(lib().sscs_update_settings(self._h, ctypes.byref(st)))
        self.settings = settings

    def update_bc(self, b, c):
        b, c = (b, c) if self.settings.data_on_device else (_f64(b), _f64(c))
        _check(lib().sscs_update_bc(self._h, _vptr(b), _vptr(c)))

    def _out(self, k):
        return np.empty(k)

    def solve(self, u0=None, out=None):
        """Runs Algorithm 1.  Host numpy arrays unless settings.data_on_device,
        in which case u0 and out=(x, y, s) must be device tensors."""
        if self.settings.data_on_device:
            x, y, s = out
        else:
            x, y, s = (out if out is not None else (self._out(self.n), self._out(self.m), self._out(self.m)))
            if u0 is not None:
                u0 = _f64(u0)
        inf = _Info()
        _check(lib().sscs_solve(self._h, _vptr(u0), _vptr(x), _vptr(y), _vptr(s), ctypes.byref(inf)))
        return x, y, s, _info_dict(inf)

    def linear_step(self, r):
        r = _f64(r)
        out = np.empty(self.N)
        _check(lib().sscs_linear_step(self._h, _vptr(r), _vptr(out)))
        return out

    def residual(self, u):
        u = _f64(u)
        ut, Ru = np.empty(self.N), np.empty(self.N)
        _check(lib().sscs_residual(self._h, _vptr(u), _vptr(ut), _vptr(Ru)))
        return ut, Ru

    def project_dual_cone(self, y):
        y = _f64(y)
        out = np.empty(self.m)
        _check(lib().sscs_project_dual_cone(self._h, _vptr(y), _vptr(out)))
        return out

    def spmv(self, x, transpose=False):
        x = _f64(x)
        out = np.empty(self.m if not transpose else self.n)
        _check(lib().sscs_spmv(self._h, int(transpose), _vptr(x), _vptr(out)))
        return out

    def spmv_bench(self, transpose=False, reps=100):
        ms = ctypes.c_double()
        _check(lib().sscs_spmv_bench(self._h, int(transpose), int(reps), ctypes.byref(ms)))
        return ms.value

    def trace(self, safeguards=False):
        """(res, kind, ls) per iteration of the last solve, and (eta, r_safe)
        after each step when safeguards is set."""
        cnt = ctypes.c_int64()
        _check(lib().sscs_get_trace(self._h, 0, None, None, None, None, None, ctypes.byref(cnt)))
        k = cnt.value
        res, kind, ls = np.empty(k), np.empty(k, np.int32), np.empty(k, np.int32)
        eta, rs = np.empty(k), np.empty(k)
        if k:
            _check(lib().sscs_get_trace(self._h, k, _vptr(res), _vptr(kind), _vptr(ls), _vptr(eta), _vptr(rs),
                                        ctypes.byref(cnt)))
        return (res, kind, ls, eta, rs) if safeguards else (res, kind, ls)


class BatchSolver:
    """Many independent instances solved in one persistent launch."""

    def __init__(self, probs: Sequence, settings: Optional[Settings] = None, stream=None,
                 share_A: bool = False):
        self.settings = settings or Settings()
        self.count = len(probs)
        if share_A:
            # one marshalled copy of A (and the cone sizes); per instance only b and c
            first = _Marshal(probs[0].A, probs[0].b, probs[0].c, probs[0].cone)
            self._marsh = [first]
            self._bc = [(_f64(p.b), _f64(p.c)) for p in probs]
            datas = (_Data * self.count)()
            cones = (_Cone * self.count)()
            for i, (b, c) in enumerate(self._bc):
                d = _Data(first.data.m, first.data.n, first.data.nnz, first.data.rowptr, first.data.colind,
                          first.data.val, _ptr(b, ctypes.c_double), _ptr(c, ctypes.c_double))
                datas[i] = d
                cones[i] = first.cone
        else:
            self._marsh = [_Marshal(p.A, p.b, p.c, p.cone) for p in probs]
            datas = (_Data * self.count)(*[mm.data for mm in self._marsh])
            cones = (_Cone * self.count)(*[mm.cone for mm in self._marsh])
        self.ns = np.array([p.A.shape[1] for p in probs])
        self.ms = np.array([p.A.shape[0] for p in probs])
        st = self.settings.to_c()
        h = ctypes.c_void_p()
        _check(lib().sscs_batch_create(self.count, datas, cones, ctypes.byref(st), ctypes.c_void_p(stream),
                                       ctypes.byref(h)))
        self._h = h
        self._bc = None

    def close(self):
        if getattr(self, "_h", None):
            lib().sscs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_bc(self, b_packed, c_packed):
        """Packed b and c: device tensors when settings.data_on_device, else
        host arrays."""
        if self.settings.data_on_device:
            b, c = b_packed, c_packed
        else:
            b, c = _f64(b_packed), _f64(c_packed)
        _check(lib().sscs_batch_update_bc(self._h, _vptr(b), _vptr(c)))

    def solve(self, u0_packed=None, out=None):
        if self.settings.data_on_device:
            x, y, s = out
        else:
            x, y, s = np.empty(int(self.ns.sum())), np.empty(int(self.ms.sum())), np.empty(int(self.ms.sum()))
            if u0_packed is not None:
                u0_packed = _f64(u0_packed)
        infos = (_Info * self.count)()
        _check(lib().sscs_batch_solve(self._h, _vptr(u0_packed), _vptr(x), _vptr(y), _vptr(s), infos))
        return x, y, s, [_info_dict(infos[i]) for i in range(self.count)]

    def autotune(self, iters: int = 20, cap: int = 8):
        """Tunes the SpMV segment width per size class by timing
        (sscs_batch_autotune); returns one dict per class: the rule's width,
        the kept width and the candidates' times in ms (factor 2^(j-2), -1
        where the width falls outside 1..64)."""
        n = ctypes.c_int32()
        cls, chosen = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
        ms = np.zeros(5 * cap)
        _check(lib().sscs_batch_autotune(self._h, int(iters), int(cap), ctypes.byref(n), _vptr(cls), _vptr(chosen),
                                         _vptr(ms)))
        k = min(cap, n.value)
        return [{"class_seg": int(cls[c]), "chosen_seg": int(chosen[c]), "ms": [float(v) for v in ms[5 * c:5 * c + 5]]}
                for c in range(k)]

    def split(self, x, y, s):
        """Per-instance views of packed outputs."""
        ox = np.concatenate([[0], np.cumsum(self.ns)])
        oy = np.concatenate([[0], np.cumsum(self.ms)])
        return [(x[ox[i]:ox[i + 1]], y[oy[i]:oy[i + 1]], s[oy[i]:oy[i + 1]]) for i in range(self.count)]


def solve_noalloc(prob, settings: Optional[Settings] = None, u0=None, out=None, stream=None):
    """One solve through sscs_solve_noalloc (no device allocation: every
    device buffer lives in the library's static scratch array).  Host numpy
    arrays unless settings.data_on_device, in which case u0 and
    out=(x, y, s) are device tensors."""
    settings = settings or Settings()
    mm = _Marshal(prob.A, prob.b, prob.c, prob.cone)
    m, n = prob.A.shape
    if settings.data_on_device:
        x, y, s = out
    else:
        x, y, s = out if out is not None else (np.empty(n), np.empty(m), np.empty(m))
        if u0 is not None:
            u0 = _f64(u0)
    st = settings.to_c()
    inf = _Info()
    _check(lib().sscs_solve_noalloc(ctypes.byref(mm.data), ctypes.byref(mm.cone), ctypes.byref(st),
                                    ctypes.c_void_p(stream), _vptr(u0), _vptr(x), _vptr(y), _vptr(s),
                                    ctypes.byref(inf)))
    return x, y, s, _info_dict(inf)
