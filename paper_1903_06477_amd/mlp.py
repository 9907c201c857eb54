"""Thin ctypes binding of the warm-start network (include/sscs_mlp.h).

Tensors are torch tensors on cuda:0 (FP32, contiguous); torch only provides
device memory and the stream.  Every step runs in libsscs's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np

from . import sscs as _s

_fp = ctypes.POINTER(ctypes.c_float)
_bound = False


def _lib():
    global _bound
    L = _s.lib()
    if not _bound:
        vp = ctypes.c_void_p
        L.sscs_mlp_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                      ctypes.c_uint64, vp, ctypes.POINTER(vp)]
        L.sscs_mlp_destroy.argtypes = [vp]
        L.sscs_mlp_set_params.argtypes = [vp, ctypes.POINTER(_fp), ctypes.POINTER(_fp)]
        L.sscs_mlp_get_params.argtypes = [vp, ctypes.POINTER(_fp), ctypes.POINTER(_fp)]
        L.sscs_mlp_forward.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.sscs_mlp_train_step.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
        L.sscs_mlp_gradients.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.POINTER(_fp), ctypes.POINTER(_fp),
                                         ctypes.POINTER(ctypes.c_float)]
        L.sscs_mlp_gemm_nt.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        L.sscs_assemble_u0.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        _bound = True
    return L


def _ptrs(arrays):
    return (_fp * len(arrays))(*[a.ctypes.data_as(_fp) for a in arrays])


def _dev(t):
    assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


class MLP:
    def __init__(self, widths: Sequence[int], max_batch: int, seed: int = 0, stream=None):
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        self.stream = stream
        w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        _s._check(_lib().sscs_mlp_create(len(self.widths) - 1, w, self.max_batch, seed, ctypes.c_void_p(stream),
                                         ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib().sscs_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shapes(self):
        return [(self.widths[l + 1], self.widths[l]) for l in range(len(self.widths) - 1)]

    def get_params(self):
        Ws = [np.empty(s, np.float32) for s in self._shapes()]
        bs = [np.empty(s[0], np.float32) for s in self._shapes()]
        _s._check(_lib().sscs_mlp_get_params(self._h, _ptrs(Ws), _ptrs(bs)))
        return Ws, bs

    def set_params(self, Ws, bs):
        Ws = [np.ascontiguousarray(W, np.float32) for W in Ws]
        bs = [np.ascontiguousarray(b, np.float32) for b in bs]
        _s._check(_lib().sscs_mlp_set_params(self._h, _ptrs(Ws), _ptrs(bs)))

    def forward(self, X, out=None):
        import torch
        if out is None:
            out = torch.empty((X.shape[0], self.widths[-1]), dtype=torch.float32, device=X.device)
        _s._check(_lib().sscs_mlp_forward(self._h, X.shape[0], _dev(X), _dev(out)))
        return out

    def train_step(self, X, T, lr: float) -> float:
        loss = ctypes.c_float()
        _s._check(_lib().sscs_mlp_train_step(self._h, X.shape[0], _dev(X), _dev(T), lr, ctypes.byref(loss)))
        return loss.value

    def gradients(self, X, T):
        dWs = [np.empty(s, np.float32) for s in self._shapes()]
        dbs = [np.empty(s[0], np.float32) for s in self._shapes()]
        loss = ctypes.c_float()
        _s._check(_lib().sscs_mlp_gradients(self._h, X.shape[0], _dev(X), _dev(T), _ptrs(dWs), _ptrs(dbs),
                                            ctypes.byref(loss)))
        return loss.value, dWs, dbs


def gemm_nt(A, B, stream=None):
    """C = A B^T on the matrix cores (BF16 operands, FP32 accumulation)."""
    import torch
    M, K = A.shape
    N = B.shape[0]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _s._check(_lib().sscs_mlp_gemm_nt(M, N, K, _dev(A), _dev(B), _dev(C), ctypes.c_void_p(stream)))
    return C


def assemble_u0(pred, n, m, stream=None):
    """u0 rows (x, y + s, 1) in FP64 from prediction rows (x, y, s)."""
    import torch
    count = pred.shape[0]
    u0 = torch.empty((count, n + m + 1), dtype=torch.float64, device=pred.device)
    _s._check(_lib().sscs_assemble_u0(count, n, m, _dev(pred), _dev(u0), ctypes.c_void_p(stream)))
    return u0
