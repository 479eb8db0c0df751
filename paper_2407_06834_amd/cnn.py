"""Thin binding of the warm-start network of libnld (include/nld_cnn.h): argument marshalling
only; every layer runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import nld

P = ctypes.c_void_p
I32 = ctypes.c_int32


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


_sigs = {
    "cnn_create": ([ctypes.POINTER(P), I32, ctypes.c_uint64], ctypes.c_int),
    "cnn_destroy": ([P], ctypes.c_int),
    "cnn_param_count": ([P], ctypes.c_int64),
    "cnn_get_params": ([P, P, P], ctypes.c_int),
    "cnn_set_params": ([P, P], ctypes.c_int),
    "cnn_predict": ([P, P, P, I32, I32, I32, P, P], ctypes.c_int),
    "cnn_loss_grad": ([P, P, P, P, I32, I32, I32, ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
    "cnn_adam_step": ([P, ctypes.POINTER(Adam), P], ctypes.c_int),
}
SYMBOLS = tuple(_sigs)


def _lib():
    lib = nld.load()
    if not getattr(lib, "_cnn_sigs", False):
        for name, (args, res) in _sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        lib._cnn_sigs = True
    return lib


def _img(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 3):
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor (n, h, w)")
    return ctypes.c_void_p(t.data_ptr())


class WarmStartNet:
    """The network of nld_cnn.h; cond rows are (log alpha, log sigma_1..L) per image."""

    def __init__(self, n_cond: int, seed: int = 0):
        lib = _lib()
        h = ctypes.c_void_p()
        nld._check(lib.cnn_create(ctypes.byref(h), int(n_cond), int(seed)))
        self.handle = h
        self.n_cond = n_cond
        self.count = int(lib.cnn_param_count(h))

    def close(self):
        if getattr(self, "handle", None):
            nld._check(_lib().cnn_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        th = np.empty(self.count, dtype=np.float32)
        nld._check(_lib().cnn_get_params(self.handle, th.ctypes.data_as(P), None))
        return th

    def grad(self) -> np.ndarray:
        g = np.empty(self.count, dtype=np.float32)
        nld._check(_lib().cnn_get_params(self.handle, None, g.ctypes.data_as(P)))
        return g

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.count:
            raise ValueError(f"expected {self.count} parameters")
        nld._check(_lib().cnn_set_params(self.handle, th.ctypes.data_as(P)))

    def _cond(self, cond, n):
        c = np.ascontiguousarray(np.asarray(cond, dtype=np.float32).reshape(n, self.n_cond))
        return c, c.ctypes.data_as(P)

    def predict(self, f: torch.Tensor, cond, out: torch.Tensor | None = None, stream=None):
        n, h, w = f.shape
        u0 = torch.empty_like(f) if out is None else out
        c, cp = self._cond(cond, n)
        nld._check(_lib().cnn_predict(self.handle, _img(f, "f"), cp, n, h, w, _img(u0, "u0"),
                                      nld._stream(stream)))
        return u0

    def loss_grad(self, f: torch.Tensor, cond, target: torch.Tensor, stream=None) -> float:
        n, h, w = f.shape
        c, cp = self._cond(cond, n)
        loss = ctypes.c_double()
        nld._check(_lib().cnn_loss_grad(self.handle, _img(f, "f"), cp, _img(target, "target"),
                                        n, h, w, ctypes.byref(loss), nld._stream(stream)))
        return loss.value

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        opt = Adam(lr, beta1, beta2, eps)
        nld._check(_lib().cnn_adam_step(self.handle, ctypes.byref(opt), nld._stream(stream)))
