"""ctypes wrapper of the C/OpenMP direct-sum rows (csum.c).  Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csum.c")
_LIB = os.path.join(_HERE, "_csum.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile csum.c with gcc (-O2 -fopenmp, no fast-math) into oracle/_csum.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC,
                               "-lm"])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        f = lib.oracle_anova_rows
        P = ctypes.c_void_p
        f.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P,
                      ctypes.c_int64, P]
        f.restype = ctypes.c_int
        _lib = lib
    return _lib


def anova_rows(F, wins, sigmas, weights, v, rows) -> np.ndarray:
    """(W v)[rows] by direct summation in C (FP64, OpenMP over rows)."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    d, N = F.shape
    win_dim = np.array([len(w) for w in wins], dtype=np.int32)
    win_feat = np.array([c for w in wins for c in w], dtype=np.int32)
    sig = np.ascontiguousarray(sigmas, dtype=np.float64)
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.shape[0])
    rc = lib.oracle_anova_rows(F.ctypes.data, N, d, len(wins), win_dim.ctypes.data,
                               win_feat.ctypes.data, sig.ctypes.data, wt.ctypes.data,
                               v.ctypes.data, rows.ctypes.data, rows.shape[0], out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_anova_rows: invalid arguments")
    return out
