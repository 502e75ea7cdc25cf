"""Smooth-rule (far) sums of the oracle in plain C with OpenMP (oracle/far.c), FP64.

TEST INFRASTRUCTURE ONLY.  The same sums as ``OracleOperator.far_rows`` (Section 6.1.3 applied
to eq:explicit_remainder with c = 0, and to the parametrix for the representation), written out
term by term in C so that whole-operator applies at 10^5 - 10^6 nodes run on every host core.
``build()`` compiles the library with gcc (-O2 -fopenmp, no fast-math); ``far_rows`` loads it.
Pinned by ``tests/test_oracle_large.py``: agreement with the NumPy rows on variable-coefficient
surfaces, and the unit-sphere closed form R = -1/(4 pi) for a = 1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "far.c")
LIB = os.path.join(HERE, "liboracle_far.so")
_lib = None


def build() -> str:
    """Compile oracle/far.c into oracle/liboracle_far.so (every call compiles)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.oracle_far_remainder.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, vp, i64, vp, vp]
        L.oracle_far_remainder.restype = None
        L.oracle_far_parametrix.argtypes = [i64, vp, vp, vp, i32, vp, i64, vp, vp]
        L.oracle_far_parametrix.restype = None
        L.oracle_far_threads.argtypes = []
        L.oracle_far_threads.restype = i32
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the sums run on (OMP_NUM_THREADS, else every host core)."""
    return int(_load().oracle_far_threads())


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def far_rows(orc, targets, sigma: np.ndarray, kernel: str = "R") -> np.ndarray:
    """sum_{j != i} w_j F(x_i, x_j) sigma_j for the targets; sigma (N, n_rhs) -> (len(targets), n_rhs).

    ``orc`` is an ``OracleOperator`` (its node arrays are used as they are).
    """
    L = _load()
    N = orc.N
    sig = _c(np.asarray(sigma, dtype=np.float64).reshape(N, -1).T)   # n_rhs rows of N
    n_rhs = sig.shape[0]
    if n_rhs > 1024:
        raise ValueError("at most 1024 right-hand sides per call")
    tg = _c(np.asarray(targets), np.int64)
    out = np.empty((len(tg), n_rhs))
    keep = [_c(orc.x), _c(orc.n), _c(orc.H), _c(orc.a), _c(orc.gs), _c(orc.w)]
    x, n, H, a, gs, w = keep
    if kernel == "R":
        L.oracle_far_remainder(N, x.ctypes.data, n.ctypes.data, H.ctypes.data, a.ctypes.data, gs.ctypes.data,
                               w.ctypes.data, n_rhs, sig.ctypes.data, len(tg), tg.ctypes.data, out.ctypes.data)
    elif kernel == "K":
        L.oracle_far_parametrix(N, x.ctypes.data, a.ctypes.data, w.ctypes.data, n_rhs, sig.ctypes.data, len(tg),
                                tg.ctypes.data, out.ctypes.data)
    else:
        raise ValueError(kernel)
    return out
