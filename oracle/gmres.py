"""ctypes wrapper over the C FP64 GMRES oracle (test infrastructure only).

Fields are numpy float64 arrays of shape (ny, nx) or (nz, ny, nx), row-major
with x fastest; the operator is A = -lap_h with zero Dirichlet boundary on the
unit square/cube, h = 1/(N+1) per axis (the paper's discrete Poisson problem,
Section 1.4, with the positive-definite sign).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("cycles", ctypes.c_int32), ("relres_init", ctypes.c_double),
                ("relres_first_cycle", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


@dataclass
class OracleStats:
    status: int
    iters: int
    cycles: int
    relres_init: float
    relres_first_cycle: float
    relres_est: float
    relres_true: float


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.or_apply.argtypes = [ctypes.c_int32, i64, i64, i64, dp, dp]
        L.or_apply.restype = None
        L.or_residual_norm.argtypes = [ctypes.c_int32, i64, i64, i64, dp, dp, dp, dp]
        L.or_residual_norm.restype = None
        L.or_gmres.argtypes = [ctypes.c_int32, i64, i64, i64, dp, dp, ctypes.c_int32,
                               ctypes.c_double, i64, i64, ctypes.c_int32,
                               ctypes.POINTER(_Stats), dp]
        L.or_gmres.restype = ctypes.c_int32
        L.or_arnoldi.argtypes = [ctypes.c_int32, i64, i64, i64, dp, ctypes.c_int32,
                                 ctypes.c_int32, dp, dp]
        L.or_arnoldi.restype = ctypes.c_int32
        L.or_set_threads.argtypes = [ctypes.c_int32]
        L.or_set_threads.restype = None
        L.or_set_threads(1)
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (results do not depend on it)."""
    lib().or_set_threads(int(n))


def _dims(shape):
    if len(shape) == 2:
        return 2, shape[1], shape[0], 1
    if len(shape) == 3:
        return 3, shape[2], shape[1], shape[0]
    raise ValueError("fields must be 2D or 3D")


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def apply(u: np.ndarray) -> np.ndarray:
    """A u for the zero-Dirichlet discrete Laplacian (A = -lap_h)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    dim, nx, ny, nz = _dims(u.shape)
    lib().or_apply(dim, nx, ny, nz, _ptr(u), _ptr(out))
    return out


def residual_norm(b: np.ndarray, x: np.ndarray):
    """(|b - A x|, |b|) with compensated summation."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    dim, nx, ny, nz = _dims(b.shape)
    rn, bn = ctypes.c_double(), ctypes.c_double()
    lib().or_residual_norm(dim, nx, ny, nz, _ptr(b), _ptr(x), ctypes.byref(rn), ctypes.byref(bn))
    return rn.value, bn.value


def gmres(b: np.ndarray, x0: np.ndarray | None = None, m: int = 20, rtol: float = 1e-8,
          max_iters: int = 10 ** 7, fixed_iters: int = 0, ortho: str = "cgs2",
          history: bool = False):
    """Restarted GMRES(m); returns (x, OracleStats[, hist])."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    dim, nx, ny, nz = _dims(b.shape)
    st = _Stats()
    hist = None
    if history:
        hist = np.full(max(max_iters if fixed_iters == 0 else fixed_iters, 0) + 1, np.nan)
    rc = lib().or_gmres(dim, nx, ny, nz, _ptr(b), _ptr(x), int(m), float(rtol),
                        int(max_iters), int(fixed_iters), 0 if ortho == "cgs2" else 1,
                        ctypes.byref(st), _ptr(hist) if hist is not None else None)
    if rc < 0:
        raise ValueError(f"oracle gmres rejected the arguments (rc={rc})")
    stats = OracleStats(st.status, st.iters, st.cycles, st.relres_init,
                        st.relres_first_cycle, st.relres_est, st.relres_true)
    if history:
        return x, stats, hist[: st.iters + 1]
    return x, stats


def arnoldi(r0: np.ndarray, k: int, ortho: str = "cgs2"):
    """One Arnoldi cycle of k steps: (V [(k+1), n], Hbar [(k+1), k], steps)."""
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    dim, nx, ny, nz = _dims(r0.shape)
    n = r0.size
    V = np.zeros((k + 1, n))
    H = np.zeros((k + 1, k))
    steps = lib().or_arnoldi(dim, nx, ny, nz, _ptr(r0), int(k), 0 if ortho == "cgs2" else 1,
                             _ptr(V), _ptr(H))
    return V, H, steps
