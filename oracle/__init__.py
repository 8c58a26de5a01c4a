"""FP64 CPU oracle for all-pairs Pearson correlation.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the HIP path.  The arithmetic lives in ``pcc_oracle.c`` (plain C,
FP64, Eq. (1) evaluated literally pair by pair); this module only marshals
numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_pearson_packed.argtypes = [_dp, _i64, _i64, _i64, _dp]
    lib.oracle_pearson_packed.restype = ctypes.c_int
    lib.oracle_pearson_xy.argtypes = [_dp, _i64, _i64, _dp, _i64, _i64, _i64, _dp]
    lib.oracle_pearson_xy.restype = ctypes.c_int
    lib.oracle_pearson_pairs.argtypes = [_dp, _i64, _i64, _i64, _lp, _lp, _i64, _dp]
    lib.oracle_pearson_pairs.restype = ctypes.c_int
    lib.oracle_transform.argtypes = [_dp, _i64, _i64, _i64, _dp, _dp, _dp]
    lib.oracle_transform.restype = ctypes.c_int
    lib.oracle_edges.argtypes = [_dp, _i64, _i64, _i64, ctypes.c_double, _i64, _lp, _lp, _dp]
    lib.oracle_edges.restype = _i64
    lib.oracle_permcounts.argtypes = [_dp, _i64, _i64, _i64, _ip, _i32, _lp, _lp, _i64, _ip, _dp,
                                      ctypes.c_double, _ip, _ip]
    lib.oracle_permcounts.restype = ctypes.c_int
    lib.oracle_enumerate_upper.argtypes = [_i64, _i32, _lp, _lp]
    lib.oracle_enumerate_upper.restype = _i64
    _lib = lib
    return lib


def _f64(X):
    X = np.ascontiguousarray(X, dtype=np.float64)   # FP32 promotes exactly
    if X.ndim != 2:
        raise ValueError("X must be 2-D (n x l)")
    return X


def _ptr(a, t):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def pearson_packed(X) -> np.ndarray:
    """All pairs i < j (strict upper triangle, row by row), FP64."""
    X = _f64(X)
    n, l = X.shape
    out = np.empty(n * (n - 1) // 2, dtype=np.float64)
    rc = _load().oracle_pearson_packed(_ptr(X, _dp), n, l, l, _ptr(out, _dp))
    if rc != 0:
        raise RuntimeError(f"oracle_pearson_packed: {rc}")
    return out


def pearson_xy(X, Y) -> np.ndarray:
    """Non-symmetric all pairs: r[i, j] = r(X_i, Y_j), an nx x ny FP64 matrix."""
    X = _f64(X)
    Y = _f64(Y)
    nx, l = X.shape
    ny, ly = Y.shape
    if ly != l:
        raise ValueError("X and Y must have the same number of samples")
    out = np.empty((nx, ny), dtype=np.float64)
    rc = _load().oracle_pearson_xy(_ptr(X, _dp), nx, l, _ptr(Y, _dp), ny, l, l, _ptr(out, _dp))
    if rc != 0:
        raise RuntimeError(f"oracle_pearson_xy: {rc}")
    return out


def pearson_pairs(X, I, J) -> np.ndarray:
    X = _f64(X)
    n, l = X.shape
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.empty(I.shape[0], dtype=np.float64)
    rc = _load().oracle_pearson_pairs(_ptr(X, _dp), n, l, l, _ptr(I, _lp), _ptr(J, _lp),
                                      I.shape[0], _ptr(out, _dp))
    if rc != 0:
        raise RuntimeError(f"oracle_pearson_pairs: {rc}")
    return out


def transform(X):
    """(U, mean, M2) of Eq. (4), FP64."""
    X = _f64(X)
    n, l = X.shape
    U = np.empty((n, l), dtype=np.float64)
    mean = np.empty(n, dtype=np.float64)
    m2 = np.empty(n, dtype=np.float64)
    rc = _load().oracle_transform(_ptr(X, _dp), n, l, l, _ptr(U, _dp), _ptr(mean, _dp),
                                  _ptr(m2, _dp))
    if rc != 0:
        raise RuntimeError(f"oracle_transform: {rc}")
    return U, mean, m2


def edges(X, thr: float, cap: int = 1 << 20):
    """Full scan: (I, J, R) of all pairs i < j with |r| >= thr, (i, j) order."""
    X = _f64(X)
    n, l = X.shape
    EI = np.empty(cap, dtype=np.int64)
    EJ = np.empty(cap, dtype=np.int64)
    ER = np.empty(cap, dtype=np.float64)
    cnt = _load().oracle_edges(_ptr(X, _dp), n, l, l, float(thr), cap, _ptr(EI, _lp),
                               _ptr(EJ, _lp), _ptr(ER, _dp))
    if cnt < 0:
        raise RuntimeError(f"oracle_edges: {cnt}")
    if cnt > cap:
        raise RuntimeError(f"oracle_edges: {cnt} edges exceed cap {cap}")
    return EI[:cnt].copy(), EJ[:cnt].copy(), ER[:cnt].copy()


def permcounts(X, perms, I, J, band=None):
    """(counts int32, gap FP64) of the permutation test on pairs (I, J).
    With band, also (c_lo, c_hi): the counts of |r_p| >= |r_obs| + band and
    of |r_p| >= |r_obs| - band, the range a computation whose every |r| is
    off by less than band/2 can produce."""
    X = _f64(X)
    n, l = X.shape
    perms = np.ascontiguousarray(perms, dtype=np.int32)
    if perms.ndim != 2 or perms.shape[1] != l:
        raise ValueError("perms must be (P, l)")
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    counts = np.empty(I.shape[0], dtype=np.int32)
    gap = np.empty(I.shape[0], dtype=np.float64)
    lo = hi = None
    if band is not None:
        lo = np.empty(I.shape[0], dtype=np.int32)
        hi = np.empty(I.shape[0], dtype=np.int32)
    rc = _load().oracle_permcounts(_ptr(X, _dp), n, l, l, _ptr(perms, _ip), perms.shape[0],
                                   _ptr(I, _lp), _ptr(J, _lp), I.shape[0], _ptr(counts, _ip),
                                   _ptr(gap, _dp), float(band or 0.0),
                                   None if lo is None else _ptr(lo, _ip),
                                   None if hi is None else _ptr(hi, _ip))
    if rc != 0:
        raise RuntimeError(f"oracle_permcounts: {rc}")
    if band is None:
        return counts, gap
    return counts, gap, lo, hi


def enumerate_upper(n: int, diag: bool):
    """(ys, xs): the cell of every job id, numbering the upper triangle
    row by row (diagonal counted in when ``diag``)."""
    lib = _load()
    cnt = lib.oracle_enumerate_upper(n, 1 if diag else 0, None, None)
    ys = np.empty(cnt, dtype=np.int64)
    xs = np.empty(cnt, dtype=np.int64)
    lib.oracle_enumerate_upper(n, 1 if diag else 0, _ptr(ys, _lp), _ptr(xs, _lp))
    return ys, xs
