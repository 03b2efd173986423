"""ctypes wrapper of the oracle's C eigensolver (test infrastructure only).

``eigh_lowest`` returns the nev algebraically smallest eigenpairs of a
complex Hermitian matrix: the plain definition of what the paper's
eigensolver computes (low-lying excitons, full eigenpairs; Sec. "Solving
the BSE eigenvalue problem on massively parallel architectures").  The C
side follows the textbook direct method that section contrasts with
(Golub & Van Loan, 4th ed., Sec. 8.3).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_eigh_lowest.restype = ctypes.c_int
    lib.oracle_eigh_lowest.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_tridiag_qr.restype = ctypes.c_int
    lib.oracle_tridiag_qr.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def eigh_lowest(H, nev=None, vectors=True, nthreads=0):
    """Lowest ``nev`` eigenpairs of Hermitian ``H`` (only its lower triangle
    is read).  Returns (w ascending, V with unit columns, phase-normalised so
    the entry of largest modulus is real and positive) or (w, None)."""
    H = np.asarray(H)
    N = H.shape[0]
    assert H.shape == (N, N)
    nev = N if nev is None else int(nev)
    A = np.asfortranarray(H, dtype=np.complex128)
    w = np.zeros(nev, dtype=np.float64)
    V = np.zeros((N, nev), dtype=np.complex128, order="F") if vectors else None
    st = _load().oracle_eigh_lowest(
        N, A.ctypes.data, N, nev, w.ctypes.data,
        V.ctypes.data if vectors else None, int(nthreads))
    if st != 0:
        raise RuntimeError(f"oracle_eigh_lowest failed with status {st}")
    return w, V


def tridiag_eig(d, e, vectors=True):
    """Eigen-decomposition of the real symmetric tridiagonal with diagonal
    ``d`` and off-diagonal ``e``; returns (w ascending, Z columns)."""
    d = np.array(d, dtype=np.float64)
    n = d.size
    e = np.zeros(max(n, 1), dtype=np.float64) if n <= 1 else np.concatenate(
        [np.asarray(e, dtype=np.float64), [0.0]])
    Z = np.eye(n, dtype=np.float64) if vectors else None  # row-major
    st = _load().oracle_tridiag_qr(n, d.ctypes.data, e.ctypes.data,
                                   Z.ctypes.data if vectors else None, 0)
    if st != 0:
        raise RuntimeError(f"oracle_tridiag_qr failed with status {st}")
    order = np.argsort(d, kind="stable")
    return d[order], (Z[:, order] if vectors else None)
