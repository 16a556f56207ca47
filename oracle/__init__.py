"""CPU oracle for PLE decomposition over GF(2) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

The arithmetic lives in ``gf2_oracle.c`` (plain C, 64-bit words, no
intrinsics): plain Gaussian elimination with the first-non-zero pivot rule of
Algorithm 1, whole-row swaps recorded LAPACK-style (Section 1.2), and the
"compress L" column moves of Algorithms 1-2; RREF by back-substitution
(Section 2 definitions); the GF(2) product and the MakeTable table from their
definitions (Appendix A).  This module only marshals numpy arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (OpenMP over the rows of one pivot step)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.gf2o_ple.restype = i64
        lib.gf2o_ple.argtypes = [p, i64, i64, i64, p, p]
        lib.gf2o_ple_cols.restype = i64
        lib.gf2o_ple_cols.argtypes = [p, i64, i64, i64, p, p, i64]
        lib.gf2o_echelon_from_ple.argtypes = [p, i64, i64, i64, i64]
        lib.gf2o_rref_from_ple.argtypes = [p, i64, i64, i64, p, i64]
        lib.gf2o_addmul.argtypes = [p, i64, p, i64, p, i64, i64, i64, i64]
        lib.gf2o_make_table.argtypes = [p, i64, i64, i64, p]
        lib.gf2o_threads.restype = ctypes.c_int
        lib.gf2o_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_packed(A):
    if A.dtype != np.uint64 or A.ndim != 2 or not A.flags["C_CONTIGUOUS"]:
        raise ValueError("packed matrix must be a C-contiguous 2-D uint64 array")


def ple(A, n):
    """PLE of the packed m x n matrix A (m x ldw uint64), in place.

    Returns (r, P, Q) with P int64[m], Q int64[min(m, n)]; A holds L\\E.
    """
    _check_packed(A)
    m, ldw = A.shape
    if ldw * 64 < n:
        raise ValueError("ldw too small for n")
    P = np.empty(m, dtype=np.int64)
    Q = np.empty(min(m, n), dtype=np.int64)
    r = _load().gf2o_ple(_ptr(A), m, n, ldw, _ptr(P), _ptr(Q))
    return int(r), P, Q


def ple_cols(A, n, c_end):
    """The first c_end column steps of ple() on A, in place (then L compressed
    for the pivots found).  Returns (r, P, Q) of that partial elimination."""
    _check_packed(A)
    m, ldw = A.shape
    if ldw * 64 < n:
        raise ValueError("ldw too small for n")
    P = np.empty(m, dtype=np.int64)
    Q = np.empty(min(m, n), dtype=np.int64)
    r = _load().gf2o_ple_cols(_ptr(A), m, n, ldw, _ptr(P), _ptr(Q), int(c_end))
    return int(r), P, Q


def echelon_from_ple(A, n, r):
    _check_packed(A)
    m, ldw = A.shape
    _load().gf2o_echelon_from_ple(_ptr(A), m, n, ldw, r)


def rref_from_ple(A, n, Q, r):
    _check_packed(A)
    m, ldw = A.shape
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    _load().gf2o_rref_from_ple(_ptr(A), m, n, ldw, _ptr(Q), r)


def rref(A, n):
    """RREF of A (copy), via PLE then back-substitution. Returns (RREF, r, Q)."""
    B = np.array(A, copy=True)
    r, P, Q = ple(B, n)
    rref_from_ple(B, n, Q, r)
    return B, r, Q


def addmul(C, A, B, k, n):
    """C ^= A * B over GF(2); A is m x k packed, B is k x n packed."""
    for X in (C, A, B):
        _check_packed(X)
    m = C.shape[0]
    _load().gf2o_addmul(_ptr(C), C.shape[1], _ptr(A), A.shape[1], _ptr(B), B.shape[1], m, k, n)


def make_table(rows, k):
    """All 2^k combinations of the k packed rows; index MSB = first row."""
    _check_packed(rows)
    nw = rows.shape[1]
    T = np.empty((1 << k, nw), dtype=np.uint64)
    _load().gf2o_make_table(_ptr(rows), rows.shape[1], k, nw, _ptr(T))
    return T


def threads():
    return int(_load().gf2o_threads())


def set_threads(t):
    _load().gf2o_set_threads(int(t))
