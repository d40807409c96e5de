"""ctypes loader for the oracle's plain-C inner loops (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_c.c")
_SO = os.path.join(_HERE, "_oracle_c.so")
_lib = None


def build(force=True):
    """Compile oracle_c.c with the system C compiler."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int)
        L.orc_rinv.restype = ctypes.c_int
        L.orc_rinv.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64,
                               ctypes.c_uint64, u64p]
        L.orc_reduce.restype = ctypes.c_int
        L.orc_reduce.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_int, i32p, ctypes.c_int, i32p,
                                 ctypes.c_int, i32p, i32p,
                                 u64p, ctypes.c_int, i32p,
                                 ctypes.c_int, i32p, i32p, ctypes.c_int,
                                 u64p, u64p, u64p]
        _lib = L
    return _lib


def u64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def ptr_u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def ptr_i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def right_inverse(A, q, p):
    """Right inverse of A (rows x cols, entries mod q) via orc_rinv.

    Returns (X, rank): X is cols x rows with A X = I mod q when rank == rows."""
    A = u64(np.asarray(A, dtype=object) % q) if A.dtype == object else u64(A % np.uint64(q))
    rows, cols = A.shape
    out = np.zeros((cols, rows), dtype=np.uint64)
    rank = lib().orc_rinv(rows, cols, ptr_u64(A), q, p, ptr_u64(out))
    return out, rank
