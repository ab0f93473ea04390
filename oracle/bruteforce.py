"""Loader for the exhaustive-search pin (``bruteforce.c``).

TEST INFRASTRUCTURE ONLY. Compiles the C file with gcc on first use (or
through ``build_bruteforce``) and calls it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bruteforce.c")
_LIB = os.path.join(_HERE, "_bruteforce.so")
_handle = None


def build_bruteforce() -> str:
    """Compile the enumeration library (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_bruteforce()
        h = ctypes.CDLL(_LIB)
        h.ubqp_bruteforce.restype = ctypes.c_int
        h.ubqp_bruteforce.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]
        _handle = h
    return _handle


def brute_force(Q, b):
    """Exact minimum of x^T Q x + b^T x over {0,1}^n (n <= 30), integer data.

    Returns (obj, x as uint8 array); ties go to the smallest binary value.
    """
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    n = len(b)
    obj = ctypes.c_int64()
    mask = ctypes.c_uint64()
    rc = _lib().ubqp_bruteforce(n, Q.ctypes.data, b.ctypes.data, ctypes.byref(obj), ctypes.byref(mask))
    if rc != 0:
        raise ValueError("brute force supports 1 <= n <= 30")
    x = np.array([(mask.value >> i) & 1 for i in range(n)], dtype=np.uint8)
    return int(obj.value), x
