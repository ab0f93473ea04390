"""Exact reference of the library's integer product path (test infrastructure).

The library can store Q off the diagonal as int8 and round the vector operand
of every Q.X product to a fixed-point grid; int8 matrix units then form the
product exactly (operand type I8 and the call psdp_qx_digits of the public
header). This module states that contract in plain integer arithmetic, so
that tests compare the GPU results bit for bit:

* 4-digit operand (iterates, x in [0,1]): x_q = rint(x 2^27) 2^-27 with ties
  to even; the product Q_off x_q is returned exactly (it is a multiple of
  2^-27 below 2^53 in magnitude, so FP64 holds it).
* 8-digit operand (lambda_min and CG vectors): e = the least integer with
  max|v| < 2^e (0 for a zero vector); v_q = rint(v 2^(55-e)) 2^(e-55); the
  exact product Q_off v_q is rounded once to FP64 (ties to even).

This is not the paper's arithmetic, which forms Qx in floating point; the
pins of this module bound the difference (the rounding of the grid). The
integer split used here (floor division by 2^28) is deliberately not the
digit decomposition the kernels use.

Parity unpinned: none; every function is pinned in tests/test_fixed_point_pins.py.
Only tests/, the smoke check and the benchmark's CPU leg may import this module.
"""
from __future__ import annotations

import math

import numpy as np

MAIN_BITS = 27   # iterate grid 2^-27
AUX_BITS = 55    # scaled vector grid 2^(e-55)


def q_off(Q) -> np.ndarray:
    """Q as int64 with its diagonal set to zero."""
    Qo = np.array(Q, dtype=np.int64, copy=True)
    np.fill_diagonal(Qo, 0)
    return Qo


def main_grid(X) -> np.ndarray:
    """Integers T = rint(X 2^27) (ties to even) of entries in [0,1]."""
    X = np.asarray(X, dtype=np.float64)
    if not ((X >= 0.0) & (X <= 1.0)).all():
        raise ValueError("the 4-digit operand takes entries in [0,1]")
    return np.rint(np.ldexp(X, MAIN_BITS)).astype(np.int64)


def aux_exponent(v) -> int:
    """The least integer e with max|v| < 2^e (0 for a zero vector)."""
    m = float(np.max(np.abs(v))) if np.size(v) else 0.0
    if m == 0.0:
        return 0
    _, e = math.frexp(m)  # m = f 2^e with f in [0.5, 1)
    return e


def aux_grid(v):
    """(T, e): integers T = rint(v 2^(55-e)) (ties to even) and the exponent e."""
    e = aux_exponent(v)
    return np.rint(np.ldexp(np.asarray(v, dtype=np.float64), AUX_BITS - e)).astype(np.int64), e


def qx_fixed_point(Q, X, digits: int, rows=None) -> np.ndarray:
    """Y[c, i] = (Q_off X_q[c])_i for the rows of X (shape (B, n)).

    digits 4: exact. digits 8: the exact integer product rounded once to FP64.
    rows: optional index array; only those entries i are computed (the result
    then has shape (B, len(rows))).
    """
    Qo = q_off(Q)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    if rows is not None:
        Qo = Qo[np.asarray(rows)]
    if digits == 4:
        T = main_grid(X)
        S = T @ Qo.T                       # |S| <= 127 n 2^27 < 2^53: exact in int64 and in FP64
        return S.astype(np.float64) / float(1 << MAIN_BITS)
    if digits != 8:
        raise ValueError("digits must be 4 or 8")
    out = np.empty((X.shape[0], Qo.shape[0]))
    for c in range(X.shape[0]):
        T, e = aux_grid(X[c])
        hi, lo = T >> 28, T & ((1 << 28) - 1)   # T = hi 2^28 + lo, 0 <= lo < 2^28
        s_hi = Qo @ hi                           # |.| <= 127 n 2^27: exact in int64
        s_lo = Qo @ lo
        for i in range(Qo.shape[0]):
            S = int(s_hi[i]) * (1 << 28) + int(s_lo[i])   # exact Python integer
            out[c, i] = math.ldexp(float(S), e - AUX_BITS)  # int -> float rounds to nearest even
    return out


class GridProduct:
    """The 4-digit product Q_off x_q as a callable on one vector x in [0,1].

    Same contract as qx_fixed_point(Q, x, 4), with Q_off kept once as FP64:
    every partial sum of Q_off T (|Q_ij| <= 127, |T| <= 2^27, n <= 65536) is
    an integer below 2^53, so the FP64 matrix product is exact whatever its
    summation order, and so is the scaling by 2^-27. The off-diagonal
    entries must be integers of magnitude at most 127.
    """

    def __init__(self, Q):
        Qf = np.array(Q, dtype=np.float64, copy=True)
        np.fill_diagonal(Qf, 0.0)
        if not (np.rint(Qf) == Qf).all() or np.abs(Qf).max(initial=0.0) > 127:
            raise ValueError("the integer operand type needs integer |Q_ij| <= 127 off the diagonal")
        self.Qoff = Qf

    def __call__(self, x) -> np.ndarray:
        T = main_grid(x).astype(np.float64)
        return (self.Qoff @ T) / float(1 << MAIN_BITS)
