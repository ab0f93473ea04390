"""Pins of oracle/fixed_point.py against facts that do not depend on it:
exact rational arithmetic on tiny inputs, closed forms, rounding rules and
the error bound of the grid."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fixed_point as F


def _frac_product(Q, xs):
    n = len(xs)
    return [sum(Fraction(int(Q[i][j])) * xs[j] for j in range(n) if j != i) for i in range(n)]


def _rint_half_even(fr: Fraction) -> int:
    fl = math.floor(fr)
    d = fr - fl
    if d > Fraction(1, 2):
        return fl + 1
    if d < Fraction(1, 2):
        return fl
    return fl if fl % 2 == 0 else fl + 1


def test_main_grid_brute_force_rationals():
    rng = np.random.default_rng(5)
    n = 7
    Q = rng.integers(-127, 128, (n, n))
    Q = np.triu(Q) + np.triu(Q, 1).T
    X = rng.random((3, n))
    X[0, 0], X[1, 1], X[2, 2] = 0.0, 1.0, 0.5
    got = F.qx_fixed_point(Q, X, 4)
    for c in range(3):
        xs = [Fraction(_rint_half_even(Fraction(float(v)) * 2**27), 2**27) for v in X[c]]
        ref = _frac_product(Q, xs)
        assert [Fraction(v) for v in got[c]] == ref


def test_main_grid_ties_to_even_and_endpoints():
    k = np.array([4, 5, 1000, 0])
    x = (2 * k + 1) / 2.0**28            # exactly halfway between k and k + 1 on the grid
    T = F.main_grid(x)
    assert list(T) == [4, 6, 1000, 0]
    assert list(F.main_grid(np.array([0.0, 1.0]))) == [0, 2**27]
    with pytest.raises(ValueError):
        F.main_grid(np.array([1.0 + 2**-52]))


def test_main_grid_closed_form_all_ones():
    n = 9
    Q = np.full((n, n), -127)
    np.fill_diagonal(Q, 10**6)          # the diagonal never enters the product
    Y = F.qx_fixed_point(Q, np.ones((1, n)), 4)
    assert (Y == -127.0 * (n - 1)).all()


def test_main_grid_error_bound():
    rng = np.random.default_rng(9)
    n = 300
    Q = rng.integers(-100, 101, (n, n))
    Q = np.triu(Q) + np.triu(Q, 1).T
    X = rng.random((4, n))
    Y = F.qx_fixed_point(Q, X, 4)
    Qo = Q.astype(np.float64)
    np.fill_diagonal(Qo, 0.0)
    exact = X @ Qo.T
    bound = np.abs(Qo).sum(axis=1) * 2.0**-28
    assert (np.abs(Y - exact) <= bound[None, :] * (1 + 1e-9) + 1e-9).all()


def test_aux_exponent_is_least_power_above():
    assert F.aux_exponent(np.array([1.0, -0.25])) == 1      # 1 < 2^1, not < 2^0
    assert F.aux_exponent(np.array([0.75])) == 0
    assert F.aux_exponent(np.array([-3.0, 2.0])) == 2
    assert F.aux_exponent(np.zeros(4)) == 0
    assert F.aux_exponent(np.array([2.0**-40 * 1.5])) == -39
    for v in np.random.default_rng(2).standard_normal(50) * 1e3:
        e = F.aux_exponent(np.array([v]))
        assert abs(v) < 2.0**e and abs(v) >= 2.0**(e - 1)


def test_aux_grid_brute_force_rationals():
    rng = np.random.default_rng(13)
    n = 6
    Q = rng.integers(-127, 128, (n, n))
    Q = np.triu(Q) + np.triu(Q, 1).T
    X = rng.standard_normal((4, n)) * np.array([[1e-3], [1.0], [1e5], [2.0**-30]])
    X[2, 3] = 0.0
    got = F.qx_fixed_point(Q, X, 8)
    for c in range(4):
        m = max(abs(Fraction(float(v))) for v in X[c])
        e = 0
        while m >= Fraction(2) ** e:
            e += 1
        while m < Fraction(2) ** (e - 1):
            e -= 1
        scale = Fraction(2) ** (55 - e)
        xs = [Fraction(_rint_half_even(Fraction(float(v)) * scale)) / scale for v in X[c]]
        ref = _frac_product(Q, xs)
        # float(Fraction) rounds to nearest, ties to even
        assert list(got[c]) == [float(r) for r in ref]


def test_aux_grid_relative_error_bound():
    rng = np.random.default_rng(21)
    n = 200
    Q = rng.integers(-127, 128, (n, n))
    Q = np.triu(Q) + np.triu(Q, 1).T
    X = rng.standard_normal((3, n)) * 10.0 ** rng.integers(-8, 8, (3, 1))
    Y = F.qx_fixed_point(Q, X, 8)
    Qo = Q.astype(np.float64)
    np.fill_diagonal(Qo, 0.0)
    for c in range(3):
        e = F.aux_exponent(X[c])
        exact = Qo @ X[c]
        quant = np.abs(Qo).sum(axis=1) * 2.0 ** (e - 56)       # grid rounding
        fp = np.abs(Qo) @ np.abs(X[c]) * n * 2.0**-52          # slack of the FP64 reference
        assert (np.abs(Y[c] - exact) <= quant + fp + np.abs(exact) * 2.0**-52).all()


def test_row_subset_matches_full():
    rng = np.random.default_rng(3)
    n = 50
    Q = rng.integers(-127, 128, (n, n))
    X = rng.random((2, n))
    rows = np.array([0, 7, 49])
    for d in (4, 8):
        assert np.array_equal(F.qx_fixed_point(Q, X, d, rows=rows), F.qx_fixed_point(Q, X, d)[:, rows])
