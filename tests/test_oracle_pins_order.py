"""Pins of the oracle's outer loop, its perturbation scale, its real-valued
objective and its integer-operand product mode.

Each test checks the oracle against a fact that does not come from the
oracle itself: an independent eigensolver (generalized symmetric, not the
oracle's scaled standard one), the KKT test at a penalty rebuilt from the
trace, exact rational arithmetic, and the integer contract of
oracle.fixed_point. Where a test guards against a specific mistake, a second
test plants that mistake in a copy of the oracle's loop (on the CPU) and
shows the check rejects it.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import fixed_point as FP
from oracle import psdp as O
from workloads import gen


# --- Algorithm 3: order of lambda_min, the penalty update and the subproblem --

def _rebuild_and_check(Q, b, r, prm):
    """Checks a solve's trace against Algorithm 3 (Section 3.4, eqs. (alpha),
    (alpha1), (pp1)) with the reading that the subproblem runs at the
    just-updated penalty.

    The penalty before update s is rebuilt from the trace alone:
    p_0 = 0 and p_{s+1} = p_s + alpha_s z_s on I_s, z_s = x_s - x_s^2 at the
    update's start point x_s. Then, for every update:
      (a) lambda_s is the smallest eigenvalue of the pencil
          ((Q_r - Diag p_s)_II, Diag(z_II)), from scipy's generalized
          symmetric eigensolver (the oracle scales and calls the standard
          one), i.e. it is taken BEFORE the update;
      (b) alpha_s = eta max(lambda_s, floor rho(p_s));
      (c) the point the subproblem returned (the next update's start, or the
          final iterate) meets the stop test of eq. (cret) at p_{s+1}, i.e.
          the subproblem ran AFTER the update.
    Returns the number of updates whose subproblem was checked by (c).
    """
    n = len(b)
    Qt = np.asarray(Q, dtype=np.float64)
    gam = O.reformation_gamma(Qt, np.asarray(b, dtype=np.float64))
    Q_r = Qt + np.diag(gam)
    b_r = np.asarray(b, dtype=np.float64) - gam
    p = np.zeros(n)
    checked = 0
    for s, t in enumerate(r.trace):
        x = t["x"]
        I = (x > 0) & (x < 1)
        assert int(I.sum()) == t["nI"]
        z = x[I] - x[I] * x[I]
        A = Q_r[np.ix_(I, I)] - np.diag(p[I])
        lam_gen = scipy.linalg.eigh(A, np.diag(z), eigvals_only=True)[0]
        scale = np.abs(A).sum(axis=1).max() / z.min()
        assert abs(t["lam"] - lam_gen) <= 1e-9 * scale, (s, t["lam"], lam_gen)
        rho = O.rho_scale(Q_r, b_r, p)
        assert t["alpha"] == prm.eta * max(t["lam"], prm.lambda_floor_rel * rho)
        p = p.copy()
        p[I] += t["alpha"] * z
        x_next = r.trace[s + 1]["x"] if s + 1 < len(r.trace) else r.x
        if t["rel"] < prm.tol_kkt and t["inner"] < prm.max_inner:
            g = O.penalty_grad(Q_r, b_r, p, x_next)
            assert O.kkt_violation(x_next, g) / O.rho_scale(Q_r, b_r, p) < prm.tol_kkt, s
            checked += 1
    assert np.allclose(p, r.p, rtol=0, atol=0)
    return checked


@pytest.mark.parametrize("case", ["n64", "n40", "n30x0"])
def test_update_order_lambda_before_and_subproblem_after(case):
    if case == "n64":
        Q, b = gen.small_dense(0)
        r = O.solve(Q, b)
    elif case == "n40":
        Q, b = gen.dense_int(40, 8)
        r = O.solve(Q, b)
    else:
        Q, b = gen.dense_int(30, 9)
        r = O.solve(Q, b, x0=gen.random_box_points(30, 1, 4)[0])
    assert len(r.trace) >= 3
    assert _rebuild_and_check(Q, b, r, O.Params()) >= 2


def _planted_solve(Q, b, mistake):
    """Algorithm 3 with one planted ordering mistake (test only):
    "lambda_after": lambda taken at the updated penalty p + alpha z;
    "solve_before": the subproblem run at the penalty before the update."""
    prm = O.Params()
    n = len(b)
    Qt = np.asarray(Q, dtype=np.float64)
    bt = np.asarray(b, dtype=np.float64)
    gam = O.reformation_gamma(Qt, bt)
    Q_r, b_r = Qt + np.diag(gam), bt - gam
    x = O.initial_point(Q_r, b_r)
    p = np.zeros(n)
    trace = []
    for s in range(30):
        if O.binary_gap(x) <= prm.tol_binary:
            break
        rho = O.rho_scale(Q_r, b_r, p)
        x_start = x.copy()
        lam, I, z = O.lambda_min_scaled(Q_r, p, x)
        alpha = prm.eta * max(lam, prm.lambda_floor_rel * rho)
        p_new = p.copy()
        p_new[I] += alpha * z
        if mistake == "lambda_after":
            lam = O.lambda_min_scaled(Q_r, p_new, x)[0]
        p_sub = p if mistake == "solve_before" else p_new
        x, it, rel, _ = O.solve_subproblem_pabb(Q_r, b_r, p_sub, x, prm)
        p = p_new
        trace.append(dict(s=s, nI=int(I.sum()), lam=lam, alpha=alpha, inner=it, rel=rel, x=x_start))
    return O.Result(x=x, xhat=O.round_binary(x), obj=0, exit_reason=0, outer_iters=len(trace),
                    inner_iters=0, aux_matvecs=0, trace=trace, p=p)


@pytest.mark.parametrize("mistake", ["lambda_after", "solve_before"])
def test_update_order_check_rejects_planted_mistakes(mistake):
    Q, b = gen.small_dense(0)
    r = _planted_solve(Q, b, mistake)
    with pytest.raises(AssertionError):
        _rebuild_and_check(Q, b, r, O.Params())


# --- the no-progress exit (an addition to Algorithm 3) ----------------------

def _stall_cases():
    cases = [(f"bf{seed}", Q, b, None) for seed, Q, b in gen.bruteforce_set()[::5]]
    Q, b = gen.small_dense(0)
    cases.append(("n64", Q, b, None))
    Q, b = gen.dense_int(64, 3)
    for c, x in enumerate(gen.random_box_points(64, 3, 11)):
        cases.append((f"n64x{c}", Q, b, x))
    Q, b, X0 = gen.sparse_2500_starts(n=200, B=3)
    for c in range(3):
        cases.append((f"n200x{c}", Q, b, X0[c]))
    return cases


@pytest.mark.parametrize("name,Q,b,x0", _stall_cases(), ids=[c[0] for c in _stall_cases()])
def test_no_progress_exit_changes_no_result(name, Q, b, x0):
    """The no-progress exit against a loop that never takes it (stall_outer
    beyond the outer cap, so the loop runs to Algorithm 3's own exits): the
    same rounded point and objective. Once lambda sits at its floor, a later
    update can still move the continuous iterate a little (an update adds at
    most 2.5e-9 rho to a gradient entry); on these sets it moves by at most
    1e-4, never across 1/2."""
    a = O.solve(Q, b, O.Params(stall_outer=2), x0=x0)
    c = O.solve(Q, b, O.Params(stall_outer=10**9), x0=x0)
    assert a.obj == c.obj
    assert np.array_equal(a.xhat, c.xhat)
    if a.exit_reason == O.STALL:
        assert c.outer_iters >= a.outer_iters
        assert np.abs(a.x - c.x).max() <= 1e-4


# --- perturbation scale (Section 3.5) ----------------------------------------

@pytest.mark.parametrize("sigma", [0.37, 3.0])
def test_perturbation_sigma_is_a_standard_deviation(sigma):
    """mu(sigma) is sigma times the unit draw up to the 2^-16 grid, so its
    variance scales as sigma^2 (a variance reading would give sigma)."""
    n = 80
    unit = O.perturbation(n, 1.0, 77, "full")
    mu = O.perturbation(n, sigma, 77, "full")
    assert np.abs(mu - sigma * unit).max() <= (1.0 + sigma) * 2.0 ** -17 + 1e-15
    iu = np.triu_indices(n)
    v = mu[iu]
    assert abs(v.var() / sigma ** 2 - 1.0) < 0.1
    assert abs(v.mean()) < 0.1 * sigma
    assert np.abs(v).max() <= 2 * math.sqrt(3) * sigma + 2.0 ** -16


# --- the real-valued objective (Section 2, eq. (bqp)) -------------------------

def _exact_round(Q, b, x):
    """The exact rational value of f(x) on 0/1 x, converted once to float
    (Fraction -> float rounds to nearest, ties to even)."""
    idx = np.flatnonzero(x)
    tot = Fraction(0)
    for i in idx:
        tot += Fraction(float(b[i]))
        for j in idx:
            tot += Fraction(float(Q[i, j]))
    return float(tot)


def test_real_objective_is_the_correctly_rounded_sum():
    rng = np.random.default_rng(31)
    for trial in range(40):
        n = int(rng.integers(2, 24))
        A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-60, 60, size=(n, n)))
        Q = np.triu(A) + np.triu(A, 1).T
        b = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, size=n))
        if trial % 4 == 0:  # catastrophic cancellation: pairs that cancel exactly plus a tiny residue
            Q[0, 1] = Q[1, 0] = 1e300
            Q[0, 0], Q[1, 1] = -1e300, -1e300
            b[0] = 3e-300
        x = rng.integers(0, 2, size=n).astype(np.uint8)
        x[:2] = 1
        assert O.objective_real(Q, b, x) == _exact_round(Q, b, x)
    # integer-valued float data: the same value as the exact integer objective
    Qi, bi = gen.dense_int(20, 5)
    x = (np.arange(20) % 3 == 0).astype(np.uint8)
    assert O.objective_real(Qi.astype(np.float64), bi.astype(np.float64), x) == O.objective_exact(Qi, bi, x)


def test_real_valued_solve_against_enumeration():
    """Real Q ~ N(0,1): the oracle's solve never beats the exact minimum
    found by enumeration (in exact rationals), and reaches it on most of the
    set (quality band; Table 2 reports GAPs near 0.1% at this size)."""
    hits = 0
    for seed in range(12):
        n = 10
        Q, b = gen.real_normal(n, 600 + seed)
        r = O.solve(Q, b)
        assert isinstance(r.obj, float)
        best = None
        for bits in range(1 << n):
            x = np.array([(bits >> k) & 1 for k in range(n)], dtype=np.uint8)
            v = _exact_round(Q, b, x)
            best = v if best is None or v < best else best
        assert r.obj >= best
        assert r.obj == _exact_round(Q, b, r.xhat)
        hits += int(r.obj == best)
    assert hits >= 8


# --- the integer operand product mode ----------------------------------------

def test_grid_product_equals_the_integer_contract():
    Q, _ = gen.dense_int(70, 12, lo=-127, hi=127)
    gp = FP.GridProduct(Q)
    rng = np.random.default_rng(3)
    for t in range(6):
        x = rng.random(70)
        x[rng.random(70) < 0.2] = 0.0
        x[rng.random(70) < 0.2] = 1.0
        assert np.array_equal(gp(x), FP.qx_fixed_point(Q, x[None, :], 4)[0])
    with pytest.raises(ValueError):
        FP.GridProduct(Q + 0.5)
    Q2 = Q.copy()
    Q2[0, 1] = Q2[1, 0] = 128
    with pytest.raises(ValueError):
        FP.GridProduct(Q2)


def test_i8_gradient_matches_fp64_on_the_grid_and_within_the_grid_bound_off_it():
    """On a point of the 2^-27 grid the two product modes give the same
    gradient up to FP64 rounding; off the grid they differ by at most
    2 * 2^-28 * sum_j |Q_ij| per entry (the grid error of the product)."""
    Q, b = gen.dense_int(50, 21)
    gam = O.reformation_gamma(Q, b)
    Q_r, b_r = Q + np.diag(gam), b - gam
    p = np.random.default_rng(1).uniform(0, 100, 50)
    gp = FP.GridProduct(Q_r)
    prm = O.Params(product="i8")
    rng = np.random.default_rng(2)
    row = np.abs(Q_r).sum(axis=1)
    for t in range(5):
        x = np.rint(rng.random(50) * 2 ** 27) / 2 ** 27
        g8 = O._subproblem_gradient(Q_r, b_r, p, x, prm, gp)
        g64 = O.penalty_grad(Q_r, b_r, p, x)
        assert np.abs(g8 - g64).max() <= 1e-12 * row.max()
        y = rng.random(50)
        d = np.abs(O._subproblem_gradient(Q_r, b_r, p, y, prm, gp) - O.penalty_grad(Q_r, b_r, p, y))
        assert (d <= 2 * 2.0 ** -28 * np.abs(Q).sum(axis=1) + 1e-12 * row.max()).all()


# --- exact inner products and norms (eq. (bb1), Section 3.3) ----------------

def _exact_dot(a, b):
    return float(sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0)))


def test_dot_exact_is_the_correctly_rounded_inner_product():
    rng = np.random.default_rng(8)
    for trial in range(60):
        n = int(rng.integers(1, 400))
        a = rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, size=n))
        b = rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, size=n))
        if trial % 3 == 0:   # cancellation: b = a almost everywhere with the sign of a pair flipped
            b = a.copy()
            b[::2] *= -1
            b[0] += 1e-9
        if trial % 5 == 0:   # tiny products handled through exact rationals
            a[0] = 1e-300
            b[0] = 3e-20
        assert O.dot_exact(a, b) == _exact_dot(a, b), trial
    assert O.dot_exact(np.zeros(0), np.zeros(0)) == 0.0


def test_row_sums_and_rho_are_exact_row_norms():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((30, 30)) * np.exp2(rng.integers(-30, 30, size=(30, 30)))
    exact = [float(sum((Fraction(abs(float(v))) for v in row), Fraction(0))) for row in M]
    assert O.row_abs_sums(M).tolist() == exact
    # the per-solve cache gives the same rho and H_p diagonal as the plain functions
    Q, b = gen.dense_int(40, 3)
    Qt = Q + O.perturbation(40, 0.7, 5, "diag")
    gam = O.reformation_gamma(Qt, b)
    Q_r, b_r = Qt + np.diag(gam), b - gam
    norms = O._RowNorms(Q_r)
    for t in range(4):
        p = rng.uniform(0, 2 * gam.max(), 40)
        assert norms.rho(b_r, p) == O.rho_scale(Q_r, b_r, p)
        assert np.array_equal(norms.hp(p, 1e-8), O.proximal_diagonal(Q_r, p, 1e-8))
