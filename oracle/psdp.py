"""Plain FP64 CPU oracle of the vectorized PSDP method for UBQP.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
link this module: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library.

Problem (Section 2, eq. (bqp)): minimize f(x) = x^T Q x + b^T x over
x in {0,1}^n, Q real symmetric.

Everything here follows the paper's steps and notation directly, in float64
NumPy/SciPy, with no blocking or fusion: the reformulated data
Q_r = Q + Diag(gamma), b_r = b - gamma (Section 3.5, Algorithm 3) are
materialized, the penalty starts at p = 0, and the penalty function is
h(x, p) = x^T (Q_r - Diag p) x + (b_r + p)^T x (eq. (p1)/(dp1)).

Where the paper is silent or garbled, the reading used is stated at the
function that needs it; the same readings are listed in the design notes.

Pin status: every function below is pinned by tests against brute force,
closed forms or the paper's lemmas, except ``solve`` as a whole, whose
trajectory beyond those pins is "parity unpinned" (the paper prints no
worked example and its instances are unavailable).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.linalg

# Status codes reported as exit reasons (mirrored, independently, by the library).
CONVERGED = 0     # outer binary test met (Algorithm 3 loop condition)
OUTER_CAP = 1     # outer iteration cap reached
STALL = 2         # no-progress exit, or outer cap with a component pinned at 1/2

MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# Objective and penalty function.

def objective_exact(Q, b, xhat) -> int:
    """f(x) = x^T Q x + b^T x for a 0/1 vector, in exact Python integers.

    Section 2, eq. (bqp). Used on the rounded solution only.
    """
    idx = [i for i, v in enumerate(np.asarray(xhat).tolist()) if v]
    Qi = np.asarray(Q)
    tot = 0
    for i in idx:
        row = Qi[i]
        for j in idx:
            tot += int(row[j])
        tot += int(np.asarray(b)[i])
    return tot


def objective_real(Q, b, xhat) -> float:
    """f(x) = x^T Q x + b^T x for a 0/1 vector and real (float) Q, b.

    Section 2, eq. (bqp). The exact value of the sum of the selected entries
    Q_ij (x_i = x_j = 1) and b_i (x_i = 1), rounded once to FP64 (nearest,
    ties to even): math.fsum returns the correctly rounded sum of its terms,
    so the result does not depend on any summation order.
    """
    idx = [i for i, v in enumerate(np.asarray(xhat).tolist()) if v]
    Qf = np.asarray(Q, dtype=np.float64)
    bf = np.asarray(b, dtype=np.float64)
    terms = [float(Qf[i, j]) for i in idx for j in idx]
    terms += [float(bf[i]) for i in idx]
    return math.fsum(terms)


def is_integer_instance(Q, b) -> bool:
    """True when Q and b have integer dtypes (exact int objective)."""
    return np.issubdtype(np.asarray(Q).dtype, np.integer) and np.issubdtype(np.asarray(b).dtype, np.integer)


def objective(Q, b, x) -> float:
    """f(x) = x^T Q x + b^T x in float64 for any real x."""
    x = np.asarray(x, dtype=np.float64)
    return float(x @ (np.asarray(Q, dtype=np.float64) @ x) + np.asarray(b, dtype=np.float64) @ x)


def penalty(Q, b, p, x) -> float:
    """h(x, p) = f(x) + sum_i p_i (x_i - x_i^2).

    Eq. (p1) in Section 2.2 and the definition of h in Section 4.1.
    """
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return objective(Q, b, x) + float(p @ (x - x * x))


def penalty_grad(Q, b, p, x) -> np.ndarray:
    """grad_x h(x, p) = 2 (Q - Diag p) x + (b + p).

    Gradient of the Lagrangian in eq. (kkt1) without the multipliers
    (Section 3.3); Q symmetric.
    """
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    Qbar = np.asarray(Q, dtype=np.float64) - np.diag(p)
    return 2.0 * (Qbar @ x) + (np.asarray(b, dtype=np.float64) + p)


def penalty_batch(Q, b, p, X):
    """h and grad h for a batch of points; X has shape (B, n).

    Returns (h of shape (B,), G of shape (B, n)). Plain loop over points.
    """
    X = np.asarray(X, dtype=np.float64)
    h = np.array([penalty(Q, b, p, x) for x in X])
    G = np.stack([penalty_grad(Q, b, p, x) for x in X]) if len(X) else np.zeros((0, len(b)))
    return h, G


def penalty_adjoint(Q, b, p, X, w):
    """Gradients of L = sum_c w_c h(x_c, p) with respect to X, Q, b and p.

    h is linear in Q, b and p (eq. (p1)), so with the entries of Q taken as
    independent: dL/dQ = sum_c w_c x_c x_c^T, dL/db = sum_c w_c x_c,
    dL/dp = sum_c w_c (x_c - x_c^2), and dL/dx_c = w_c grad h(x_c, p).
    Returns (dX (B, n), dQ (n, n), db (n,), dp (n,)).
    """
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = X.shape[1]
    dX = np.stack([w[c] * penalty_grad(Q, b, p, X[c]) for c in range(len(X))])
    dQ = np.zeros((n, n))
    db = np.zeros(n)
    dp = np.zeros(n)
    for c in range(len(X)):
        dQ += w[c] * np.outer(X[c], X[c])
        db += w[c] * X[c]
        dp += w[c] * (X[c] - X[c] * X[c])
    return dX, dQ, db, dp


# ---------------------------------------------------------------------------
# Random perturbation (Section 3.5, "Random Perturbation").

def splitmix64(state: int) -> int:
    """One output of SplitMix64 (Steele, Lea and Flood, 2014) from ``state``.

    The generator advances its state by the golden-ratio increment and
    returns the finalized (mixed) value of the new state.
    """
    z = (state + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def perturbation(n: int, sigma: float, seed: int, mode: str = "full") -> np.ndarray:
    """Symmetric perturbation mu with mu_ij = mu_ji ~ N(0, sigma) (Section 3.5).

    The paper draws mu from a normal distribution without fixing the
    generator; this reading fixes a counter-based one so that any two
    implementations agree bit for bit:
      key = splitmix64(seed); for i <= j and t = 0..3, c = (i*n + j)*4 + t
      and u_t = splitmix64(key XOR c) >> 11 (a 53-bit integer) (the seed is
      mixed first: XOR-ing it directly with c would let seeds that differ
      only in their two low bits permute the same four draws);
      S = u_0 + u_1 + u_2 + u_3 summed exactly as integers;
      N = (double(S) * 2^-53 - 2) * sqrt(3)  (Irwin-Hall(4), unit variance);
      mu_ij = rint(N * sigma * 2^16) * 2^-16 (round half to even).
    mode "full" fills every i <= j, "diag" only i == j, "none" nothing.
    """
    mu = np.zeros((n, n))
    if mode == "none" or sigma == 0.0:
        return mu
    s3 = math.sqrt(3.0)
    key = splitmix64(seed & MASK64)
    for i in range(n):
        js = [i] if mode == "diag" else range(i, n)
        for j in js:
            S = 0
            for t in range(4):
                c = ((i * n + j) * 4 + t) & MASK64
                S += splitmix64(key ^ c) >> 11
            N = (float(S) * 2.0 ** -53 - 2.0) * s3
            v = float(np.rint((N * sigma) * 65536.0)) / 65536.0
            mu[i, j] = v
            mu[j, i] = v
    return mu


# ---------------------------------------------------------------------------
# Initialization (Section 3.5, "Reformation"; Algorithm 3 initialization).

def reformation_gamma(Q, b) -> np.ndarray:
    """gamma_i = 2 sum_j |Q_ij| + |b_i| + 1.

    The paper asks for gamma_i > sum_j 2|Q_ij| + |b_i| (Section 3.5); the
    margin 1 makes the inequality strict and keeps gamma integral for
    integer data.
    """
    Q = np.asarray(Q, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return 2.0 * np.abs(Q).sum(axis=1) + np.abs(b) + 1.0


def initial_point(Q_r, b_r) -> np.ndarray:
    """x^0 solving 2 Q_r x = -b_r, i.e. 2 (Q + Diag gamma) x = gamma - b.

    Eq. (gamma) in Section 3.5; Q_r is symmetric positive definite
    (strictly diagonally dominant with positive diagonal), so a Cholesky
    factorization solves it.
    """
    c, low = scipy.linalg.cho_factor(2.0 * np.asarray(Q_r, dtype=np.float64))
    return scipy.linalg.cho_solve((c, low), -np.asarray(b_r, dtype=np.float64))


# ---------------------------------------------------------------------------
# Subproblem machinery (Sections 3.1-3.3).

# ---------------------------------------------------------------------------
# Inner products and norms as exact values rounded once.
#
# The BB step lengths (eq. (bb1)) and the scale rho (Section 3.3) are real
# inner products and norms. The oracle computes each one as its exact value
# rounded once to FP64 (nearest, ties to even), so no summation order enters
# the trajectory.

def _two_product(a, b):
    """(p, e) with p = fl(a b) and p + e = a b exactly (Dekker's product with
    Veltkamp's splitting), elementwise. Exact when no |a|, |b| exceeds 2^995
    and no nonzero product falls below 2^-969 (callers check)."""
    c = 134217729.0  # 2^27 + 1
    ta = c * a
    ah = ta - (ta - a)
    al = a - ah
    tb = c * b
    bh = tb - (tb - b)
    bl = b - bh
    p = a * b
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dot_exact(a, b) -> float:
    """sum_i a_i b_i: the exact value rounded once to FP64.

    math.fsum returns the correctly rounded sum of its (exact) terms; each
    product enters as the exact pair of _two_product. Inputs outside that
    pair's range are summed as exact rationals instead.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = a * b
    big = max(float(np.abs(a).max(initial=0.0)), float(np.abs(b).max(initial=0.0)))
    tiny = (p != 0.0) & (np.abs(p) < 2.0 ** -960)
    lost = (p == 0.0) & (a != 0.0) & (b != 0.0)
    if big > 2.0 ** 995 or tiny.any() or lost.any():
        from fractions import Fraction
        return float(sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0)))
    p, e = _two_product(a, b)
    return math.fsum(np.concatenate([p, e]).tolist())


def row_abs_sums(M) -> np.ndarray:
    """sum_j |M_ij| for every row: exact values rounded once (math.fsum)."""
    return np.array([math.fsum(row) for row in np.abs(np.asarray(M, dtype=np.float64)).tolist()])


def rho_scale(Q_r, b_r, p) -> float:
    """rho = max{1, ||2(Q_r - Diag p)||_inf, ||b_r + p||_inf} (Section 3.3).

    The paper leaves the norms unstated; the induced infinity norm (largest
    absolute row sum) and the vector infinity norm are used, as in the
    bounds of the proof of Theorem 2. Each row sum is exact, rounded once.
    """
    Qbar = np.asarray(Q_r, dtype=np.float64) - np.diag(p)
    return max(1.0, float(row_abs_sums(2.0 * Qbar).max()),
               float(np.abs(np.asarray(b_r) + p).max()))


class _RowNorms:
    """rho and the row sums of |Q_r| for one solve, exact and rounded once.

    The off-diagonal part of Q_r - Diag p does not change with p, so its exact
    absolute row sums are kept as rationals once; each evaluation adds the
    row's one diagonal term |(Q_r)_ii - p_i| (itself rounded as the matrix
    entry is) exactly and rounds once. Same values as rho_scale and
    proximal_diagonal, without re-summing every row.
    """

    def __init__(self, Q_r):
        from fractions import Fraction
        Q_r = np.asarray(Q_r, dtype=np.float64)
        off = np.abs(Q_r)
        np.fill_diagonal(off, 0.0)
        self._F = Fraction
        self.diag = np.diag(Q_r).copy()
        self.off = []
        for row in off.tolist():
            if all(v == int(v) for v in row):
                self.off.append(Fraction(int(sum(int(v) for v in row))))
            else:
                self.off.append(sum((Fraction(v) for v in row), Fraction(0)))

    def _rows(self, d):
        F = self._F
        return np.array([float(o + F(float(abs(v)))) for o, v in zip(self.off, d)])

    def rho(self, b_r, p) -> float:
        rows = 2.0 * self._rows(self.diag - p)   # 2 |a| rounds like |a|: scaling by 2 is exact
        return max(1.0, float(rows.max()), float(np.abs(np.asarray(b_r) + p).max()))

    def hp(self, p, eps) -> np.ndarray:
        return np.maximum(self._rows(self.diag) - p, eps)


def kkt_violation(x, g) -> float:
    """cret over the index sets I = {0<x<1}, J = {x=0}, K = {x=1} (Section 3.3).

    cret = max(max_I |g_i|, max_J |min(g_j, 0)|, max_K max(g_k, 0)) with an
    empty max taken as 0; g is the full gradient of h restricted to each set
    (the paper's cret_1 omits a factor 2 on its Q_IK e_K term, read as a
    typo since eq. (kkt1) has the full gradient).
    """
    I = (x > 0.0) & (x < 1.0)
    J = x == 0.0
    K = x == 1.0
    c = 0.0
    if I.any():
        c = max(c, float(np.abs(g[I]).max()))
    if J.any():
        c = max(c, float(np.abs(np.minimum(g[J], 0.0)).max()))
    if K.any():
        c = max(c, float(np.maximum(g[K], 0.0).max()))
    return c


def box_projection(x) -> np.ndarray:
    """The operator P of Section 3.1: clip each component to [0, 1]."""
    return np.minimum(np.maximum(x, 0.0), 1.0)


@dataclasses.dataclass
class Params:
    inner: str = "pabb"        # "pabb" (Algorithm 2) or "ppa" (Algorithm 1)
    max_inner: int = 10000     # Section 5: 10000 subproblem iterations
    max_outer: int = 1000      # Section 5: 1000 penalty updates
    tol_kkt: float = 1e-5      # delta in eq. (cret)
    tol_binary: float = 1e-5   # Algorithm 3 loop condition
    eta: float = 0.999         # 0 < eta < 1 in eq. (alpha1), a "slight" scaling
    stall_outer: int = 2       # consecutive non-moving subproblems that end the loop
    eps_hp: float = 1e-8       # epsilon in H_p
    lambda_floor_rel: float = 1e-8
    alpha_min: float = 1e-30
    alpha_max: float = 1e30
    sigma: float = 0.0         # perturbation standard deviation
    perturb: str = "none"      # "none", "full" or "diag"
    seed: int = 0
    # lambda_min after a subproblem that did not move x: "shift" takes the
    # previous value minus the previous alpha (x, I and z are unchanged, so
    # eq. (alpha) shifts the scaled matrix by -alpha and its smallest
    # eigenvalue by the same amount); "solve" calls the eigensolver again
    lambda_reuse: str = "shift"
    # subproblem product: "fp64" forms (Q_r - Diag p) x in FP64 as written;
    # "i8" applies the off-diagonal part of Q_r to the iterate rounded to the
    # grid 2^-27 (the library's integer operand type, oracle.fixed_point),
    # exactly, and the diagonal part to x itself in FP64
    product: str = "fp64"


def _subproblem_gradient(Q_r, b_r, p, x, prm: Params, grid_product=None):
    """grad h(x, p) as the subproblem solvers evaluate it.

    "fp64": 2 (Q_r - Diag p) x + (b_r + p) (eq. (kkt1)). "i8": the same
    gradient with the off-diagonal product taken on the 2^-27 grid, i.e.
    2 (Q_off x_q + (diag(Q_r) - p) o x) + (b_r + p) with Q_off x_q exact
    (``grid_product``, from oracle.fixed_point).
    """
    if prm.product == "fp64" or grid_product is None:
        return penalty_grad(Q_r, b_r, p, x)
    u = grid_product(x)
    return 2.0 * (u + (np.diag(Q_r) - p) * x) + (np.asarray(b_r, dtype=np.float64) + p)


def _bb_step(k, s, y, rho, prm: Params):
    """Alternating BB step (eq. (bb1)) with the safeguards of this reading.

    k = 0 has no history: alpha = 1/rho. Odd k: BB1 = s^T s / s^T y; even
    k: BB2 = s^T y / y^T y. A non-positive curvature s^T y gives alpha_max
    (the projected spectral-gradient convention); alpha is clamped to
    [alpha_min, alpha_max].
    """
    if k == 0:
        return 1.0 / rho
    ss = dot_exact(s, s)
    sy = dot_exact(s, y)
    yy = dot_exact(y, y)
    if sy <= 0.0:
        a = prm.alpha_max
    elif k % 2 == 1:
        a = ss / sy
    else:
        a = sy / yy
    return min(max(a, prm.alpha_min), prm.alpha_max)


def solve_subproblem_pabb(Q_r, b_r, p, x, prm: Params, rho: Optional[float] = None, callback=None,
                          grid_product=None):
    """Algorithm 2 (PABB) for problem (p1) at fixed p, from x.

    Each iteration k evaluates g^k = grad h(x^k, p), stops when
    cret/rho < delta (eq. (cret)), otherwise takes
    x^{k+1} = P(x^k - alpha_k g^k) with the alternating BB step (eqs. (bb1),
    (x2)), s_{k-1} = x^k - x^{k-1}, y_{k-1} = g^k - g^{k-1}. The iteration
    counter restarts at 0 for every subproblem. A zero step s (the point did
    not move) is a KKT point of the projected iteration and also stops.
    Returns (x, iterations taken = gradient evaluations, final cret/rho,
    moved) where moved is False when the test held at the starting point.
    ``callback(k, x, g)``, if given, sees every evaluated iterate.
    """
    if rho is None:
        rho = rho_scale(Q_r, b_r, p)
    x = np.array(x, dtype=np.float64)
    x_prev = g_prev = None
    rel = math.inf
    for k in range(prm.max_inner):
        g = _subproblem_gradient(Q_r, b_r, p, x, prm, grid_product)
        rel = kkt_violation(x, g) / rho
        if callback is not None:
            callback(k, x, g)
        if rel < prm.tol_kkt:
            return x, k + 1, rel, k > 0
        if k > 0:
            s = x - x_prev
            y = g - g_prev
            if not (s != 0.0).any():
                # the previous step left x unchanged: the BB quotients are
                # undefined and the iteration cannot proceed
                return x, k + 1, rel, True
            alpha = _bb_step(k, s, y, rho, prm)
        else:
            alpha = _bb_step(0, None, None, rho, prm)
        x_prev, g_prev = x, g
        x = box_projection(x - alpha * g)
    return x, prm.max_inner, rel, True


def proximal_diagonal(Q_r, p, eps) -> np.ndarray:
    """Diagonal of H_p: max(sum_i |(Q_r)_ji| - p_j, eps) (Section 3.1).

    The row sum runs over every column, diagonal included, as the positive
    semidefiniteness argument for H_p + P requires; it is exact, rounded once.
    """
    return np.maximum(row_abs_sums(Q_r) - p, eps)


def solve_subproblem_ppa(Q_r, b_r, p, x, prm: Params, rho: Optional[float] = None, callback=None,
                         grid_product=None, hp=None):
    """Algorithm 1 (PPA) for problem (p1) at fixed p, from x.

    d~ = -grad h / (2 h_p) (eq. for d~), x^{k+1} = P(x^k + d~) (eq. (x1)),
    with the same stopping test as Algorithm 2.
    Returns (x, iterations, final cret/rho, moved).
    """
    if rho is None:
        rho = rho_scale(Q_r, b_r, p)
    if hp is None:
        hp = proximal_diagonal(Q_r, p, prm.eps_hp)
    x = np.array(x, dtype=np.float64)
    rel = math.inf
    for k in range(prm.max_inner):
        g = _subproblem_gradient(Q_r, b_r, p, x, prm, grid_product)
        rel = kkt_violation(x, g) / rho
        if callback is not None:
            callback(k, x, g)
        if rel < prm.tol_kkt:
            return x, k + 1, rel, k > 0
        x = box_projection(x + (-g / (2.0 * hp)))
    return x, prm.max_inner, rel, True


# ---------------------------------------------------------------------------
# Penalty update (Section 3.4).

def lambda_min_scaled(Q_r, p, x):
    """lambda_min(Z_II^{-1/2} Qbar_II Z_II^{-1/2}) with Qbar = Q_r - Diag p.

    Eq. (alpha) in Section 3.4; I = {i : 0 < x_i < 1}, z = x - x^2. A dense
    symmetric eigensolver computes the smallest eigenvalue.
    Returns (lambda, I as a boolean mask, z on I).
    """
    I = (x > 0.0) & (x < 1.0)
    z = x[I] - x[I] * x[I]
    Qbar = np.asarray(Q_r, dtype=np.float64)[np.ix_(I, I)] - np.diag(p[I])
    d = 1.0 / np.sqrt(z)
    M = (d[:, None] * Qbar) * d[None, :]
    lam = float(scipy.linalg.eigh(M, eigvals_only=True, subset_by_index=[0, 0])[0])
    return lam, I, z


def binary_gap(x) -> float:
    """max_i min(x_i, 1 - x_i): the distance to the nearest 0/1 vector.

    Algorithm 3's loop test ||P(x) - x||_inf > 1e-5 is vacuous with the box
    projection P of Section 3.1 (x is always in the box); it is read with P
    the projection onto {0,1}^n.
    """
    return float(np.minimum(x, 1.0 - x).max()) if len(x) else 0.0


def round_binary(x) -> np.ndarray:
    """x^_i = 1 iff x_i > 1/2 (a tie rounds to 0). Not stated in the paper."""
    return (np.asarray(x) > 0.5).astype(np.uint8)


@dataclasses.dataclass
class Result:
    x: np.ndarray            # final continuous iterate
    xhat: np.ndarray         # rounded 0/1 solution (uint8)
    obj: object              # objective of xhat on the original Q, b: int (integer data,
                             # exact) or float (real data, correctly rounded)
    exit_reason: int
    outer_iters: int
    inner_iters: int         # total gradient evaluations in subproblems
    aux_matvecs: int         # eigen/linear solves are dense here: 0
    trace: list              # per outer step: dict(s, nI, lam, alpha, inner, rel, x)
    p: np.ndarray            # final penalty vector (reformulated problem)
    eig_solves: int = 0      # lambda_min computations (eigensolver calls)


def solve(Q, b, prm: Optional[Params] = None, x0=None, p0=None) -> Result:
    """Algorithm 3 (vectorized PSDP) in float64.

    1. Optional symmetric perturbation of Q (Section 3.5), applied before the
       reformation; the final objective always uses the original Q and b.
    2. Reformation Q_r = Q + Diag(gamma), b_r = b - gamma (Algorithm 3, reformation).
    3. x^0 from eq. (gamma) (Algorithm 3, initial point) unless x0 is supplied, in
       which case x0 replaces it; p^0 = 0 unless p0 is supplied.
    4. While x is not within tol_binary of a 0/1 vector and s < max_outer:
       alpha = eta * max(lambda_min(...), floor) (eqs. (alpha), (alpha1));
       p <- p + alpha z (eq. (pp1)); then solve (p1) at the updated p from the
       current x with Algorithm 2 or 1 (reading Algorithm 3's "p = p^s" as
       the just-updated penalty: solving at p^0 from x^0 would return x^0,
       which already is that problem's stationary point).
    The floor is lambda_floor_rel * rho: the paper does not cover a
    non-positive lambda_min.
    5. No-progress exit (an addition to Algorithm 3, not a reading of it):
       when ``stall_outer`` consecutive subproblems stop at their starting
       point, the loop ends. With x unchanged, I and z are unchanged, and by
       eq. (alpha) the next scaled matrix is the previous one shifted by
       -alpha, so lambda shrinks by the factor (1 - eta) until it reaches the
       floor lambda_floor_rel * rho; from there every update adds
       eta * lambda_floor_rel * rho * z_i (1 - 2 x_i) <= 2.5e-9 rho to a
       gradient entry, at most 2.5e-6 rho over the 1000 updates of the cap,
       a quarter of the KKT tolerance. A start point whose violation lies
       within that margin of the tolerance could still move later, so the
       exit is a stated deviation; the tests pin that it changes no result
       on the seeded sets they cover (stall_outer=2 against an exit that
       never fires).
    The objective of the rounded point is exact: an integer for integer Q and
    b, else the correctly rounded FP64 value of the exact sum. The BB inner
    products and the row norms of rho and H_p are exact values rounded once
    (dot_exact, row_abs_sums), so the trajectory depends on no summation order
    except the matrix-vector products' (none in the "i8" product mode).
    ``product`` "i8" evaluates the subproblem gradients with the library's
    integer operand grid (see Params); lambda_min and x^0 stay dense FP64.
    Every trace record also holds "x", the point the update starts from.
    """
    prm = prm or Params()
    Q = np.asarray(Q)
    b = np.asarray(b)
    n = len(b)
    Qt = np.asarray(Q, dtype=np.float64) + perturbation(n, prm.sigma, prm.seed, prm.perturb)
    bt = np.asarray(b, dtype=np.float64)
    gamma = reformation_gamma(Qt, bt)
    Q_r = Qt + np.diag(gamma)
    b_r = bt - gamma
    x = initial_point(Q_r, b_r) if x0 is None else np.array(x0, dtype=np.float64)
    p = np.zeros(n) if p0 is None else np.array(p0, dtype=np.float64)
    sub = solve_subproblem_pabb if prm.inner == "pabb" else solve_subproblem_ppa
    norms = _RowNorms(Q_r)
    grid_product = None
    if prm.product == "i8":
        from oracle.fixed_point import GridProduct
        grid_product = GridProduct(Qt)
    elif prm.product != "fp64":
        raise ValueError("product must be 'fp64' or 'i8'")
    trace = []
    s = 0
    stall = 0
    inner_total = 0
    eig_solves = 0
    moved = True
    while True:
        if binary_gap(x) <= prm.tol_binary:
            reason = CONVERGED
            break
        if stall >= prm.stall_outer:
            reason = STALL
            break
        if s >= prm.max_outer:
            reason = STALL if bool((np.abs(x - 0.5) < 1e-9).any()) else OUTER_CAP
            break
        rho = norms.rho(b_r, p)
        x_start = x.copy()
        if prm.lambda_reuse == "shift" and trace and not moved:
            # warm start by the shift law: the last subproblem left x as it was
            lam = trace[-1]["lam"] - trace[-1]["alpha"]
            I = (x > 0.0) & (x < 1.0)
            z = x[I] - x[I] * x[I]
        else:
            lam, I, z = lambda_min_scaled(Q_r, p, x)
            eig_solves += 1
        alpha = prm.eta * max(lam, prm.lambda_floor_rel * rho)
        p = p.copy()
        p[I] += alpha * z
        extra = {} if prm.inner == "pabb" else {"hp": norms.hp(p, prm.eps_hp)}
        x, it, rel, moved = sub(Q_r, b_r, p, x, prm, rho=norms.rho(b_r, p), grid_product=grid_product, **extra)
        stall = 0 if moved else stall + 1
        inner_total += it
        trace.append(dict(s=s, nI=int(I.sum()), lam=lam, alpha=alpha, inner=it, rel=rel, x=x_start))
        s += 1
    xhat = round_binary(x)
    obj = objective_exact(Q, b, xhat) if is_integer_instance(Q, b) else objective_real(Q, b, xhat)
    return Result(x=x, xhat=xhat, obj=obj, exit_reason=reason,
                  outer_iters=s, inner_iters=inner_total, aux_matvecs=0, trace=trace, p=p,
                  eig_solves=eig_solves)
