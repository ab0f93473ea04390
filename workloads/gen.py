"""Seeded synthetic UBQP workloads.

This module only draws numbers: it builds problem data (Q, b), starting
points and upstream weights with ``numpy.random.default_rng`` in a fixed
call order. It holds none of the method's arithmetic, so both the FP64
oracle and the HIP path may take their inputs from here.

The paper states the problem as min x^T Q x + b^T x over x in {0,1}^n with
Q real symmetric (Section 2, eq. (bqp)). Its benchmark sets are not
available, so each generator below stands in for one workload family with
the shapes and value ranges the paper states for it (random instances,
Section 5.2; Billionnet-Elloumi value ranges, Section 5.2; Max-Cut graphs
with +-1 weights, Section 5.3).
"""
from __future__ import annotations

import numpy as np


def _mirror_upper(U: np.ndarray) -> np.ndarray:
    """Symmetric matrix from the upper triangle (diagonal included) of U."""
    return np.triu(U) + np.triu(U, 1).T


def dense_int(n: int, seed: int, lo: int = -100, hi: int = 100):
    """Dense symmetric integer Q and integer b, entries uniform in [lo, hi].

    Small dense random instance (the paper's random instances, Table 2,
    n = 20..80; here n = 64 and the n = 16..20 brute-force set).
    """
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
    Q = _mirror_upper(A).astype(np.int32)
    b = rng.integers(lo, hi + 1, size=n, dtype=np.int64).astype(np.int32)
    return Q, b


def sparse_int(n: int, seed: int, density: float = 0.10, vmax: int = 100):
    """Symmetric integer Q at the given density, b = 0.

    Upper-triangle entries (diagonal included) are nonzero with probability
    ``density``; nonzeros are uniform over +-{1..vmax}; the lower triangle
    mirrors the upper.
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    mag = rng.integers(1, vmax + 1, size=(n, n), dtype=np.int64)
    sgn = np.where(rng.random((n, n)) < 0.5, -1, 1)
    U = np.where(mask, mag * sgn, 0)
    Q = _mirror_upper(U).astype(np.int32)
    b = np.zeros(n, dtype=np.int32)
    return Q, b


def maxcut_graph(n: int, seed: int, p_edge: float = 0.05):
    """Erdos-Renyi G(n, p_edge) with weights uniform in {-1, +1}.

    Returns the weight matrix W (symmetric, zero diagonal, int32).
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < p_edge
    sgn = np.where(rng.random((n, n)) < 0.5, -1, 1)
    U = np.triu(np.where(mask, sgn, 0), 1)
    W = (U + U.T).astype(np.int32)
    return W


def be_dense(n: int, seed: int, density: float):
    """Dense-ish instance with Billionnet-Elloumi value ranges, b = 0.

    Off-diagonal upper entries are nonzero with probability ``density`` and
    uniform integers in [-50, 50]; the diagonal is uniform in [-100, 100].
    """
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    off = rng.integers(-50, 51, size=(n, n), dtype=np.int64)
    U = np.triu(np.where(mask, off, 0), 1)
    diag = rng.integers(-100, 101, size=n, dtype=np.int64)
    Q = (U + U.T + np.diag(diag)).astype(np.int32)
    b = np.zeros(n, dtype=np.int32)
    return Q, b


# ---------------------------------------------------------------------------
# Named workloads.

def small_dense(seed: int = 0):
    """n = 64 dense integer instance (entries and b uniform in [-100, 100])."""
    return dense_int(64, seed)


def bruteforce_set():
    """Fifty dense integer instances, n = 16..20 (ten each), seeds 100..149."""
    out = []
    seed = 100
    for n in range(16, 21):
        for _ in range(10):
            Q, b = dense_int(n, seed)
            out.append((seed, Q, b))
            seed += 1
    return out


def sparse_1000(seed: int = 1):
    """n = 1000, 10% density, nonzeros +-{1..100}, b = 0."""
    return sparse_int(1000, seed)


def sparse_2500_starts(seed_q: int = 2, seed_x: int = 3, n: int = 2500, B: int = 256):
    """n = 2500 at 10% density, b = 0, plus B starts uniform in [0, 1)^n.

    Starts are returned as an array of shape (B, n): row j is start j, so the
    buffer is the column-major n x B matrix the library takes.
    """
    Q, b = sparse_int(n, seed_q)
    X0 = np.random.default_rng(seed_x).random((B, n))
    return Q, b, X0


def uneven_group(seed: int = 4, count: int = 512, nmin: int = 100, nmax: int = 3000):
    """Uneven batch: first half Max-Cut-as-UBQP, second half dense BE-range.

    Sizes n_i are uniform integers in [nmin, nmax]. Max-Cut instances use
    Q = W and b = -W e (a 0/1 encoding of the cut), dense ones have density
    uniform in [0.1, 0.8]. Returns a list of dicts with keys n, Q, b, kind,
    seed (the per-instance perturbation seed, equal to the index).
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    dens = rng.uniform(0.1, 0.8, size=count)
    sub_seeds = rng.integers(0, 2**31 - 1, size=count)
    out = []
    half = count // 2
    for i in range(count):
        n = int(ns[i])
        if i < half:
            W = maxcut_graph(n, int(sub_seeds[i]))
            Q = W
            b = (-W.astype(np.int64).sum(axis=1)).astype(np.int32)
            kind = "maxcut"
        else:
            Q, b = be_dense(n, int(sub_seeds[i]), float(dens[i]))
            kind = "dense"
        out.append(dict(n=n, Q=Q, b=b, kind=kind, seed=i))
    return out


def dense_normal_batch(seed: int = 5, n: int = 4096, B: int = 64):
    """FP32 dense Q ~ N(0,1) (symmetric), b ~ N(0,1), B points in (0,1)^n.

    Also returns p uniform in [0, 2) and upstream weights w ~ N(0,1). X has
    shape (B, n) (row j is point j).
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n), dtype=np.float32)
    Q = _mirror_upper(A).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    X = rng.uniform(1e-3, 1 - 1e-3, size=(B, n)).astype(np.float32)
    p = rng.uniform(0.0, 2.0, size=n).astype(np.float32)
    w = rng.standard_normal(B).astype(np.float32)
    return Q, b, X, p, w


def random_box_points(n: int, B: int, seed: int):
    """B points uniform in [0, 1)^n, shape (B, n)."""
    return np.random.default_rng(seed).random((B, n))


def random_vector(n: int, seed: int, scale: float = 1.0):
    """Standard normal vector of length n times scale."""
    return np.random.default_rng(seed).standard_normal(n) * scale


def real_normal(n: int, seed: int):
    """Real symmetric Q with entries N(0,1) (upper triangle mirrored) and
    b ~ N(0,1), both FP64: the real-valued form of the problem (Section 2)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    Q = _mirror_upper(A)
    b = rng.standard_normal(n)
    return Q, b
