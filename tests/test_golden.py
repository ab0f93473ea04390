"""The stored exact optima (tests/golden/bruteforce_n16_20.txt) against an
independent integer evaluation, and the oracle's solutions against them.

The fixture holds the minimum of x^T Q x + b^T x over {0,1}^n (Section 2,
eq. (bqp)) for each seeded instance of the brute-force set. The method is a
heuristic (its GAP is positive on some instances, Table 2), so solutions are
checked for never beating the optimum and for a quality band, not equality.
"""
import numpy as np

from golden_data import bruteforce_optima
from oracle import psdp as O
from oracle.bruteforce import brute_force
from workloads import gen


def _f(Q, b, x):
    """x^T Q x + b^T x in Python integers."""
    xs = [int(v) for v in x]
    n = len(xs)
    return sum(int(Q[i, j]) * xs[i] * xs[j] for i in range(n) for j in range(n)) + \
        sum(int(b[i]) * xs[i] for i in range(n))


def test_golden_optima_are_minima():
    gold = bruteforce_optima()
    cases = gen.bruteforce_set()
    assert sorted(gold) == [seed for seed, _, _ in cases]
    for seed, Q, b in cases:
        n, opt, x = gold[seed]
        assert n == len(b)
        assert _f(Q, b, x) == opt
        # a global minimizer is also a local one: no single flip improves it
        for i in range(n):
            y = x.copy()
            y[i] ^= 1
            assert _f(Q, b, y) >= opt
        # and the enumeration finds the same value today
        assert brute_force(Q, b)[0] == opt


def test_oracle_solutions_against_golden_optima():
    gold = bruteforce_optima()
    hits, gaps = 0, []
    for seed, Q, b in gen.bruteforce_set():
        _, opt, _ = gold[seed]
        r = O.solve(Q, b)
        assert r.obj >= opt
        hits += r.obj == opt
        gaps.append((r.obj - opt) / abs(opt) * 100.0)
    print(f"oracle: {hits}/50 optimal, mean GAP {np.mean(gaps):.3f}%", flush=True)
    assert hits >= 35 and np.mean(gaps) < 1.0
