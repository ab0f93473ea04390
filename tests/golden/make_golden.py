"""Writes the stored expected values under tests/golden/.

bruteforce_n16_20.txt: the exact minimum and minimizer of every instance of
the seeded brute-force set, by exhaustive enumeration over {0,1}^n.
oracle_n1000_single.txt: the oracle's solve of the n = 1000 single instance
(its objective and iteration counts). Run from the repository root:

    python tests/golden/make_golden.py

Uses only the oracle and the seeded instance generators.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.bruteforce import brute_force  # noqa: E402
from workloads import gen  # noqa: E402

HEADER = """\
# Exact minima of f(x) = x^T Q x + b^T x over {0,1}^n (Section 2, eq. (bqp)),
# by exhaustive enumeration, for the seeded dense integer instances of the
# brute-force set (n = 16..20, seeds 100..149). Table 2 reports GAP against
# exact optima of instances of this size (n = 20..80).
# Written by tests/golden/make_golden.py.
# columns: seed n optimum minimizer (x_0 .. x_{n-1} as 0/1 characters)
"""


HEADER_N1000 = """\
# The oracle's solve (Algorithm 3 with PABB, FP64) of the single instance of
# n = 1000 at 10% density (nonzeros +-{1..100}, b = 0, workloads seed 1) from
# x^0 of eq. (gamma), with the subproblem cap at 1000 iterations.
# Written by tests/golden/make_golden.py.
# columns: objective outer_iterations inner_iterations exit_reason
"""


def main():
    from oracle import psdp as O
    Q, b = gen.sparse_1000()
    r = O.solve(Q, b, O.Params(max_inner=1000))
    with open(os.path.join(HERE, "oracle_n1000_single.txt"), "w") as f:
        f.write(HEADER_N1000 + f"{r.obj} {r.outer_iters} {r.inner_iters} {r.exit_reason}\n")
    lines = [HEADER.rstrip("\n")]
    for seed, Q, b in gen.bruteforce_set():
        opt, x = brute_force(Q, b)
        lines.append(f"{seed} {len(b)} {opt} {''.join(str(int(v)) for v in x)}")
    with open(os.path.join(HERE, "bruteforce_n16_20.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
