"""Writes the stored expected values under tests/golden/.

bruteforce_n16_20.txt: the exact minimum and minimizer of every instance of
the seeded brute-force set, by exhaustive enumeration over {0,1}^n. Run from
the repository root:

    python tests/golden/make_golden.py

Uses only the oracle's enumeration and the seeded instance generators.
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


def main():
    lines = [HEADER.rstrip("\n")]
    for seed, Q, b in gen.bruteforce_set():
        opt, x = brute_force(Q, b)
        lines.append(f"{seed} {len(b)} {opt} {''.join(str(int(v)) for v in x)}")
    with open(os.path.join(HERE, "bruteforce_n16_20.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
