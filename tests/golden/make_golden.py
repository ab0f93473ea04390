"""Writes the stored expected values under tests/golden/.

bruteforce_n16_20.txt: the exact minimum and minimizer of every instance of
the seeded brute-force set, by exhaustive enumeration over {0,1}^n.
oracle_replay.jsonl: whole oracle solves at the configurations' full sizes,
one JSON record per solve with its per-update trace (lambda_min, alpha, |I|,
subproblem length), exit, objective and rounded point; the GPU tests replay
each record's alpha sequence and compare every update with it.

Every oracle solve here runs with one BLAS thread: at n >= 1000 the
trajectory depends on the summation order of the library's matrix-vector
products (the same solve gives different objectives with 1, 2 and 8
threads), so the fixtures record one reproducible order.

Run from the repository root:

    python tests/golden/make_golden.py            # every fixture
    python tests/golden/make_golden.py replay     # oracle_replay.jsonl only

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





def replay_cases():
    """(name, Q, b, Params, x0 or None, store_x0) of every replayed solve:
    the single instance n = 1000 (subproblem cap 1000) from x^0 of eq.
    (gamma), in both product modes, with x^0 stored in the record (the
    last bits of a LAPACK Cholesky depend on the host's BLAS kernels); 16 of
    the 256 starts of the n = 2500 batched workload in both product modes;
    16 instances of the uneven batch (8 Max-Cut graphs, 8 dense) from seeded
    random starts in both product modes, each with the diagonal perturbation
    of sigma = 1e-3 max|Q_ij| of that instance and seed = its index. Every
    update computes lambda_min with the eigensolver (lambda_reuse "solve")."""
    import numpy as np
    from oracle import psdp as O
    out = []
    Q, b = gen.sparse_1000()
    gam = O.reformation_gamma(Q, b)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        x0 = O.initial_point(Q + np.diag(gam), b - gam)
    for mode in ("fp64", "i8"):
        out.append((f"n1000_x0_{mode}", Q, b, O.Params(max_inner=1000, product=mode, lambda_reuse="solve"), x0,
                    True))
    Q, b, X0 = gen.sparse_2500_starts()
    for mode in ("fp64", "i8"):
        for c in range(16):
            out.append((f"n2500_start{c}_{mode}", Q, b, O.Params(product=mode, lambda_reuse="solve"), X0[c],
                        False))
    group = gen.uneven_group()
    for mode in ("fp64", "i8"):
        for k in list(range(8)) + list(range(256, 264)):
            d = group[k]
            sigma = 1e-3 * float(abs(d["Q"]).max())
            x0 = gen.random_box_points(d["n"], 1, 1000 + k)[0]
            out.append((f"group{k}_{d['kind']}_{mode}", d["Q"], d["b"],
                        O.Params(perturb="diag", sigma=sigma, seed=d["seed"], product=mode, lambda_reuse="solve"),
                        x0, False))
    return out


def _replay_one(case):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import psdp as O
    name, Q, b, prm, x0, store_x0 = case
    with threadpool_limits(1):
        r = O.solve(Q, b, prm, x0=x0)
    rec = dict(name=name, n=len(b), product=prm.product, sigma=prm.sigma, perturb=prm.perturb,
               seed=prm.seed, max_inner=prm.max_inner, obj=r.obj, outer=r.outer_iters, exit=r.exit_reason,
               inner_total=r.inner_iters, alpha=[t["alpha"] for t in r.trace], lam=[t["lam"] for t in r.trace],
               nI=[t["nI"] for t in r.trace], inner=[t["inner"] for t in r.trace],
               xhat=np.packbits(r.xhat).tobytes().hex())
    if store_x0:
        rec["x0"] = np.asarray(x0, dtype="<f8").tobytes().hex()
    return rec


def make_replay(workers=8):
    import json
    import multiprocessing as mp
    cases = replay_cases()
    with mp.Pool(workers) as pool:
        # longest first: the n = 2500 and large group solves
        order = sorted(range(len(cases)), key=lambda i: -len(cases[i][2]))
        done = pool.map(_replay_one, [cases[i] for i in order], chunksize=1)
        recs = [None] * len(cases)
        for i, r in zip(order, done):
            recs[i] = r
    with open(os.path.join(HERE, "oracle_replay.jsonl"), "w") as f:
        f.write(json.dumps({"comment": "Whole oracle solves (Algorithm 3, PABB, FP64, one BLAS thread, exact "
                            "inner products and norms) with their per-update traces; x0 (where present) is the "
                            "start as little-endian FP64 bytes in hex; written by tests/golden/make_golden.py"})
                + "\n")
        for r in recs:
            f.write(json.dumps(r) + "\n")


def main():
    lines = [HEADER.rstrip("\n")]
    for seed, Q, b in gen.bruteforce_set():
        opt, x = brute_force(Q, b)
        lines.append(f"{seed} {len(b)} {opt} {''.join(str(int(v)) for v in x)}")
    with open(os.path.join(HERE, "bruteforce_n16_20.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1:] == ["replay"]:
        make_replay()
    else:
        main()
        make_replay()
