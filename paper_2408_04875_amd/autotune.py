"""Autotuner of the exact integer product (the I8 operand path).

For every problem size n asked for, and for 4-digit products (subproblem
iterates) and 8-digit products (lambda_min / CG vectors) of a range of
live-column counts, every block layout of the int8 MFMA kernel is timed with
several K-slice counts through psdp_qx_digits_ex (HIP events around repeated
launches on the device), and the fastest setting per column count becomes an
entry of the library's table for (n, digits) (psdp_set_digit_table). Every
setting yields the same integers (exact sums in any order), so the table
changes the speed of a solve and never its results.

The tables are written as JSON (default: tuning/digits.json beside this
file, which binding.install_tuning reads) with every timing measured, so a
run can be checked against the table it produced.

    python -m paper_2408_04875_amd.autotune --n 2500 --out <file>
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import binding

COLUMNS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
SLICES = {"few": (1, 2, 4, 8), "mid": (1, 2, 4), "many": (1, 2, 4), "wide": (1, 2), "tall": (1, 2)}


def _operands(n, cols, digits, seed):
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    A = rng.integers(-127, 128, (n, n))
    Q = np.triu(A) + np.triu(A, 1).T
    if digits == 4:
        X = rng.random((cols, n))
    else:
        X = rng.standard_normal((cols, n))
    return (torch.from_numpy(Q.astype(np.int32)).cuda(), torch.from_numpy(X).cuda())


def tune(n: int, columns=COLUMNS, reps: int = 20, log=print):
    """Times every (layout, slices) per column count; returns the table
    documents of both digit counts."""
    out = []
    for digits in (4, 8):
        entries = []
        Q, Xall = _operands(n, max(columns), digits, 1000 + n + digits)
        for cols in columns:
            X = Xall[:cols].contiguous()
            ref = None
            timings = {}
            for layout, slices in SLICES.items():
                for ks in slices:
                    Y, us = binding.qx_digits(Q, X, digits=digits, layout=layout, slices=ks, reps=reps)
                    if ref is None:
                        ref = Y
                    elif not bool((Y == ref).all()):
                        raise RuntimeError(f"n={n} digits={digits} cols={cols}: {layout}/{ks} differs")
                    timings[f"{layout}/{ks}"] = us
            best = min(timings, key=timings.get)
            layout, ks = best.split("/")
            entries.append({"max_cols": cols, "layout": binding.DIGIT_LAYOUTS[layout], "slices": int(ks),
                            "us": timings[best], "timings_us": timings})
            log(f"n={n} digits={digits} columns={cols}: best {best} {timings[best]:.2f} us "
                f"(built-in rule {timings.get(_builtin(n, cols, digits), float('nan')):.2f} us)")
        out.append({"n": n, "digits": digits, "entries": entries})
    return out


def _builtin(n, cols, digits):
    """The built-in rule's setting for one product alone, as a timing key."""
    names = {v: k for k, v in binding.DIGIT_LAYOUTS.items()}
    c4, c8 = binding.digit_choice(n, cols if digits == 4 else 0, cols if digits == 8 else 0)
    mt, ks = c4 if digits == 4 else c8
    return f"{names[mt]}/{ks}"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[2500])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--columns", default=",".join(str(c) for c in COLUMNS))
    ap.add_argument("--out", default=os.path.join(binding.TUNING_DIR, "digits.json"))
    args = ap.parse_args(argv)
    import torch
    binding.load(tuning=False)
    cols = tuple(int(c) for c in args.columns.split(","))
    t0 = time.time()
    tables = []
    for n in args.n:
        for d in (4, 8):
            binding.set_digit_table(n, d, [])  # time the built-in rule without a table
        tables += tune(n, cols, args.reps, log=lambda s: print(s, flush=True))
    doc = {"device": torch.cuda.get_device_name(0), "reps": args.reps, "seconds": time.time() - t0,
           "digit_tables": [{"n": t["n"], "digits": t["digits"],
                             "entries": [{k: e[k] for k in ("max_cols", "layout", "slices", "us", "timings_us")}
                                         for e in t["entries"]]} for t in tables]}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {args.out} ({doc['seconds']:.0f} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
