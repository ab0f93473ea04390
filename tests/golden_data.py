"""Reader of the stored expected values under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def bruteforce_optima():
    """{seed: (n, optimum, minimizer as uint8 array)} from bruteforce_n16_20.txt."""
    out = {}
    with open(os.path.join(GOLDEN, "bruteforce_n16_20.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, n, opt, bits = line.split()
            x = np.array([int(c) for c in bits], dtype=np.uint8)
            assert len(x) == int(n)
            out[int(seed)] = (int(n), int(opt), x)
    return out
