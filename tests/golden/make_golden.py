"""Writes exact_systems.json: small integer systems with their exact rational
solutions, computed only with the oracle's exact solver (oracle/exact.py).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402


def main():
    out = {
        "source": "exact rational Gaussian elimination (Section 2.1 definition of the direct "
                  "solve, carried out without rounding); solutions are p/q strings",
        "systems": [],
    }
    g = np.random.default_rng(20080818)
    for n in (1, 2, 3, 5, 8, 12, 17):
        while True:
            A = g.integers(-9, 10, (n, n))
            b = g.integers(-9, 10, n)
            try:
                x = exact.solve(A.tolist(), b.tolist())
                break
            except ZeroDivisionError:
                continue
        out["systems"].append({"n": n, "A": A.tolist(), "b": b.tolist(),
                               "x": [f"{v.numerator}/{v.denominator}" for v in x]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_systems.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
