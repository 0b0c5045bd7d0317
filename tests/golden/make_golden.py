"""Writes tests/golden/tiny_exact.json: tiny integer BIL cubes with their
exact global-RX scores (Eq. 1 of the paper, Section "System Implementation /
Detection Algorithm") as rationals "num/den", computed only by the
exact-rational brute force in oracle/brute.py (Gauss-Jordan inverse).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import brute  # noqa: E402

CASES = [  # (seed, lines, samples, bands, max value, ddof, ridge num, ridge den)
    (0, 2, 8, 3, 16, 0, 0, 1),
    (1, 3, 7, 4, 4096, 0, 0, 1),
    (2, 4, 5, 5, 64, 1, 0, 1),
    (3, 2, 9, 6, 4096, 0, 1, 1000),
    (4, 1, 16, 2, 8, 0, 0, 1),
]


def main():
    out = []
    for seed, l, s, b, hi, ddof, rn, rd in CASES:
        rng = np.random.default_rng([seed, 99])
        cube = rng.integers(0, hi, size=(l, b, s))
        px = cube.transpose(0, 2, 1).reshape(l * s, b).tolist()
        sc = brute.exact_scores(px, ddof=ddof, ridge_num=rn, ridge_den=rd)
        out.append({
            "cite": "Eq. 1, Section 'System Implementation / Detection Algorithm'",
            "layout": "BIL [lines][bands][samples]",
            "lines": l, "samples": s, "bands": b, "ddof": ddof,
            "ridge_rel": [rn, rd],
            "cube": cube.tolist(),
            "scores": [f"{v.numerator}/{v.denominator}" for v in sc],
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
