"""The FP64 oracle against stored exact-rational scores (tests/golden/
tiny_exact.json, written by tests/golden/make_golden.py from oracle/brute.py;
Eq. 1 of the paper, Section "System Implementation / Detection Algorithm")."""
import json
import os
from fractions import Fraction

import numpy as np

from oracle import rx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")


def load_golden():
    with open(GOLDEN) as f:
        cases = json.load(f)
    for c in cases:
        c["cube"] = np.array(c["cube"], dtype=np.uint16)
        c["scores"] = np.array([float(Fraction(s)) for s in c["scores"]])
    return cases


def test_oracle_matches_exact_rational_fixture():
    for c in load_golden():
        px = rx.pixels(c["cube"])
        mu, cov = rx.stats(px, c["ddof"])
        rn, rd = c["ridge_rel"]
        got = rx.scores(px, mu, rx.regularise(cov, rn / rd))
        assert np.max(np.abs(got - c["scores"]) / np.maximum(c["scores"], 1e-300)) <= 1e-12
