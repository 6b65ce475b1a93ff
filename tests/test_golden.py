"""The stored exact fixtures against the FP64 oracle routines and hand-derived values (no GPU)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "exact_small.json")))


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_oracle_matches_golden(case):
    g = (case["n"], np.array(case["row_ptr"], np.int64), np.array(case["col"], np.int32))
    c = float(Fraction(case["c"]))
    p = None if case["p"] is None else np.array(case["p"], float)
    ref = np.array(case["pi"])
    assert abs(sum(Fraction(v) for v in case["pi_exact"]) - 1) == 0
    x, _, delta = oracle.power(g, c, p, tol=1e-15, max_iter=100000)
    assert np.abs(x - ref).sum() <= c / (1 - c) * delta + 1e-14
    for r in (oracle.ifp1(g, c, p, xi=1e-16), oracle.ifp2(g, c, p, xi=1e-16)):
        assert np.abs(r["pi"] - ref).sum() < 1e-12


def test_two_vertex_hand_value():
    case = next(c for c in GOLD["cases"] if c["name"] == "two_vertices")
    # 1 -> 2 with c = 17/20: pi = (1, 1 + c) / (2 + c) = (20/57, 37/57)
    assert case["pi_exact"] == ["20/57", "37/57"]


def test_in_star_hand_value():
    case = next(c for c in GOLD["cases"] if c["name"] == "in_star_5")
    # k = 5 leaves -> centre: centre (1 + ck)/(1 + k + ck), leaf 1/(1 + k + ck); c = 17/20
    ck = Fraction(17, 20) * 5
    assert Fraction(case["pi_exact"][0]) == (1 + ck) / (1 + 5 + ck)
    assert all(Fraction(v) == 1 / (1 + 5 + ck) for v in case["pi_exact"][1:])
