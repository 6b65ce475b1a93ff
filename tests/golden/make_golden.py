"""Write tests/golden/exact_small.json: exact rational PageRank / PPR vectors of small
graphs, computed only with ``oracle.exact`` (Gauss-Jordan over Fractions on Eq. 2,
cross-checked against Eq. 4 of section 3.1).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402


def csr(n, edges):
    edges = sorted(edges)
    rp = [0] * (n + 1)
    for s, _ in edges:
        rp[s + 1] += 1
    for i in range(n):
        rp[i + 1] += rp[i]
    return rp, [d for _, d in edges]


CASES = [
    # name, n, edges, p (None = uniform), c
    ("two_vertices", 2, [(0, 1)], None, "17/20"),
    ("in_star_5", 6, [(k, 0) for k in range(1, 6)], None, "17/20"),
    ("self_loop_and_dangling", 4, [(0, 0), (0, 1), (1, 2), (2, 0), (2, 3)], None, "17/20"),
    ("multi_edges", 5, [(0, 1), (0, 1), (0, 2), (1, 3), (2, 3), (3, 0), (3, 4), (3, 4)], None, "17/20"),
    ("ppr_source_2", 6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (2, 0), (5, 1)], [0, 0, 1, 0, 0, 0], "17/20"),
    ("ppr_weighted_p", 5, [(0, 1), (1, 2), (2, 0), (0, 3), (3, 4)], [1, 0, 2, 0, 1], "9/10"),
    ("dag_two_layers", 7, [(0, 3), (0, 4), (1, 4), (1, 5), (2, 6), (2, 3), (3, 5), (4, 6)], None, "17/20"),
    ("low_damping", 4, [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)], None, "1/100"),
    ("high_damping", 4, [(0, 1), (1, 2), (2, 3), (1, 0)], None, "99/100"),
]


def main():
    out = {
        "source": "Exact rational solutions of Eq. 2, (I - cP')pi = (1-c)p with P' = P + p d^T, "
                  "identical to Eq. 4, pi = normalize((I - cP)^{-1} p) (section 3.1 of arXiv 2302.03245); "
                  "written by tests/golden/make_golden.py using oracle.exact only.",
        "cases": [],
    }
    for name, n, edges, p, c in CASES:
        rp, col = csr(n, edges)
        pf = None if p is None else [Fraction(v) for v in p]
        a = exact.eq2(n, rp, col, Fraction(c), pf)
        b = exact.eq4(n, rp, col, Fraction(c), pf)
        assert a == b
        out["cases"].append({
            "name": name, "n": n, "row_ptr": rp, "col": col, "c": c,
            "p": p, "pi_exact": [str(v) for v in a], "pi": [float(v) for v in a],
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
