"""Writes the stored expected values under tests/golden/ using only the CPU oracle.

one_loop_korobov.json: the Korobov parameter a of the one-loop sector's lattice
(n = 65521, d = 3), chosen by exhaustive minimisation of P_2 over a in [1, (n-1)/2]
(P_2(a) = P_2(n - a), so the upper half adds nothing), with candidates within a
relative 1e-12 of the minimum treated as tied and the smallest a kept.  P_2 is the
worst-case error criterion (Korobov space, alpha = 2, product weights) that the paper
names for its precomputed lattices (Sec. 2.2).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def main():
    n, d = 65521, 3
    t0 = time.time()
    cands = list(range(1, (n - 1) // 2 + 1))
    a, vals = oracle.korobov_search(n, d, cands, threads=os.cpu_count() or 1)
    out = {"n": n, "d": d, "a": a, "p2": float(vals[a - 1]),
           "p2_second_best_distinct": float(sorted(set(vals.round(15)))[1]),
           "criterion": "P_2, Korobov space alpha=2, unit product weights (paper Sec. 2.2)",
           "tie_rule": "relative 1e-12, smallest a",
           "search": "exhaustive a in [1, (n-1)/2]", "seconds": round(time.time() - t0, 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "one_loop_korobov.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
