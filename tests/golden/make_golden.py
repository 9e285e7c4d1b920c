"""Writes the stored expected results in this folder from the CPU oracle
alone (oracle/ and the seeded input generators, nothing of the HIP path).

pin_cell_7g_1e4x30.json: the 7-group pin cell (r = 0.54 cm fuel in a 1.26 cm
reflective square; the small configuration of the benchmark set, standing in
for the paper's pin-cell problems of Sec. 4), 1e4 histories per generation,
30 generations of which 10 inactive, seed 1: per-generation k estimators,
Shannon entropy and event counts, and the active-generation flux mean and
sigma per (region, group) bin.  Floats are written with Python's shortest
round-trip repr, so reading them back gives the same doubles.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2501_05440_amd import problems as P  # noqa: E402

PIN_CELL = dict(n_per_gen=10_000, n_gen=30, n_inactive=10, seed=1, xs_seed=1000)


def pin_cell_problem():
    return P.pin_cell(**PIN_CELL)


def main():
    r = O.run(pin_cell_problem())
    out = {
        "problem": dict(name="pin_cell_7g", **PIN_CELL),
        "count_names": list(O.COUNT_NAMES),
        "gen_k": r["gen_k"].tolist(),
        "gen_entropy": r["gen_entropy"].tolist(),
        "gen_counts": r["gen_counts"].tolist(),
        "flux_mean": r["flux_mean"].tolist(),
        "flux_sigma": r["flux_sigma"].tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pin_cell_7g_1e4x30.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
