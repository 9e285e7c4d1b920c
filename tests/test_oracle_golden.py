"""The oracle reproduces its stored results in tests/golden/ (written by
tests/golden/make_golden.py from the oracle alone) exactly: a regression
fixture for the oracle's arithmetic and its thread-count independence."""
import json
import os

import numpy as np

from paper_2501_05440_amd import problems as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "pin_cell_7g_1e4x30.json")


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_oracle_reproduces_golden_pin_cell(oracle):
    gd = load_golden()
    pr = dict(gd["problem"])
    pr.pop("name")
    prob = P.pin_cell(**pr)
    for threads in (1, 5):
        r = oracle.run(prob, n_threads=threads)
        assert list(oracle.COUNT_NAMES) == gd["count_names"]
        assert np.array_equal(r["gen_counts"], np.array(gd["gen_counts"]))
        for k in ("gen_k", "gen_entropy", "flux_mean", "flux_sigma"):
            assert np.array_equal(r[k], np.array(gd[k])), (threads, k)
