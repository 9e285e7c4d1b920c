"""GPU: full per-flight event logs against the oracle's on tiny runs.

Every flight of every history (position after it, length, energy, cell,
region, group or energy bin, and how it ended) must agree: integers exactly,
floating point to 1e-12 relative."""
import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def compare_events(g, o):
    assert g.shape == o.shape
    for f in ("cell", "region", "group", "type"):
        d = g[f] != o[f]
        assert not d.any(), f"{f}: {d.sum()} differ, first {np.argwhere(d)[:3].tolist()}"
    for f in ("x", "y", "d", "e"):
        a, b = g[f], o[f]
        bad = np.abs(a - b) > 1e-12 * np.maximum(np.abs(a), np.abs(b))
        assert not bad.any(), f"{f}: {bad.sum()} differ, first {np.argwhere(bad)[:3].tolist()}"


@pytest.mark.parametrize("case,flights", [("pin", 0), ("pin", 1), ("lattice", 0), ("ce", 0),
                                          ("ce", 1)])
def test_event_logs_match_oracle(oracle, case, flights):
    banner(f"event logs {case} flights={flights}")
    if case == "pin":
        prob, cap = P.pin_cell(n_per_gen=63, n_gen=3, n_inactive=1), 256
    elif case == "lattice":
        prob, cap = P.lattice_17x17(n_per_gen=64, n_gen=3, n_inactive=1), 512
    else:
        prob, cap = P.ce_pin_cell(n_per_gen=64, n_gen=3, n_inactive=1), 1024
    g = mcx.run(prob, record=True, event_log=cap, flights=flights, tail_threshold=-1)
    o = oracle.run(prob, records=True, events=cap)
    assert np.array_equal(g["gen_counts"], o["gen_counts"])
    compare_events(g["events"], o["events"])
    # the tail kernel logs the same flights
    t = mcx.run(prob, record=True, event_log=cap, tail_threshold=1 << 30)
    compare_events(t["events"], o["events"])
