"""GPU: the monolithic engine (the paper's event scheme, Sec. 2: one
launch runs one whole segment of every live particle, from a
to-be-processed bank into a processed bank, with no sorting).

Every engine runs the same operations of every history in the same order,
so the monolithic engine must reproduce the oracle history by history (FP64
parity bar) and the decomposed event engine bit for bit."""
import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P
from test_gpu_parity import compare_runs, flux_atol

pytestmark = pytest.mark.gpu

KEYS = ("gen_k", "gen_counts", "gen_entropy", "k_mean", "k_sigma", "flux_mean", "flux_sigma",
        "prod_mean", "prod_sigma")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def same(a, b, keys=KEYS):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


def test_monolithic_pin_cell_matches_oracle(oracle):
    banner("monolithic engine: pin cell 1e4 x 30 vs oracle")
    prob = P.pin_cell()
    g = mcx.run(prob, engine="monolithic", record=True)
    o = oracle.run(prob, records=True)
    compare_runs(g, o, atol_flux=flux_atol(g, prob))


def test_monolithic_lattice_matches_event_engine(oracle):
    banner("monolithic engine: lattice 5e4 x 6 vs event engine and oracle")
    prob = P.lattice_17x17(n_per_gen=50_000, n_gen=6, n_inactive=2)
    m = mcx.run(prob, engine="monolithic", record=True)
    e = mcx.run(prob, record=True)
    same(m, e)
    assert np.array_equal(m["records"], e["records"])
    o = oracle.run(P.with_run(prob, n_gen=2, n_inactive=1), records=True)
    for gen in range(2):
        for f in ("n_seg", "n_col", "n_cross", "fate", "n_sites", "ctr_final"):
            assert np.array_equal(m["records"][gen][f], o["records"][gen][f]), (gen, f)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_monolithic_continuous_energy_matches_event_engine(prec):
    banner(f"monolithic engine: CE pin cell 4000 x 3 ({prec})")
    prob = P.ce_pin_cell(n_per_gen=4000, n_gen=3, n_inactive=1)
    m = mcx.run(prob, engine="monolithic", record=True, precision=prec)
    e = mcx.run(prob, record=True, precision=prec)
    same(m, e)
    assert np.array_equal(m["records"], e["records"])


def test_monolithic_continuous_energy_matches_oracle(oracle):
    banner("monolithic engine: CE pin cell 3000 x 3 vs oracle")
    prob = P.ce_pin_cell(n_per_gen=3000, n_gen=3, n_inactive=1)
    g = mcx.run(prob, engine="monolithic", record=True)
    o = oracle.run(prob, records=True)
    assert np.array_equal(g["gen_counts"], o["gen_counts"])
    for gen in range(3):
        for f in ("n_seg", "n_col", "n_cross", "fate", "n_sites", "ctr_final"):
            assert np.array_equal(g["records"][gen][f], o["records"][gen][f]), (gen, f)
    np.testing.assert_allclose(g["gen_k"], o["gen_k"], rtol=1e-12)


def test_monolithic_time_dependent_and_fp32_match_event_engine():
    banner("monolithic engine: pulsed lattice and FP32-mixed lattice")
    prob = P.pulsed_lattice(n_per_gen=20_000, n_gen=2)
    same(mcx.run(prob, engine="monolithic"), mcx.run(prob))
    prob = P.lattice_17x17(n_per_gen=20_000, n_gen=3, n_inactive=1)
    same(mcx.run(prob, engine="monolithic", precision="fp32"), mcx.run(prob, precision="fp32"))


def test_monolithic_guard_and_block_size():
    banner("monolithic engine: event guard and block sizes")
    prob = P.with_run(P.lattice_17x17(n_per_gen=5000, n_gen=2, n_inactive=1), max_events=7)
    a = mcx.Context(prob, engine="monolithic", record=True)
    try:
        assert a.run(check=False) == mcx.EGUARD
        ra = a.records(0)
    finally:
        a.close()
    b = mcx.Context(prob, record=True)
    try:
        assert b.run(check=False) == mcx.EGUARD
        assert np.array_equal(ra, b.records(0))
    finally:
        b.close()
    prob = P.lattice_17x17(n_per_gen=30_000, n_gen=3, n_inactive=1)
    same(mcx.run(prob, engine="monolithic", block_size=64),
         mcx.run(prob, engine="monolithic", block_size=1024))


# ---------------------------------------------------------------------------
# asynchronous engine: global per-event-type queues, no grid-wide barrier
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_async_lattice_matches_event_engine(prec):
    banner(f"async engine: lattice 1e5 x 4 ({prec}) vs event engine")
    prob = P.lattice_17x17(n_per_gen=100_000, n_gen=4, n_inactive=1)
    a = mcx.run(prob, engine="async", precision=prec)
    e = mcx.run(prob, precision=prec)
    same(a, e)


def test_async_pin_cell_matches_oracle(oracle):
    banner("async engine: pin cell 1e4 x 30 vs oracle")
    prob = P.pin_cell()
    g = mcx.run(prob, engine="async")
    o = oracle.run(prob)
    compare_runs(g, o, records=False, atol_flux=flux_atol(g, prob))


@pytest.mark.parametrize("grid,flights", [(1, 1), (7, 8), (2048, 3)])
def test_async_launch_shapes_give_identical_results(grid, flights):
    """One workgroup (every event of every history through one block's
    queue traffic), a few, and more workgroups than fit at once; one or
    several flights per advance item."""
    banner(f"async engine: grid {grid}, flights {flights}")
    prob = P.lattice_17x17(n_per_gen=20_000, n_gen=3, n_inactive=1)
    a = mcx.run(prob, engine="async", persistent={"grid": grid}, flights=flights)
    e = mcx.run(prob)
    same(a, e)


def test_async_fixed_source_and_guard():
    banner("async engine: fixed-source pin cell and the event guard")
    prob = P.with_run(P.pin_cell(n_per_gen=30_000, n_gen=3, n_inactive=0), fixed_source=True)
    same(mcx.run(prob, engine="async"), mcx.run(prob))
    prob = P.with_run(P.lattice_17x17(n_per_gen=5000, n_gen=2, n_inactive=1), max_events=7)
    a = mcx.run(prob, engine="async")
    e = mcx.run(prob)
    assert a["rc"] == mcx.EGUARD and e["rc"] == mcx.EGUARD
    same(a, e)


def test_async_batch_matches_persistent_batch():
    banner("async engine: 64-problem batch vs the persistent engine")
    probs = P.batch_pin_cells(n_problems=64, n_max=40_000)
    res = {}
    for eng in ("persistent", "async"):
        b = mcx.Batch(probs, engine=eng)
        try:
            b.run()
            k, cnt = b.results()
            tal = [b.tallies_of(p) for p in (0, 17, 63)]
        finally:
            b.close()
        res[eng] = (k, cnt, tal)
    assert np.array_equal(res["persistent"][0], res["async"][0])
    assert np.array_equal(res["persistent"][1], res["async"][1])
    for a, b in zip(res["persistent"][2], res["async"][2]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_async_refuses_what_it_does_not_run():
    banner("async engine: refusals")
    for prob, kw in ((P.ce_pin_cell(n_per_gen=100, n_gen=2, n_inactive=1), {}),
                     (P.pulsed_lattice(n_per_gen=100, n_gen=1), {}),
                     (P.pin_cell(n_per_gen=100, n_gen=2, n_inactive=1), {"record": True})):
        with pytest.raises(mcx.MCXError) as e:
            mcx.Context(prob, engine="async", **kw)
        assert e.value.code == mcx.EINVAL
