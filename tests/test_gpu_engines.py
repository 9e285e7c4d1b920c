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
