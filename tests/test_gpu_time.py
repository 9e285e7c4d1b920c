"""GPU parity of the time-dependent fixed-source mode against the CPU oracle.

A source pulse at t = 0, fission counted as capture, a flux tally split into
time bins and a census at the last time edge (MC/DC's time-dependent mode,
Sec. 1).  The kernels repeat the oracle's operations in the same order, so
every history agrees: integer record fields and counters exactly, floating
point (final time and position, track lengths, the time-binned flux) to
1e-12 relative."""
import math

import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu

RTOL = 1e-12
FATE_CENSUS = 5
INT_FIELDS = ["n_seg", "n_col", "n_cross", "n_refl", "fate", "n_sites", "g_final", "ctr_final"]
FP_FIELDS = ["tl_sum", "kcol_sum", "x_final", "y_final", "t_final"]


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def assert_close(a, b, rtol=RTOL, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    assert a.shape == b.shape, what
    bad = np.abs(a - b) > rtol * np.maximum(np.abs(a), np.abs(b))
    assert not bad.any(), f"{what}: {bad.sum()} differ, first at {np.argwhere(bad)[:3].tolist()}"


def flux_quantum(prob):
    """The GPU sums each flux contribution as an integer multiple of a fixed
    quantum, 2^(e - 61) with 2^e the power of two just above 1.01 * 36.8 /
    min(sigma_t) (the longest flight a 53-bit uniform can draw); the oracle
    sums in compensated floating point.  A time bin can hold a few tiny
    pieces of flights cut at a bin edge, so the two may differ by up to half
    a quantum per contribution there, beyond the relative bound."""
    _, e = math.frexp(1.01 * 36.8 / float(np.min(prob["xs"]["sig_t"])))
    return math.ldexp(1.0, e - 61)


def compare(g, o, prob):
    assert np.array_equal(g["gen_counts"], o["gen_counts"]), (g["gen_counts"], o["gen_counts"])
    for gen in range(g["records"].shape[0]):
        for f in INT_FIELDS:
            d = g["records"][gen][f] != o["records"][gen][f]
            assert not d.any(), f"gen {gen} {f}: {d.sum()} differ, first {np.argwhere(d)[:3]}"
        for f in FP_FIELDS:
            assert_close(g["records"][gen][f], o["records"][gen][f], what=f"gen {gen} {f}")
    n = prob["run"]["n_per_gen"]
    q = flux_quantum(prob)
    seg = g["gen_counts"][:, 0].astype(float)
    # at most one contribution per flight lands in a given bin
    atol = (seg * q / 2 / n)[:, None]
    for gen in range(len(seg)):
        a, b = g["gen_flux"][gen], o["gen_flux"][gen]
        bad = np.abs(a - b) > RTOL * np.maximum(np.abs(a), np.abs(b)) + atol[gen]
        assert not bad.any(), f"gen_flux {gen}: {bad.sum()} differ, first {np.argwhere(bad)[:3]}"
    bad = np.abs(g["flux_mean"] - o["flux_mean"]) > (
        RTOL * np.maximum(np.abs(g["flux_mean"]), np.abs(o["flux_mean"])) + atol.max())
    assert not bad.any(), f"flux_mean: {bad.sum()} differ"


def test_pulsed_lattice_records_and_time_bins(oracle):
    """The pulsed 17x17 lattice, 3000 histories x 3 batches: every history,
    the time-binned flux per batch and its mean."""
    banner("pulsed lattice 3000 x 3 records parity")
    prob = P.pulsed_lattice(n_per_gen=3000, n_gen=3)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare(g, o, prob)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = g["gen_counts"].T
    assert np.all(ab + leak + cen == n) and np.all(sites == 0) and np.all(cen > 0)
    t_max = prob["time"]["t_edges"][-1]
    rec = g["records"]
    assert np.all(rec["t_final"][rec["fate"] == FATE_CENSUS] == t_max)
    assert np.all(rec["t_final"][rec["fate"] != FATE_CENSUS] < t_max)


def test_pulsed_lattice_event_logs(oracle):
    banner("pulsed lattice event logs")
    prob = P.pulsed_lattice(n_per_gen=64, n_gen=2)
    cap = 2048
    for flights, tail in ((0, -1), (1, -1), (8, 1 << 30)):
        g = mcx.run(prob, record=True, event_log=cap, flights=flights, tail_threshold=tail)
        o = oracle.run(prob, records=True, events=cap)
        assert np.array_equal(g["gen_counts"], o["gen_counts"])
        ge, oe = g["events"], o["events"]
        for f in ("cell", "region", "group", "type"):
            assert np.array_equal(ge[f], oe[f]), (flights, tail, f)
        for f in ("x", "y", "d"):
            assert_close(ge[f], oe[f], what=f"{f} flights={flights} tail={tail}")


@pytest.mark.parametrize("flights,tail,block", [(1, -1, 64), (8, 0, 256), (3, 1 << 30, 512)])
def test_time_launch_configuration_does_not_change_results(flights, tail, block):
    banner(f"time mode determinism flights={flights} tail={tail} block={block}")
    prob = P.pulsed_lattice(n_per_gen=20000, n_gen=2)
    ref = mcx.run(prob, record=True)
    got = mcx.run(prob, record=True, flights=flights, tail_threshold=tail, block_size=block)
    for k in ("gen_counts", "flux_mean", "flux_sigma"):
        assert np.array_equal(ref[k], got[k]), k
    assert np.array_equal(ref["records"], got["records"])


def test_one_group_infinite_medium_closed_form(oracle):
    """One group, infinite medium: the flux in time bin [a, b] per source
    particle is (exp(-sa v a) - exp(-sa v b)) / sa and the census fraction
    exp(-sa v T); the GPU equals the oracle and both match these."""
    banner("one-group time bins vs closed form")
    xs = P.one_group(1.0, 0.3, 0.1)
    v = 1.0e5
    edges = np.array([0.0, 1e-6, 3e-6, 1e-5, 3e-5])
    n, batches = 50000, 8
    prob = P.with_time(P.homogeneous(xs, n, batches, 0, seed=31, fixed_source=True), edges,
                       speed=[v])
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare(g, o, prob)
    fl = g["flux_mean"].reshape(-1, 1, 4).sum(0)[0]
    sg = np.sqrt((g["flux_sigma"].reshape(-1, 1, 4) ** 2).sum(0))[0]
    sa = 0.7
    want = (np.exp(-sa * v * edges[:-1]) - np.exp(-sa * v * edges[1:])) / sa
    assert np.all(np.abs(fl - want) < 4 * sg + 1e-12), (fl, want, sg)
    cen = g["gen_counts"][:, 10].sum() / (n * batches)
    p = math.exp(-sa * v * edges[-1])
    assert abs(cen - p) < 4 * math.sqrt(p * (1 - p) / (n * batches))


def test_full_size_pulsed_lattice_first_batch(oracle):
    """The pulsed lattice at full size (1e6 histories per batch): the first
    batch history by history, balance in every batch."""
    banner("pulsed lattice 1e6 x 2 records")
    prob = P.pulsed_lattice(n_per_gen=1_000_000, n_gen=2)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = g["gen_counts"].T
    assert np.all(ab + leak + cen == n) and np.all(killed == 0)
    assert np.all(seg == col + cross + cen)  # a flight ends in one of three ways
    o = oracle.run(P.with_run(prob, n_gen=1), records=True, per_gen_tallies=True)
    assert np.array_equal(g["gen_counts"][0], o["gen_counts"][0])
    for f in INT_FIELDS:
        assert np.array_equal(g["records"][0][f], o["records"][0][f]), f
    for f in FP_FIELDS:
        assert_close(g["records"][0][f], o["records"][0][f], what=f)
    q = flux_quantum(prob)
    a, b = g["gen_flux"][0], o["gen_flux"][0]
    atol = g["gen_counts"][0, 0] * q / 2 / n
    assert not np.any(np.abs(a - b) > RTOL * np.maximum(np.abs(a), np.abs(b)) + atol)


def test_time_mode_refusals():
    banner("time mode refusals")
    prob = P.pulsed_lattice(n_per_gen=100, n_gen=1)
    with pytest.raises(mcx.MCXError) as e:
        mcx.Context(prob, engine="persistent")
    assert e.value.code == mcx.EINVAL
    eig = P.with_run(P.with_time(P.lattice_17x17(n_per_gen=100, n_gen=2, n_inactive=1),
                                 prob["time"]["t_edges"]), fixed_source=False)
    with pytest.raises(mcx.MCXError) as e:
        mcx.Context(eig)
    assert e.value.code == mcx.EINVAL


def test_fp32_mixed_time_mode_is_balanced_and_close_to_fp64():
    """FP32-mixed in the time-dependent mode: independent of the launch
    configuration, balanced, and its census and leakage fractions within
    statistics of FP64 on the same streams."""
    banner("pulsed lattice FP32-mixed vs FP64")
    prob = P.pulsed_lattice(n_per_gen=50000, n_gen=4)
    a = mcx.run(prob, precision="fp32", record=True)
    b = mcx.run(prob, precision="fp32", record=True, flights=1, tail_threshold=-1, block_size=64)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["flux_mean"], b["flux_mean"])
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = a["gen_counts"].T
    assert np.all(ab + leak + cen == n) and np.all(killed == 0) and np.all(sites == 0)
    g = mcx.run(prob)
    tot = n * prob["run"]["n_gen"]
    for idx in (4, 10):  # leaked, census
        p32 = a["gen_counts"][:, idx].sum() / tot
        p64 = g["gen_counts"][:, idx].sum() / tot
        assert abs(p32 - p64) < 5 * math.sqrt(p64 * (1 - p64) / tot) + 1e-12, (idx, p32, p64)
    t32 = a["records"]["t_final"]
    assert np.all(t32[a["records"]["fate"] == FATE_CENSUS] == prob["time"]["t_edges"][-1])


# ---------------------------------------------------------------------------
# continuous energy (the paper's time-dependent pin cell, Sec. 4): 14 MeV
# source pulse, speed from the energy, flux and neutron density per time bin
# ---------------------------------------------------------------------------

def ce_quanta(prob):
    """Fixed-point quanta of the GPU's flux and density sums: 2^(e - 61),
    2^e the power of two above 1.01 * 36.8 / min Sigma_t (the longest
    flight) and above 1.01 * the census time (the longest time in one bin)."""
    ce = prob["ce"]
    st_min = math.inf
    for m in range(len(ce["mat_n"])):
        st = sum(ce["mat_dens"][m][k] * ce["sig_t"][ce["mat_nuc"][m][k]]
                 for k in range(ce["mat_n"][m]))
        st_min = min(st_min, float(np.min(st)))
    _, e1 = math.frexp(1.01 * 36.8 / st_min)
    _, e2 = math.frexp(1.01 * prob["time"]["t_edges"][-1])
    return math.ldexp(1.0, e1 - 61), math.ldexp(1.0, e2 - 61)


def compare_ce_time(g, o, prob):
    assert np.array_equal(g["gen_counts"], o["gen_counts"]), (g["gen_counts"], o["gen_counts"])
    for gen in range(g["records"].shape[0]):
        for f in INT_FIELDS:
            d = g["records"][gen][f] != o["records"][gen][f]
            assert not d.any(), f"gen {gen} {f}: {d.sum()} differ, first {np.argwhere(d)[:3]}"
        for f in FP_FIELDS + ["e_final"]:
            assert_close(g["records"][gen][f], o["records"][gen][f], what=f"gen {gen} {f}")
    n = prob["run"]["n_per_gen"]
    qf, qd = ce_quanta(prob)
    seg = g["gen_counts"][:, 0].astype(float)[:, None]
    for key, q in (("gen_flux", qf), ("gen_prod", qd)):
        a, b = g[key], o[key]
        bad = np.abs(a - b) > RTOL * np.maximum(np.abs(a), np.abs(b)) + seg * q / 2 / n
        assert not bad.any(), f"{key}: {bad.sum()} bins differ"
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")


@pytest.mark.parametrize("engine", ["event", "monolithic"])
def test_ce_pulsed_pin_cell_parity(oracle, engine):
    banner(f"CE pulsed pin cell 3000 x 2 vs oracle ({engine} engine)")
    prob = P.ce_pulsed_pin_cell(n_per_gen=3000, n_gen=2)
    g = mcx.run(prob, record=True, per_gen_tallies=True, engine=engine)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare_ce_time(g, o, prob)
    n = prob["run"]["n_per_gen"]
    c = g["gen_counts"]
    assert np.all(c[:, 5] + c[:, 9] + c[:, 10] + c[:, 4] == n)


def test_ce_pulsed_launch_configurations_agree():
    banner("CE pulsed pin cell: tail, flights and block size give identical results")
    prob = P.ce_pulsed_pin_cell(n_per_gen=20_000, n_gen=2)
    a = mcx.run(prob, record=True)
    b = mcx.run(prob, record=True, flights=1, tail_threshold=-1, block_size=128)
    c = mcx.run(prob, record=True, tail_threshold=1 << 30)
    for r in (b, c):
        for k in ("gen_counts", "flux_mean", "prod_mean", "gen_k"):
            assert np.array_equal(a[k], r[k]), k
        assert np.array_equal(a["records"], r["records"])


def test_ce_pulsed_heavy_target_closed_form():
    """A flat medium of one very heavy nuclide keeps the 1 MeV speed through
    every scatter: flux and density per time bin follow the one-group decay
    exp(-Sigma_a v t) (4 sigma), census fraction binomial."""
    banner("CE heavy-target decay vs closed form")
    e0 = 1.0e6
    sig_s, sig_c, sig_f = 3.0, 0.4, 0.1
    ce = dict(P.ce_flat(sig_s, sig_c, sig_f, 1e12), src_energy=e0)
    edges = np.array([0.0, 2e-10, 5e-10, 1e-9, 2e-9, 4e-9])
    prob = P.with_time(P.ce_homogeneous(ce, 100_000, 10, 0, seed=41, fixed_source=True), edges)
    g = mcx.run(prob)
    nt = len(edges) - 1
    sa = sig_c + sig_f
    v = 2.99792458e10 * math.sqrt(2.0 * e0 / 939.56542052e6)
    decay = np.exp(-sa * v * edges[:-1]) - np.exp(-sa * v * edges[1:])
    flux = g["flux_mean"].reshape(-1, nt).sum(0)
    fsig = np.sqrt((g["flux_sigma"].reshape(-1, nt) ** 2).sum(0))
    dens = g["prod_mean"].reshape(-1, nt).sum(0)
    dsig = np.sqrt((g["prod_sigma"].reshape(-1, nt) ** 2).sum(0))
    assert np.all(np.abs(flux - decay / sa) < 4 * fsig), (flux, decay / sa, fsig)
    assert np.all(np.abs(dens - decay / (sa * v)) < 4 * dsig), (dens, decay / (sa * v), dsig)
    n = 100_000 * 10
    cen = g["gen_counts"][:, 10].sum() / n
    p = math.exp(-sa * v * edges[-1])
    assert abs(cen - p) < 4 * math.sqrt(p * (1 - p) / n)


def test_ce_pulsed_full_size_first_batch(oracle):
    """The benchmark's continuous-energy pulsed pin cell at full size
    (1e6 histories): the first batch history by history."""
    banner("CE pulsed pin cell 1e6 x 1 records parity")
    prob = P.ce_pulsed_pin_cell(n_gen=1)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare_ce_time(g, o, prob)


def test_ce_pulsed_fp32_mixed_is_deterministic_and_close_to_fp64():
    banner("CE pulsed pin cell FP32-mixed vs FP64")
    prob = P.ce_pulsed_pin_cell(n_per_gen=50_000, n_gen=4)
    a = mcx.run(prob, precision="fp32", record=True)
    b = mcx.run(prob, precision="fp32", record=True, flights=1, tail_threshold=-1, block_size=64)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["prod_mean"], b["prod_mean"])
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = a["gen_counts"].T
    assert np.all(ab + cut + cen == n) and np.all(killed == 0) and np.all(sites == 0)
    g = mcx.run(prob)
    # the density summed over every bin is the mean time alive: per batch
    # differences between the precisions stay within their spread
    nt = len(prob["time"]["t_edges"]) - 1
    d32 = a["prod_mean"].reshape(-1, nt).sum(0)
    d64 = g["prod_mean"].reshape(-1, nt).sum(0)
    s = np.hypot(a["prod_sigma"].reshape(-1, nt), g["prod_sigma"].reshape(-1, nt))
    s = np.sqrt((s ** 2).sum(0))
    ok = d64 > 1e-3 * d64.max()
    assert np.all(np.abs(d32 - d64)[ok] < 5 * s[ok] + 1e-300), (d32, d64, s)
