"""GPU parity: the HIP event-based path against the CPU oracle.

FP64 mode is defined operation by operation (single IEEE operations plus
correctly rounded ln and cos/sin(2 pi xi)), so the two implementations must
produce the same histories: every integer of every per-history record equal,
every floating-point record field equal to 1e-12 relative (in practice bit
for bit), and generation estimators and tallies equal to 1e-12 relative
(they differ only by summation order: exact fixed-point sums on the GPU,
compensated sums on the CPU).
"""
import math

import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu

RTOL = 1e-12
INT_FIELDS = ["n_seg", "n_col", "n_cross", "n_refl", "fate", "n_sites", "g_final", "ctr_final"]
FP_FIELDS = ["tl_sum", "kcol_sum", "x_final", "y_final"]


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def assert_close(a, b, rtol=RTOL, what="", atol=0.0):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    assert a.shape == b.shape, what
    scale = np.maximum(np.abs(a), np.abs(b))
    bad = np.abs(a - b) > rtol * scale + atol
    assert not bad.any(), f"{what}: {bad.sum()} differ, first at {np.argwhere(bad)[:3].tolist()}"


def flux_quantum(prob):
    """The GPU sums each flux term as an integer multiple of 2^(e - 61), 2^e
    the power of two just above 1.01 * 36.8 / min(sigma_t) (the longest flight
    a 53-bit uniform can draw); the oracle sums in compensated floating point.
    A sparsely hit bin can hold only a few short flights, so the two may
    differ there by up to half a quantum per term beyond the relative bound."""
    _, e = math.frexp(1.01 * 36.8 / float(np.min(prob["xs"]["sig_t"])))
    return math.ldexp(1.0, e - 61)


def flux_atol(g, prob):
    """Half a quantum per flight of the busiest generation, per source particle."""
    return float(g["gen_counts"][:, 0].max()) * flux_quantum(prob) / 2 / prob["run"]["n_per_gen"]


def compare_records(g_rec, o_rec, what):
    assert g_rec.shape == o_rec.shape
    for f in INT_FIELDS:
        d = g_rec[f] != o_rec[f]
        assert not d.any(), f"{what}: {f} differs for {d.sum()} histories, first {np.argwhere(d)[:3].tolist()}"
    for f in FP_FIELDS:
        assert_close(g_rec[f], o_rec[f], what=f"{what}: {f}")


def compare_runs(g, o, records=True, tallies=True, atol_flux=0.0, atol_prod=0.0):
    assert np.array_equal(g["gen_counts"], o["gen_counts"]), (g["gen_counts"], o["gen_counts"])
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")
    assert_close(g["gen_entropy"], o["gen_entropy"], what="entropy")
    assert_close(g["k_mean"], o["k_mean"], what="k_mean")
    if records:
        for gen in range(g["records"].shape[0]):
            compare_records(g["records"][gen], o["records"][gen], f"gen {gen}")
    if tallies:
        assert_close(g["flux_mean"], o["flux_mean"], what="flux_mean", atol=atol_flux)
        assert_close(g["prod_mean"], o["prod_mean"], what="prod_mean", atol=atol_prod)
        # sigma is a difference of nearly equal numbers; compare to the mean's scale
        for k in ("flux", "prod"):
            ds = np.abs(g[f"{k}_sigma"] - o[f"{k}_sigma"])
            assert np.all(ds <= 1e-9 * np.maximum(np.abs(o[f"{k}_mean"]), 1e-300) +
                          1e-9 * o[f"{k}_sigma"]), k


@pytest.fixture(scope="module")
def ctx_c0():
    prob = P.pin_cell(n_per_gen=1000, n_gen=2, n_inactive=1)
    c = mcx.Context(prob)
    yield c
    c.close()


def test_device_math_is_correctly_rounded(oracle, ctx_c0):
    banner("device ln / cos,sin(2 pi t) / sqrt vs oracle")
    rng = np.random.default_rng(41)
    words = rng.integers(0, 2**63, 1 << 20, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    xi = ((words >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    got = ctx_c0.diag_math(0, xi)
    assert np.array_equal(got, mcx.host_math(0, xi))
    sample = np.arange(0, len(xi), 97)
    assert np.array_equal(got[sample], [oracle.cr_log(v) for v in xi[sample]])
    cs = ctx_c0.diag_math(1, xi)
    assert np.array_equal(cs, mcx.host_math(1, xi))
    assert np.array_equal(cs[sample], [oracle.cr_cossin_2pi(v) for v in xi[sample]])
    y = rng.uniform(0, 4, 1 << 18)
    assert np.array_equal(ctx_c0.diag_math(2, y), np.sqrt(y))
    u = ctx_c0.diag_math(3, words.view(np.float64))
    assert np.array_equal(u, xi)


def test_device_philox_matches_oracle(oracle, ctx_c0):
    banner("device philox vs oracle")
    rng = np.random.default_rng(43)
    a = rng.integers(0, 2**63, (4096, 6), dtype=np.int64).astype(np.uint64)
    a[0] = 0
    got = ctx_c0.diag_philox(a)
    for i in range(0, 4096, 37):
        want = oracle.philox(a[i, :4].tolist(), a[i, 4:].tolist())
        assert [int(v) for v in got[i]] == want


@pytest.mark.parametrize("flights", [1, 0])
def test_pin_cell_full_parity(oracle, flights):
    """The 7-group pin cell (1e4 histories x 30 generations, 10 inactive),
    one flight per advance launch and the default."""
    banner(f"pin cell 1e4 x 30 records parity flights={flights}")
    prob = P.pin_cell()
    g = mcx.run(prob, record=True, bank=True, flights=flights)
    o = oracle.run(prob, records=True, bank_cap=3 * prob["run"]["n_per_gen"])
    compare_runs(g, o)
    assert np.array_equal(g["bank"], o["bank"])
    assert_close(g["k_sigma"], o["k_sigma"], rtol=1e-9, what="k_sigma")


def test_lattice_parity_spans_tiles_and_ragged_tail(oracle):
    """17x17 lattice, 12345 histories (not a multiple of the block), 5 gens."""
    banner("lattice 12345 x 5 records parity")
    prob = P.lattice_17x17(n_per_gen=12345, n_gen=5, n_inactive=2)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare_runs(g, o)
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux")
    assert_close(g["gen_prod"], o["gen_prod"], what="gen_prod")


def large_lattice(n=96, n_per_gen=3000, n_gen=3, n_inactive=1):
    """An n x n lattice of the 17x17 lattice's pins: its pin map alone (n^2
    words) is past the event kernels' 32 KB LDS budget for table copies."""
    fuels = [P.mg_material(np.random.default_rng(1001 + f), fissile=True) for f in range(3)]
    mod = P.mg_material(np.random.default_rng(1004), fissile=False)
    pin_map = np.random.default_rng(2002).integers(0, 3, size=(n, n))
    univ = [([P.PIN_RADIUS], [f, 3]) for f in range(3)]
    geo = P.lattice_geometry(n, n, P.PIN_PITCH, univ, pin_map, [P.VACUUM] * 4)
    return P.make_problem(f"lattice_{n}x{n}_7g", geo, P.stack_materials(fuels + [mod]),
                          P.run_params(7, n_per_gen, n_gen, n_inactive, ent=(16, 16)))


def test_tables_too_large_for_lds_read_from_hbm(oracle):
    """96 x 96 pins: the kernels run on the tables in HBM instead of LDS
    copies; every history still equals the oracle's, in FP64, and FP32-mixed
    runs are balanced and independent of the launch configuration."""
    banner("96x96 lattice (tables in HBM) parity")
    prob = large_lattice()
    g = mcx.run(prob, record=True)
    o = oracle.run(prob, records=True)
    # 129,024 bins for 3000 histories: many bins hold a few flights only
    # (production = nu_sig_f(bin) x flux)
    af = flux_atol(g, prob)
    compare_runs(g, o, atol_flux=af, atol_prod=af * float(np.max(prob["xs"]["nu_sig_f"])))
    f1 = mcx.run(prob, precision="fp32", record=True)
    f2 = mcx.run(prob, precision="fp32", record=True, flights=1, tail_threshold=-1, block_size=64)
    assert np.array_equal(f1["records"], f2["records"])
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, *_ = f1["gen_counts"].T
    assert np.all(ab + leak + killed == n) and np.all(seg == col + cross)


@pytest.mark.parametrize("block,tail,look,flights", [(64, -1, 1, 1), (512, 0, 8, 3),
                                                     (1024, 1 << 30, 4, 64), (256, 100, 2, 1),
                                                     (128, -1, 3, 65536)])
def test_launch_configuration_does_not_change_results(block, tail, look, flights):
    """Block size, tail threshold (never / default / all-tail), lookahead and
    flights per advance launch: bit-identical generation results and
    per-history records (the GPU sums are exact)."""
    banner(f"determinism block={block} tail={tail} lookahead={look} flights={flights}")
    prob = P.lattice_17x17(n_per_gen=5000, n_gen=3, n_inactive=1)
    ref = mcx.run(prob, record=True)
    got = mcx.run(prob, record=True, block_size=block, tail_threshold=tail, lookahead=look,
                  flights=flights)
    for k in ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "prod_mean", "k_mean"):
        assert np.array_equal(ref[k], got[k]), k
    assert np.array_equal(ref["records"], got["records"])


@pytest.mark.parametrize("block,rounds,flights,prec", [(256, 2, 8, "fp64"), (256, 4, 8, "fp64"),
                                                       (64, 64, 1, "fp64"), (1024, 4, 3, "fp64"),
                                                       (128, 8, 65536, "fp64"),
                                                       (256, 4, 8, "fp32")])
def test_refilled_advance_gives_identical_results(block, rounds, flights, prec):
    """The advance kernel whose lanes take the next particle of their block's
    chunk when theirs stops: bit-identical generation results and records,
    with ragged chunks (5000 histories), one-lane waves of work (one flight
    per launch) and particles that never leave the kernel before a
    collision."""
    banner(f"refilled advance block={block} rounds={rounds} flights={flights} {prec}")
    prob = P.lattice_17x17(n_per_gen=5000, n_gen=3, n_inactive=1)
    ref = mcx.run(prob, record=True, precision=prec)
    got = mcx.run(prob, record=True, block_size=block, rounds=rounds, flights=flights,
                  precision=prec)
    for k in ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "prod_mean", "k_mean"):
        assert np.array_equal(ref[k], got[k]), k
    assert np.array_equal(ref["records"], got["records"])


def test_refilled_advance_full_size_matches_oracle(oracle):
    """1e6 histories, the first generation history by history against the
    oracle, with the refilled advance kernel."""
    banner("refilled advance: lattice 1e6 x 1 vs oracle")
    prob = P.lattice_17x17(n_per_gen=1_000_000, n_gen=2, n_inactive=1)
    g = mcx.run(prob, record=True, rounds=4)
    o = oracle.run(P.with_run(prob, n_gen=1, n_inactive=0), records=True)
    assert np.array_equal(g["gen_counts"][0], o["gen_counts"][0])
    compare_records(g["records"][0], o["records"][0], "gen 0")


@pytest.mark.parametrize("flights,prec,n", [(8, "fp64", 5000), (1, "fp64", 5000),
                                           (65536, "fp64", 3001), (8, "fp32", 5000),
                                           (3, "fp64", 70001)])
def test_lds_tally_advance_gives_identical_results(flights, prec, n):
    """The advance kernel that stages the flux tally in LDS (every launch
    forced onto it, with half the flights per launch) against the one that
    adds every flight to device memory: bit-identical generation results,
    tallies and records, for ragged last chunks, one flight per launch,
    uncapped flights, FP32-mixed, and more particles than the grid holds at
    once (grid-stride chunks)."""
    banner(f"LDS-staged tally advance flights={flights} {prec} n={n}")
    prob = P.lattice_17x17(n_per_gen=n, n_gen=3, n_inactive=1)
    ref = mcx.run(prob, record=True, precision=prec, lds_tally_min=-1, flights=flights)
    got = mcx.run(prob, record=True, precision=prec, lds_tally_min=1, flights=flights,
                  lt_flights=max(1, flights // 2))
    for k in ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "prod_mean", "k_mean",
              "flux_sigma", "prod_sigma"):
        assert np.array_equal(ref[k], got[k]), k
    assert np.array_equal(ref["records"], got["records"])


def test_lds_tally_advance_full_size_matches_oracle(oracle):
    """1e6 histories with every advance launch on the LDS-staged tally
    kernel: the first generation history by history, its event counts and
    its per-bin flux and production tallies against the oracle."""
    banner("LDS-staged tally advance: lattice 1e6 x 1 vs oracle")
    prob = P.lattice_17x17(n_per_gen=1_000_000, n_gen=2, n_inactive=1)
    g = mcx.run(prob, record=True, lds_tally_min=1, per_gen_tallies=True)
    o = oracle.run(P.with_run(prob, n_gen=1, n_inactive=0), records=True, per_gen_tallies=True)
    assert np.array_equal(g["gen_counts"][0], o["gen_counts"][0])
    compare_records(g["records"][0], o["records"][0], "gen 0")
    af = flux_atol(g, prob)
    assert_close(g["gen_flux"][0], o["gen_flux"][0], what="gen 0 flux", atol=af)
    assert_close(g["gen_prod"][0], o["gen_prod"][0], what="gen 0 production",
                 atol=af * float(np.max(prob["xs"]["nu_sig_f"])))


def test_single_history_and_tiny_runs(oracle):
    """N = 63, 65 in the reflective one-material cell (k_inf = 1.2, so small
    populations survive), N = 1 as fixed-source batches, and N = 1 in the pin
    cell, where the bank empties: both sides must report the extinction."""
    banner("tiny runs N=1, N=63, N=65")
    fuel = {k: v[0] for k, v in P.pin_cell()["xs"].items()}
    for n in (63, 65):
        prob = P.homogeneous(fuel, n, 4, 1, seed=7)
        g = mcx.run(prob, record=True)
        o = oracle.run(prob, records=True)
        compare_runs(g, o)
    # a single history per batch (fixed source: no bank to empty)
    prob = P.homogeneous(fuel, 1, 5, 0, seed=7, fixed_source=True)
    g = mcx.run(prob, record=True)
    o = oracle.run(prob, records=True)
    compare_runs(g, o)
    prob = P.pin_cell(n_per_gen=1, n_gen=6, n_inactive=1, seed=7)
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(prob)
    assert e.value.code == -7
    ctx = mcx.Context(prob)
    try:
        assert ctx.run(check=False) == mcx.EEXTINCT
    finally:
        ctx.close()


def test_fixed_source_batch_parity(oracle):
    """A fixed-source pin cell (fission as capture) with a nonzero problem id."""
    banner("fixed-source parity")
    prob = P.batch_pin_cells(n_problems=8)[5]
    prob = P.with_run(prob, n_per_gen=3000, n_gen=3, n_inactive=0)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare_runs(g, o)
    assert np.all(g["gen_counts"][:, 7] == 0)


@pytest.mark.parametrize("flights,tail", [(1, -1), (8, -1), (2, 0), (8, 1 << 30)])
def test_event_guard_matches_oracle(oracle, flights, tail):
    """The guard inside a multi-flight advance launch, between launches and in
    the tail kernel."""
    banner(f"event guard parity flights={flights} tail={tail}")
    prob = P.with_run(P.pin_cell(n_per_gen=2000, n_gen=3, n_inactive=1), max_events=3)
    g = mcx.run(prob, record=True, flights=flights, tail_threshold=tail)
    o = oracle.run(prob, records=True)
    assert g["rc"] == mcx.EGUARD
    compare_runs(g, o)


def test_extinct_population_is_reported():
    banner("extinct population")
    fuel = {k: v[0] for k, v in P.pin_cell()["xs"].items()}
    fuel["nu_sig_f"] = fuel["nu_sig_f"] * 1e-12
    prob = P.homogeneous(fuel, 50, 3, 1, seed=19)
    ctx = mcx.Context(prob)
    try:
        assert ctx.run(check=False) == mcx.EEXTINCT
    finally:
        ctx.close()


def test_workspace_too_small_is_rejected():
    banner("workspace too small")
    import ctypes as C

    import torch

    prob = P.pin_cell(n_per_gen=100, n_gen=2, n_inactive=1)
    ctx = mcx.Context(prob)
    try:
        L = ctx.L
        small = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
        rc = L.mcx_bind_workspace(ctx.h, small.data_ptr(), 1024, 2)
        assert rc == mcx.ENOMEM
        rc = L.mcx_run_generations(ctx.h, 2, 1)
        assert rc == mcx.ESTATE
        n = C.c_size_t()
        assert L.mcx_workspace_size(ctx.h, 2, C.byref(n)) == 0
        assert L.mcx_bind_workspace(ctx.h, ctx.workspace.data_ptr() + 8, n.value, 2) == mcx.EINVAL
    finally:
        ctx.close()


def test_full_size_first_generations(oracle):
    """The benchmark's lattice at full size (1e6 histories): the first two
    generations history by history."""
    banner("lattice 1e6 x 2 records parity")
    prob = P.lattice_17x17(n_per_gen=1_000_000, n_gen=2, n_inactive=1)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare_runs(g, o, tallies=False)
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux")
    assert_close(g["gen_prod"], o["gen_prod"], what="gen_prod")


def test_headline_size_two_generations_parity(oracle):
    """The headline lattice at 1e7 histories per generation (the launches
    stage their flux in LDS, the tail starts at 131,072 live particles):
    both generations history by history against the oracle, so the first
    generation's fission bank, its canonical order and the combing at full
    size are checked through the second generation's histories, plus each
    generation's event counts, k estimators and flux and production
    tallies."""
    banner("lattice 1e7 x 2 records parity")
    prob = P.lattice_17x17(n_per_gen=10_000_000, n_gen=2, n_inactive=1)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    assert np.array_equal(g["gen_counts"], o["gen_counts"])
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")
    assert_close(g["gen_entropy"], o["gen_entropy"], what="entropy")
    for gen in range(2):
        compare_records(g["records"][gen], o["records"][gen], f"gen {gen}")
    af = flux_atol(g, prob)
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux", atol=af)
    assert_close(g["gen_prod"], o["gen_prod"], what="gen_prod",
                 atol=af * float(np.max(prob["xs"]["nu_sig_f"])))


def test_supercritical_generation_end_parity(oracle):
    """A one-group infinite medium with k = 3: the first generation (k_used
    = 1) banks about three sites per history, so the sites of the first
    1,024 histories (about 3,100) exceed what the generation end stages in
    LDS per bucket and are written one by one, while the next bucket and the
    later generations go through LDS.  Records, k, entropy and the last
    bank against the oracle."""
    banner("supercritical infinite medium 1500 x 3 records parity")
    prob = P.homogeneous(P.one_group(1.0, 0.2, 2.4), 1500, 3, 1, seed=62)
    g = mcx.run(prob, record=True, bank=True)
    o = oracle.run(prob, records=True, bank_cap=4 * prob["run"]["n_per_gen"])
    assert o["records"][0]["n_sites"][:1024].sum() > 2048
    compare_runs(g, o, tallies=False)
    assert np.array_equal(g["bank"], o["bank"])


def test_largest_generation_sampled_parity(oracle):
    """2^28 histories per generation, the largest power of two whose
    workspace (about 110 GB with records) fits one MI355X: particle indices
    up to 2^28, fission-site arrays past 4 GB, 65,536 scan chunks and about
    2^19 canonical buckets.  The oracle cannot run it whole, but a
    first-generation history depends only on the problem, the seed and its
    id, so 4,096 histories of generation 0 (the first and last ids, and ids
    at 2^24 and 2^27, among them) are checked record by record against the
    oracle's.  Both generations balance exactly: population, events and
    sites in the counters, and the same totals summed over the per-history
    records.  Generation 1 starts from the combed bank of generation 0; its
    k estimate agrees statistically with the oracle's second generation at
    1e6 histories."""
    import gc

    import torch

    banner("lattice 2^28 x 2 sampled records")
    n = 1 << 28
    prob = P.lattice_17x17(n_per_gen=n, n_gen=2, n_inactive=1)
    ctx = mcx.Context(prob, record=True)
    try:
        ctx.run()
        _, c = ctx.generation_stats()
        _, _, gk = ctx.keff()
        seg, col, cross, refl, leak, ab, killed, sites, scat, *_ = c.T
        assert np.all(ab + leak + killed == n) and np.all(killed == 0)
        assert np.all(col == scat + ab) and np.all(seg == col + cross)
        kcol_sd = []
        for gen in range(2):
            rec = ctx.records(gen)
            for f, tot in (("n_seg", seg), ("n_col", col), ("n_cross", cross),
                           ("n_refl", refl), ("n_sites", sites)):
                assert int(rec[f].sum(dtype=np.int64)) == int(tot[gen]), (gen, f)
            assert int((rec["fate"] == 2).sum()) == int(leak[gen])
            assert int((rec["fate"] == 1).sum()) == int(ab[gen])
            kc = rec["kcol_sum"]
            assert_close(kc.sum() / n, gk[gen, 0], rtol=1e-10, what=f"gen {gen} k_col")
            kcol_sd.append(float(kc.std()))
            if gen == 0:
                rng = np.random.default_rng(51)
                fixed = [0, 1, (1 << 24) - 1, 1 << 24, (1 << 27) - 1, 1 << 27, n - 2, n - 1]
                ids = np.unique(np.concatenate([fixed, rng.integers(0, n, 4096 - len(fixed))]))
                compare_records(rec[ids], oracle.histories(prob, ids), "gen 0 sample")
            del rec, kc
            gc.collect()
    finally:
        ctx.close()
        del ctx
        gc.collect()
        torch.cuda.empty_cache()
    no = 1_000_000
    o = oracle.run(P.with_run(prob, n_per_gen=no), records=True)
    ko = o["records"][1]["kcol_sum"]
    sigma = math.hypot(float(ko.std()) / math.sqrt(no), kcol_sd[1] / math.sqrt(n))
    assert abs(gk[1, 0] - o["gen_k"][1, 0]) < 4.5 * sigma, (gk[1, 0], o["gen_k"][1, 0], sigma)


def test_headline_invariants_in_bench_configuration():
    """The bench's headline run (1e7 x 60, 20 inactive) in its launch
    configuration: particle, event and site balance in every generation, no
    guard kills, and the three k estimators agree statistically."""
    banner("lattice 1e7 x 60 invariants")
    prob = P.lattice_17x17(n_per_gen=10_000_000)
    g = mcx.run(prob)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cutoff, *_ = g["gen_counts"].T
    assert np.all(ab + leak + killed == n)
    assert np.all(killed == 0)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    km, ks = g["k_mean"], g["k_sigma"]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(km[a] - km[b]) < 4 * math.hypot(ks[a], ks[b]), (km, ks)
    k_used = np.concatenate([[1.0], g["gen_k"][:-1, 0]])
    expect = n * g["gen_k"][:, 0] / k_used
    assert np.all(np.abs(sites - expect) < 4 * np.sqrt(col / 4.0))


def test_full_size_invariants_in_bench_configuration():
    """The benchmark run (1e6 x 60, 20 inactive) in its launch configuration:
    particle, event and site balance in every generation, and the three k
    estimators agree statistically."""
    banner("lattice 1e6 x 60 invariants")
    prob = P.lattice_17x17()
    g = mcx.run(prob)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cutoff, *_ = g["gen_counts"].T
    assert np.all(ab + leak + killed == n)
    assert np.all(killed == 0)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    km, ks = g["k_mean"], g["k_sigma"]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(km[a] - km[b]) < 4 * math.hypot(ks[a], ks[b]), (km, ks)
    # bank size follows k_used (see the oracle pin of the same relation)
    k_used = np.concatenate([[1.0], g["gen_k"][:-1, 0]])
    expect = n * g["gen_k"][:, 0] / k_used
    assert np.all(np.abs(sites - expect) < 4 * np.sqrt(col / 4.0))


@pytest.mark.parametrize("tail", [1 << 30, 0])
def test_flights_with_many_draws_through_the_tail(oracle, tail):
    """Collisions that bank several sites each (nu_sig_f = 2 sigma_t with
    k_used = 1 in generation 0, so a collision flight takes 8 or more draws):
    in the tail kernel such a flight runs past the end of its window of
    precomputed draws and finishes by evaluating the rest itself.  Every
    history through the tail (threshold above N) and through the event
    kernels, against the oracle, with the generation's bank."""
    banner(f"many draws per flight, tail threshold {tail}")
    xs = P.one_group(1.0, 0.2, 2.0)
    prob = P.homogeneous(xs, 2000, 2, 1, seed=41)
    g = mcx.run(prob, record=True, bank=True, tail_threshold=tail)
    o = oracle.run(prob, records=True, bank_cap=20000)
    assert np.array_equal(g["gen_counts"], o["gen_counts"])
    assert g["gen_counts"][0, 7] > 2 * 2000  # more than two sites per history
    for gen in range(2):
        compare_records(g["records"][gen], o["records"][gen], f"gen {gen}")
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")
    assert np.array_equal(g["bank"], o["bank"])


def test_pin_cell_against_stored_oracle_results():
    """The 7-group pin cell, 1e4 histories x 30 generations, against the
    oracle's results stored in tests/golden/ (no oracle run needed): event
    counts exactly, k estimators, entropy and the active flux mean and sigma
    to 1e-12 relative (flux within the fixed-point quantum)."""
    import json
    import os
    banner("pin cell 1e4 x 30 against tests/golden")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "pin_cell_7g_1e4x30.json")
    with open(path) as f:
        gd = json.load(f)
    pr = dict(gd["problem"])
    pr.pop("name")
    prob = P.pin_cell(**pr)
    g = mcx.run(prob)
    assert list(mcx.COUNT_NAMES) == gd["count_names"]
    assert np.array_equal(g["gen_counts"], np.array(gd["gen_counts"]))
    assert_close(g["gen_k"], np.array(gd["gen_k"]), what="gen_k")
    assert_close(g["gen_entropy"], np.array(gd["gen_entropy"]), what="entropy")
    atol = flux_atol(g, prob)
    assert_close(g["flux_mean"], np.array(gd["flux_mean"]), what="flux_mean", atol=atol)
    assert_close(g["flux_sigma"], np.array(gd["flux_sigma"]), what="flux_sigma", atol=atol)
