"""GPU: the persistent engine and batches of fixed-source problems.

The persistent engine runs each history through the same operations in the
same order as the event engine, so per-history outcomes are identical and,
with the exact fixed-point sums, so is every generation result: bit for bit
against the event engine on the same problem (same fixed-point scales).  A
problem inside a batch shares the batch's fixed-point scales, so its
estimators agree with a run of the problem alone to 1e-12 relative and its
counters exactly.  The oracle is the reference for both.
"""
import os

import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu

RTOL = 1e-12
EXACT_KEYS = ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "prod_mean", "k_mean",
              "flux_sigma", "prod_sigma", "k_sigma")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def assert_close(a, b, rtol=RTOL, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    assert a.shape == b.shape, what
    bad = np.abs(a - b) > rtol * np.maximum(np.abs(a), np.abs(b))
    assert not bad.any(), f"{what}: {bad.sum()} differ, first at {np.argwhere(bad)[:3].tolist()}"


def assert_same_run(ref, got, keys=EXACT_KEYS):
    for k in keys:
        assert np.array_equal(ref[k], got[k]), k


def test_persistent_engine_equals_event_engine_pin_cell():
    """k-eigenvalue pin cell, 1e4 x 30: every generation result bit for bit."""
    banner("persistent == event, pin cell 1e4 x 30")
    prob = P.pin_cell()
    ev = mcx.run(prob, per_gen_tallies=True)
    pe = mcx.run(prob, per_gen_tallies=True, engine="persistent")
    assert_same_run(ev, pe)
    assert np.array_equal(ev["gen_flux"], pe["gen_flux"])


def test_persistent_engine_matches_oracle_lattice(oracle):
    """17x17 lattice, 12345 histories (ragged against every slot count)."""
    banner("persistent vs oracle, lattice 12345 x 5")
    prob = P.lattice_17x17(n_per_gen=12345, n_gen=5, n_inactive=2)
    g = mcx.run(prob, per_gen_tallies=True, engine="persistent")
    o = oracle.run(prob, per_gen_tallies=True)
    assert np.array_equal(g["gen_counts"], o["gen_counts"])
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")
    assert_close(g["gen_entropy"], o["gen_entropy"], what="entropy")
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux")
    assert_close(g["gen_prod"], o["gen_prod"], what="gen_prod")
    ev = mcx.run(prob, engine="event")
    assert_same_run(ev, g, ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "k_mean"))


@pytest.mark.parametrize("cfg", [dict(block=128, slots=256, grid=1, tau=1.0),
                                 dict(block=128, slots=512, grid=37, tau=0.5, sort=1),
                                 dict(block=256, slots=256, grid=256, tau=0.9),
                                 dict(block=256, slots=512, grid=1024, tau=0.25, sort=1)])
def test_persistent_configuration_does_not_change_results(cfg):
    banner(f"persistent configuration {cfg}")
    prob = P.lattice_17x17(n_per_gen=5000, n_gen=3, n_inactive=1)
    ref = mcx.run(prob)
    got = mcx.run(prob, engine="persistent", persistent=cfg)
    assert_same_run(ref, got)


def test_persistent_fp32_mixed_equals_event_fp32_mixed():
    banner("persistent == event in FP32-mixed, lattice 20000 x 4")
    prob = P.lattice_17x17(n_per_gen=20000, n_gen=4, n_inactive=1)
    ev = mcx.run(prob, precision="fp32")
    pe = mcx.run(prob, precision="fp32", engine="persistent")
    assert_same_run(ev, pe)


def test_persistent_fixed_source_and_guard(oracle):
    """Fixed source (source sampled inside the persistent kernel) and the
    event guard."""
    banner("persistent fixed source + event guard")
    prob = P.with_run(P.batch_pin_cells(n_problems=8)[5], n_per_gen=3000, n_gen=3,
                      n_inactive=0)
    ev = mcx.run(prob, per_gen_tallies=True)
    pe = mcx.run(prob, per_gen_tallies=True, engine="persistent")
    assert_same_run(ev, pe)
    o = oracle.run(prob, per_gen_tallies=True)
    assert np.array_equal(pe["gen_counts"], o["gen_counts"])
    assert_close(pe["gen_k"], o["gen_k"], what="gen_k")
    guarded = P.with_run(P.pin_cell(n_per_gen=2000, n_gen=3, n_inactive=1), max_events=3)
    ev = mcx.run(guarded)
    pe = mcx.run(guarded, engine="persistent")
    assert ev["rc"] == pe["rc"] == mcx.EGUARD
    assert_same_run(ev, pe)


def test_persistent_extinction_is_reported():
    banner("persistent extinction")
    fuel = {k: v[0] for k, v in P.pin_cell()["xs"].items()}
    fuel["nu_sig_f"] = fuel["nu_sig_f"] * 1e-12
    prob = P.homogeneous(fuel, 50, 3, 1, seed=19)
    ctx = mcx.Context(prob, engine="persistent")
    try:
        assert ctx.run(check=False) == mcx.EEXTINCT
    finally:
        ctx.close()


def small_batch(n=24, cap=20000):
    probs = P.batch_pin_cells(n_problems=n)
    return [P.with_run(p, n_per_gen=min(cap, p["run"]["n_per_gen"])) for p in probs]


def single_result(prob):
    g = mcx.run(prob, per_gen_tallies=True)
    return g["gen_k"][0], g["gen_counts"][0], g["gen_flux"][0], g["gen_prod"][0]


def test_batch_equals_single_runs_and_oracle(oracle):
    """24 problems of uneven size in one launch: each problem's counters equal
    its run alone exactly, estimators and tallies to 1e-12."""
    banner("batch of 24 vs single runs and oracle")
    probs = small_batch()
    b = mcx.Batch(probs)
    try:
        b.run()
        k, cnt = b.results()
        for p, prob in enumerate(probs):
            sk, sc, sf, sp = single_result(prob)
            assert np.array_equal(cnt[p], sc), p
            assert_close(k[p], sk, what=f"k of problem {p}")
            f, q = b.tallies_of(p)
            assert_close(f, sf, what=f"flux of problem {p}")
            assert_close(q, sp, what=f"production of problem {p}")
        for p in (0, 7, 23):
            o = oracle.run(probs[p], per_gen_tallies=True)
            assert np.array_equal(cnt[p], o["gen_counts"][0]), p
            assert_close(k[p], o["gen_k"][0], what=f"oracle k {p}")
            f, q = b.tallies_of(p)
            assert_close(f, o["gen_flux"][0], what=f"oracle flux {p}")
        # the recorded graph replays to the same results
        b.run()
        k2, cnt2 = b.results()
        assert np.array_equal(k, k2) and np.array_equal(cnt, cnt2)
    finally:
        b.close()


def test_batch_sorted_collide_lists_equal_unsorted():
    banner("batch with sorted collide lists")
    probs = small_batch(n=12, cap=6000)
    out = []
    for sort in (0, 1):
        b = mcx.Batch(probs, persistent=dict(sort=sort))
        try:
            b.run()
            out.append(b.results())
        finally:
            b.close()
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[1][0])


def test_batch_fp32_mixed_equals_single_fp32_runs():
    banner("batch FP32-mixed vs single FP32-mixed runs")
    probs = small_batch(n=6, cap=8000)
    b = mcx.Batch(probs, precision="fp32")
    try:
        b.run()
        k, cnt = b.results()
        for p, prob in enumerate(probs):
            g = mcx.run(prob, precision="fp32")
            assert np.array_equal(cnt[p], g["gen_counts"][0]), p
            assert_close(k[p], g["gen_k"][0], what=f"k {p}")
    finally:
        b.close()


def test_batch_guard_and_errors():
    banner("batch guard and invalid batches")
    probs = small_batch(n=4, cap=3000)
    b = mcx.Batch(probs, max_events=3)
    try:
        assert b.run(check=False) == mcx.EGUARD
        k, cnt = b.results()
        for p, prob in enumerate(probs):
            g = mcx.run(P.with_run(prob, max_events=3))
            assert np.array_equal(cnt[p], g["gen_counts"][0])
        # a single-problem call on a batch context is refused
        assert b.L.mcx_run_generations(b.h, 1, 0) == mcx.ESTATE
    finally:
        b.close()
    bad = [dict(q) for q in small_batch(n=2, cap=100)]
    bad[1] = dict(bad[1], xs=dict(bad[1]["xs"], sig_t=bad[1]["xs"]["sig_t"][:, :5],
                                  sig_s=bad[1]["xs"]["sig_s"][:, :5, :5],
                                  nu_sig_f=bad[1]["xs"]["nu_sig_f"][:, :5],
                                  chi=bad[1]["xs"]["chi"][:, :5] /
                                  bad[1]["xs"]["chi"][:, :5].sum(1, keepdims=True).clip(1e-300)))
    with pytest.raises(mcx.MCXError) as e:
        mcx.Batch(bad)
    assert e.value.code == mcx.EINVAL


def test_autotune_picks_a_valid_configuration_and_caches(tmp_path):
    banner("autotune sweep and cache")
    probs = small_batch(n=16, cap=4000)
    cache = os.path.join(tmp_path, "tune.txt")
    b = mcx.Batch(probs)
    try:
        b.run()
        k0, c0 = b.results()
        t = b.autotune(cache)
        assert t["block"] in (128, 256) and t["slots"] in (256, 512)
        assert t["grid"] >= 1 and 0 < t["tau"] <= 1 and t["ms"] > 0
        assert t["sort"] in (0, 1)
        t2 = b.autotune(cache)  # cache hit
        assert (t2["block"], t2["slots"], t2["grid"], t2["sort"]) == (t["block"], t["slots"],
                                                                      t["grid"], t["sort"])
        b.run()
        k1, c1 = b.results()
        assert np.array_equal(c0, c1)
        assert np.array_equal(k0, k1)
    finally:
        b.close()


def test_event_engine_autotune_picks_a_valid_configuration_and_caches(tmp_path):
    """The event engine's autotuner: a configuration from its candidate sets
    (block, flights, flights of the LDS-staged launches, tail threshold), a
    cache hit on the second call, and a run afterwards equal bit for bit to
    an untuned run (results do not depend on the launch configuration)."""
    banner("event-engine autotune")
    prob = P.lattice_17x17(n_per_gen=20000, n_gen=3, n_inactive=1)
    cache = os.path.join(tmp_path, "tune.txt")
    ref = mcx.run(prob, record=True)
    ctx = mcx.Context(prob, record=True)
    try:
        t = ctx.autotune(cache)
        assert t["block"] in (256, 512) and t["flights"] in (6, 8)
        assert t["lt_flights"] in (3, 4, 5, 6) and t["tail"] >= 4096 and t["ms"] > 0
        t2 = ctx.autotune(cache)  # cache hit
        for k in ("block", "flights", "lt_flights", "tail"):
            assert t2[k] == t[k], k
        ctx.run()
        m, s, pg = ctx.keff()
        h, c = ctx.generation_stats()
        assert np.array_equal(pg, ref["gen_k"])
        assert np.array_equal(c, ref["gen_counts"])
        for g in range(3):
            assert np.array_equal(ctx.records(g), ref["records"][g])
    finally:
        ctx.close()


def test_full_batch_512_problems():
    """The 512-problem batch (about 7.4e7 histories) in one launch: balance
    per problem, and sampled problems (smallest, largest, first) equal their
    runs alone."""
    banner("512-problem batch")
    probs = P.batch_pin_cells()
    n = np.array([p["run"]["n_per_gen"] for p in probs])
    b = mcx.Batch(probs)
    try:
        b.run()
        k, cnt = b.results()
    finally:
        b.close()
    seg, col, cross, refl, leak, ab, killed, sites, scat, cutoff, *_ = cnt.T
    assert np.all(ab + leak + killed == n)
    assert np.all(killed == 0) and np.all(leak == 0)  # reflective cells
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    assert np.all(sites == 0)
    assert np.all(np.isfinite(k)) and np.all(k > 0)
    for p in (int(n.argmin()), int(n.argmax()), 0):
        sk, sc, _, _ = single_result(probs[p])
        assert np.array_equal(cnt[p], sc), p
        assert_close(k[p], sk, what=f"k of problem {p}")
