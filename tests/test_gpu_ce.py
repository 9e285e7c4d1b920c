"""GPU parity of the continuous-energy path against the CPU oracle.

The continuous-energy kernels repeat the oracle's operations in the same
order (lookup, Watt sampling, elastic kinematics and rotation included), so
histories are identical: integers of every record equal, floating-point
record fields and generation results within 1e-12 relative.
"""
import math

import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu

RTOL = 1e-12
INT_FIELDS = ["n_seg", "n_col", "n_cross", "n_refl", "fate", "n_sites", "g_final", "ctr_final"]
FP_FIELDS = ["tl_sum", "kcol_sum", "x_final", "y_final", "e_final"]


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def assert_close(a, b, rtol=RTOL, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    assert a.shape == b.shape, what
    bad = np.abs(a - b) > rtol * np.maximum(np.abs(a), np.abs(b))
    assert not bad.any(), f"{what}: {bad.sum()} differ, first at {np.argwhere(bad)[:3].tolist()}"


def compare(g, o, records=True):
    assert np.array_equal(g["gen_counts"], o["gen_counts"]), (g["gen_counts"], o["gen_counts"])
    assert_close(g["gen_k"], o["gen_k"], what="gen_k")
    assert_close(g["gen_entropy"], o["gen_entropy"], what="entropy")
    if records:
        for gen in range(g["records"].shape[0]):
            for f in INT_FIELDS:
                d = g["records"][gen][f] != o["records"][gen][f]
                assert not d.any(), f"gen {gen} {f}: {d.sum()} differ, first {np.argwhere(d)[:3]}"
            for f in FP_FIELDS:
                assert_close(g["records"][gen][f], o["records"][gen][f], what=f"gen {gen} {f}")


def test_ce_supercritical_generation_end_parity(oracle):
    """A flat continuous-energy medium with k near 2.4: the first generation
    banks about 2.4 sites per history, so the sites of the first 1,024
    histories exceed what the generation end stages in LDS per bucket and are
    written one by one (energies included), while the next bucket and the
    later generations go through LDS.  Records, k, entropy and the last bank
    against the oracle."""
    banner("CE supercritical flat medium 1500 x 3 records parity")
    ce = P.ce_flat(sig_s=0.5, sig_c=0.0, sig_f=1.5, awr=200.0)
    prob = P.ce_homogeneous(ce, 1500, 3, 1, seed=71)
    g = mcx.run(prob, record=True, bank=True)
    o = oracle.run(prob, records=True, bank_cap=20000)
    assert o["records"][0]["n_sites"][:1024].sum() > 2048
    compare(g, o)
    assert np.array_equal(g["bank"], o["bank"])


def test_ce_pin_cell_records_parity(oracle):
    """The continuous-energy pin cell, 3000 histories x 4 generations: every
    history, the flux tallies per generation and the final bank."""
    banner("CE pin cell 3000 x 4 records parity")
    prob = P.ce_pin_cell(n_per_gen=3000, n_gen=4, n_inactive=1)
    g = mcx.run(prob, record=True, per_gen_tallies=True, bank=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True, bank_cap=20000)
    compare(g, o)
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux")
    assert np.array_equal(g["bank"], o["bank"])
    assert np.all(g["gen_prod"] == 0)


@pytest.mark.parametrize("flights,tail,block", [(1, -1, 64), (8, 0, 256), (3, 1 << 30, 512)])
def test_ce_launch_configuration_does_not_change_results(flights, tail, block):
    banner(f"CE determinism flights={flights} tail={tail} block={block}")
    prob = P.ce_pin_cell(n_per_gen=4000, n_gen=3, n_inactive=1)
    ref = mcx.run(prob, record=True)
    got = mcx.run(prob, record=True, flights=flights, tail_threshold=tail, block_size=block)
    for k in ("gen_k", "gen_entropy", "gen_counts", "flux_mean", "k_mean"):
        assert np.array_equal(ref[k], got[k]), k
    assert np.array_equal(ref["records"], got["records"])


def test_ce_flat_infinite_medium_and_cutoff(oracle):
    """Flat cross sections (k_inf = nu sigma_f / sigma_a) and a pure
    hydrogen-like scatterer (every history ends at the cutoff), both against
    the oracle history by history."""
    banner("CE flat medium and cutoff")
    ce = P.ce_flat(sig_s=8.0, sig_c=1.5, sig_f=1.0, awr=200.0, dens=0.05)
    prob = P.ce_homogeneous(ce, 2000, 4, 1, seed=21)
    g = mcx.run(prob, record=True)
    o = oracle.run(prob, records=True)
    compare(g, o)
    assert np.allclose(g["gen_k"][:, 2], P.NU_CE / 2.5, rtol=1e-12)
    # nearly a pure scatterer (the source needs a fissile material; a k term
    # far below the fixed-point quantum of the estimator sums would vanish)
    ce = P.ce_flat(sig_s=10.0, sig_c=0.0, sig_f=0.01, awr=1.0, dens=0.1)
    prob = P.ce_homogeneous(ce, 3000, 2, 0, seed=22, fixed_source=True)
    g = mcx.run(prob, record=True)
    o = oracle.run(prob, records=True)
    compare(g, o)
    cut, ab = g["gen_counts"][:, 9], g["gen_counts"][:, 5]
    assert np.all(cut + ab == 3000) and np.all(cut > 0.9 * 3000)


def test_ce_uneven_and_shared_materials(oracle):
    """Materials of different sizes (3 and 5 nuclides, so the packed table
    has unused entries) that share a nuclide: history parity with the
    oracle, FP64 and, in the FP32-mixed mode, launch-configuration
    independence."""
    banner("CE uneven and shared materials")
    ce = dict(P.ce_data())
    mat_nuc = ce["mat_nuc"].copy()
    mat_dens = ce["mat_dens"].copy()
    mat_nuc[0, :3] = [9, 8, 2]          # fuel: two fissile nuclides and a moderator one
    mat_nuc[0, 3:] = 0
    mat_dens[0, 3:] = 0.0
    ce.update(mat_n=np.array([3, 5], np.int32), mat_nuc=mat_nuc, mat_dens=mat_dens)
    prob = P.ce_pin_cell(n_per_gen=2000, n_gen=3, n_inactive=1, data=ce)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(prob, records=True, per_gen_tallies=True)
    compare(g, o)
    assert_close(g["gen_flux"], o["gen_flux"], what="gen_flux")
    a = mcx.run(prob, precision="fp32", record=True)
    b = mcx.run(prob, precision="fp32", record=True, flights=1, tail_threshold=-1, block_size=64)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["gen_k"], b["gen_k"])


def test_ce_event_guard(oracle):
    banner("CE event guard")
    prob = P.with_run(P.ce_pin_cell(n_per_gen=1500, n_gen=2, n_inactive=1), max_events=20)
    g = mcx.run(prob, record=True)
    o = oracle.run(prob, records=True)
    assert g["rc"] == mcx.EGUARD
    compare(g, o)


def test_ce_persistent_engine_is_refused():
    banner("CE refuses the persistent engine")
    prob = P.ce_pin_cell(n_per_gen=100, n_gen=2, n_inactive=1)
    with pytest.raises(mcx.MCXError) as e:
        mcx.Context(prob, engine="persistent")
    assert e.value.code == mcx.EINVAL


def test_ce_fp32_mixed_against_fp64():
    """FP32-mixed continuous energy: deterministic for any launch
    configuration, balanced, and within statistics of FP64 on the same
    streams (paired per-generation differences)."""
    banner("CE FP32-mixed vs FP64, 20000 x 12")
    prob = P.ce_pin_cell(n_per_gen=20000, n_gen=12, n_inactive=2)
    g32 = mcx.run(prob, precision="fp32", record=True)
    g32b = mcx.run(prob, precision="fp32", record=True, flights=1, tail_threshold=-1,
                   block_size=128)
    for k in ("gen_k", "gen_counts", "flux_mean", "gen_entropy"):
        assert np.array_equal(g32[k], g32b[k]), k
    assert np.array_equal(g32["records"], g32b["records"])
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, *_ = g32["gen_counts"].T
    assert np.all(ab + leak + killed + cut == n) and np.all(killed == 0)
    assert np.all(col == scat + ab) and np.all(seg == col + cross)
    g64 = mcx.run(prob)
    d = g32["gen_k"][2:, 0] - g64["gen_k"][2:, 0]
    sig = d.std(ddof=1) / math.sqrt(len(d))
    assert abs(d.mean()) < 5 * sig + 1e-12, (d.mean(), sig)
    # flux spectra agree bin by bin within their statistical noise
    f32, f64 = g32["flux_mean"], g64["flux_mean"]
    s = np.hypot(g32["flux_sigma"], g64["flux_sigma"])
    ok = s > 0
    z = np.abs(f32[ok] - f64[ok]) / s[ok]
    assert np.mean(z < 4) > 0.97, np.sort(z)[-5:]


def test_ce_full_size_first_generation(oracle):
    """The benchmark's continuous-energy pin cell at full size (1e6
    histories): the first generation history by history."""
    banner("CE pin cell 1e6 x 1 records parity")
    prob = P.ce_pin_cell(n_per_gen=1_000_000, n_gen=2, n_inactive=1)
    g = mcx.run(prob, record=True, per_gen_tallies=True)
    o = oracle.run(P.with_run(prob, n_gen=1, n_inactive=0), records=True, per_gen_tallies=True)
    assert np.array_equal(g["gen_counts"][0], o["gen_counts"][0])
    assert_close(g["gen_k"][0], o["gen_k"][0], what="gen_k")
    for f in INT_FIELDS:
        assert np.array_equal(g["records"][0][f], o["records"][0][f]), f
    for f in FP_FIELDS:
        assert_close(g["records"][0][f], o["records"][0][f], what=f)
    assert_close(g["gen_flux"][0], o["gen_flux"][0], what="gen_flux")


def test_ce_bench_configuration_invariants():
    """1e6 x 50 (10 inactive) in the benchmark's launch configuration:
    balance in every generation, estimators agree."""
    banner("CE pin cell 1e6 x 50 invariants")
    prob = P.ce_pin_cell()
    g = mcx.run(prob)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, *_ = g["gen_counts"].T
    assert np.all(ab + leak + killed + cut == n)
    assert np.all(killed == 0) and np.all(leak == 0)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    km, ks = g["k_mean"], g["k_sigma"]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(km[a] - km[b]) < 5 * math.hypot(ks[a], ks[b]), (km, ks)


@pytest.mark.parametrize("seed", [4, 14])
def test_ce_fp32_mixed_full_size_within_10_pcm(seed):
    """The continuous-energy pin cell at full size (1e6 x 50, 10 inactive):
    FP32-mixed k_col within 10 pcm and 3 paired sigma of FP64 on the same
    random streams."""
    banner(f"CE pin cell 1e6 x 50 FP32-mixed vs FP64, seed {seed}")
    prob = P.ce_pin_cell(seed=seed)
    g64 = mcx.run(prob)
    g32 = mcx.run(prob, precision="fp32")
    ni = prob["run"]["n_inactive"]
    d = g32["gen_k"][ni:, 0] - g64["gen_k"][ni:, 0]
    dk = g32["k_mean"][0] - g64["k_mean"][0]
    paired = d.std(ddof=1) / math.sqrt(len(d))
    print(f"seed {seed}: k64 {g64['k_mean'][0]:.7f} k32 {g32['k_mean'][0]:.7f} "
          f"dk {dk * 1e5:.3f} pcm paired sigma {paired * 1e5:.3f} pcm", flush=True)
    assert abs(dk) <= 10e-5
    assert abs(dk) <= 3 * paired
