"""FP32-mixed mode: k-eff against FP64 (the GPU FP64 path, which the parity
tests tie to the oracle history by history, and the oracle itself).

Acceptance: |dk| <= 10 pcm and |dk| <= 3 paired sigma (the two runs share
their random streams, so sigma comes from the per-generation differences),
on the lattice at 1e7 histories per generation and on the continuous-energy
pin cell at 1e6 histories per generation (two seeds); per-pin flux
differences within 3 sigma of independent replicas for at least 99% of the
pins."""
import math

import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def pin_flux(res, prob):
    geo = prob["geometry"]
    G = prob["xs"]["sig_t"].shape[1]
    mr1 = geo["radii"].shape[1] + 1
    m = res["flux_mean"].reshape(geo["ny"] * geo["nx"], mr1 * G).sum(axis=1)
    s = np.sqrt((res["flux_sigma"].reshape(geo["ny"] * geo["nx"], mr1 * G) ** 2).sum(axis=1))
    return m, s


def paired_dk(g32, g64, n_inactive):
    """k_col difference and its paired sigma: both runs use the same random
    streams, so the sigma comes from the per-generation differences."""
    d = g32["gen_k"][n_inactive:, 0] - g64["gen_k"][n_inactive:, 0]
    return g32["k_mean"][0] - g64["k_mean"][0], d.std(ddof=1) / math.sqrt(len(d))


def test_fp32_mixed_lattice_1e7_within_10_pcm():
    banner("lattice 1e7 x 60: FP32-mixed vs FP64")
    prob = P.lattice_17x17(n_per_gen=10_000_000)
    g64 = mcx.run(prob, precision="fp64")
    g32 = mcx.run(prob, precision="fp32")
    dk, paired = paired_dk(g32, g64, 20)
    print(f"k64 {g64['k_mean'][0]:.6f} k32 {g32['k_mean'][0]:.6f} dk {dk * 1e5:.3f} pcm "
          f"paired sigma {paired * 1e5:.3f} pcm", flush=True)
    assert abs(dk) <= 10e-5
    assert abs(dk) <= 3 * paired
    for c in ("seg", "col"):
        i = mcx.COUNT_NAMES.index(c)
        r = g32["gen_counts"][:, i].sum() / g64["gen_counts"][:, i].sum()
        assert abs(r - 1) < 1e-3, (c, r)


def test_fp32_mixed_per_pin_flux_over_independent_replicas():
    """Per-pin flux (all rings and groups of a lattice cell): K independent
    replicas (own transport seed each) of the FP32-mixed / FP64 pair give K
    differences per pin; their mean over the replica spread (Student t with
    K - 1 degrees of freedom) is within 3 sigma for at least 99% of the 289
    pins, and the z-scores follow that t distribution (no bias)."""
    from scipy import stats
    K = 40
    banner(f"lattice per-pin flux FP32-mixed vs FP64, {K} replicas of 2e5 x 40")
    base = P.lattice_17x17(n_per_gen=200_000, n_gen=40, n_inactive=10)
    d = []
    for k in range(K):
        prob = P.with_run(base, seed=7000 + k)
        f64, _ = pin_flux(mcx.run(prob, precision="fp64"), prob)
        f32, _ = pin_flux(mcx.run(prob, precision="fp32"), prob)
        d.append((f32 - f64) / f64)
    d = np.array(d)
    z = d.mean(axis=0) / (d.std(axis=0, ddof=1) / math.sqrt(K))
    frac = float(np.mean(np.abs(z) <= 3.0))
    ks = stats.kstest(z, stats.t(K - 1).cdf).pvalue
    print(f"per-pin z: within 3 sigma {frac:.4f}, max |z| {np.abs(z).max():.2f}, "
          f"mean z {z.mean():.3f}, KS p {ks:.3g}, mean |rel diff| {np.abs(d.mean(axis=0)).mean():.2e}",
          flush=True)
    assert frac >= 0.99
    assert ks > 1e-3
    # no common bias: the pin-averaged relative difference of each replica
    # is a scalar whose replica mean is within 3 sigma of 0
    a = d.mean(axis=1)
    assert abs(a.mean()) <= 3 * a.std(ddof=1) / math.sqrt(K)


def test_fp32_mixed_against_oracle(oracle):
    banner("lattice 1e5 x 30: FP32-mixed vs oracle")
    prob = P.lattice_17x17(n_per_gen=100_000, n_gen=30, n_inactive=10)
    g32 = mcx.run(prob, precision="fp32")
    o = oracle.run(prob)
    for e in range(3):
        sig = math.hypot(g32["k_sigma"][e], o["k_sigma"][e])
        assert abs(g32["k_mean"][e] - o["k_mean"][e]) <= 3 * sig, (e, g32["k_mean"], o["k_mean"])


def test_fp32_mixed_balance_and_determinism():
    banner("FP32-mixed balance and launch-configuration determinism")
    prob = P.lattice_17x17(n_per_gen=20000, n_gen=4, n_inactive=1)
    a = mcx.run(prob, precision="fp32")
    b = mcx.run(prob, precision="fp32", block_size=512, tail_threshold=-1)
    for k in ("gen_k", "gen_counts", "flux_mean", "gen_entropy"):
        assert np.array_equal(a[k], b[k]), k
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cutoff, *_ = a["gen_counts"].T
    assert np.all(ab + leak + killed == n)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)


def test_fp32_mixed_accepts_rows_that_round_above_sig_t():
    """A scattering row summing to at most sig_t in binary64 whose binary32
    running sum rounds above binary32 sig_t is valid data: FP32-mixed loads
    it (the row is clamped to sig_t, a scatter probability of 1) and the
    runs balance; FP64 accepts it as well."""
    banner("FP32-mixed load of a row that rounds above sig_t in binary32")
    t, a, b = 1.1197442375383306, 0.0013433387832206944, 1.11840089875511
    assert a + b <= t and np.float32(np.float32(a) + np.float32(b)) > np.float32(t)
    mod = dict(sig_t=np.array([t, 1.0]), sig_s=np.array([[a, b], [0.0, 0.9]]),
               nu_sig_f=np.zeros(2), chi=np.zeros(2))
    fuel = P.mg_material(np.random.default_rng(91), n_groups=2)
    geo = P.lattice_geometry(1, 1, P.PIN_PITCH, [([P.PIN_RADIUS], [0, 1])], [[0]],
                             [P.REFLECT] * 4)
    prob = P.make_problem("clamp", geo, P.stack_materials([fuel, mod]),
                          P.run_params(92, 4000, 4, 1))
    for prec in ("fp32", "fp64"):
        r = mcx.run(prob, precision=prec)
        n = prob["run"]["n_per_gen"]
        seg, col, cross, refl, leak, ab, killed, sites, scat, *_ = r["gen_counts"].T
        assert np.all(ab + leak + killed == n) and np.all(col == scat + ab), prec
