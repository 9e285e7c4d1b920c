"""Pins of the oracle's continuous-energy physics (paper Sec. 1 lists
continuous-energy transport among the method's capabilities; Sec. 4 runs a
continuous-energy pin cell).  Each building block is checked against an
independent definition: library routines (searchsorted, interp), published
distributions (Maxwellian, Watt), two-body kinematics identities, and
closed-form infinite-medium answers of whole runs.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2501_05440_amd import problems as P


def test_interval_matches_searchsorted(oracle):
    rng = np.random.default_rng(11)
    grid = np.cumsum(rng.uniform(0.1, 2.0, 257))
    e = np.concatenate([rng.uniform(grid[0] - 3, grid[-1] + 3, 2000), grid, [grid[0], grid[-1]]])
    want = np.clip(np.searchsorted(grid, e, side="right") - 1, 0, len(grid) - 2)
    got = np.array([oracle.ce_interval(grid, v) for v in e])
    assert np.array_equal(got, want)


def test_macroscopic_xs_matches_numpy_interp(oracle):
    ce = P.ce_data(n_pts=2000, n_res=20)
    rng = np.random.default_rng(12)
    e = np.exp(rng.uniform(math.log(1e-6), math.log(3e7), 500))
    for m in range(2):
        for v in e:
            got = oracle.ce_macro(ce, m, v)
            for q, key in enumerate(("sig_t", "sig_s", "sig_f")):
                want = 0.0
                for k in range(ce["mat_n"][m]):
                    n = ce["mat_nuc"][m][k]
                    # np.interp holds the end values outside the grid, as the
                    # clipped interpolation fraction does
                    want += ce["mat_dens"][m][k] * np.interp(v, ce["e_grid"], ce[key][n])
                assert abs(got[q] - want) <= 1e-13 * abs(want) + 1e-300, (m, v, key)


def _watt_sample(oracle, a, b, n, seed):
    rng = np.random.default_rng(seed)
    xi = ((rng.integers(0, 2**52, (n, 4)).astype(np.float64)) + 0.5) * 2.0**-52
    return np.array([oracle.watt_attempt(a, b, *row) for row in xi])


def test_maxwellian_part_of_the_watt_sampler(oracle):
    """b = 0 leaves the Maxwellian W: a Gamma(3/2, a) variate."""
    a = 0.988e6
    e = _watt_sample(oracle, a, 0.0, 40000, 13)
    assert stats.kstest(e, stats.gamma(1.5, scale=a).cdf).pvalue > 1e-3
    assert abs(e.mean() - 1.5 * a) < 4 * e.std() / math.sqrt(len(e))


def test_watt_spectrum_distribution(oracle):
    """Density proportional to exp(-E/a) sinh(sqrt(b E)); mean 3a/2 + a^2 b/4."""
    a, b = P.WATT_A, P.WATT_B
    e = _watt_sample(oracle, a, b, 40000, 14)
    assert np.all(e > 0)
    mean = 1.5 * a + a * a * b / 4
    assert abs(e.mean() - mean) < 4 * e.std() / math.sqrt(len(e))
    f = lambda x: math.exp(-x / a) * math.sinh(math.sqrt(b * x))
    top = 40 * a
    norm = integrate.quad(f, 0, top, limit=200)[0]
    grid = np.linspace(0, top, 4001)
    cdf_vals = np.concatenate([[0.0], np.cumsum([integrate.quad(f, grid[k], grid[k + 1])[0]
                                                 for k in range(len(grid) - 1)])]) / norm
    cdf = lambda x: np.interp(x, grid, cdf_vals)
    assert stats.kstest(e, cdf).pvalue > 1e-3


@pytest.mark.parametrize("awr", [1.0, 2.0, 12.0, 238.0])
def test_elastic_kinematics(oracle, awr):
    """Isotropic centre-of-mass scattering: E'/E uniform on [alpha, 1]
    (alpha = ((A-1)/(A+1))^2), mean lab cosine 2/(3A), and the two-body
    identity mu_lab = ((A+1) sqrt(E'/E) - (A-1) sqrt(E/E')) / 2."""
    rng = np.random.default_rng(15)
    xi = (rng.integers(0, 2**52, 20000).astype(np.float64) + 0.5) * 2.0**-52
    e0 = 1e6
    out = np.array([oracle.elastic(awr, e0, x) for x in xi])
    ratio, mu = out[:, 0] / e0, out[:, 1]
    alpha = ((awr - 1) / (awr + 1)) ** 2
    assert np.all(ratio >= alpha * (1 - 1e-12)) and np.all(ratio <= 1 + 1e-12)
    assert stats.kstest(ratio, stats.uniform(alpha, 1 - alpha).cdf).pvalue > 1e-3
    assert abs(mu.mean() - 2 / (3 * awr)) < 4 * mu.std() / math.sqrt(len(mu))
    ok = ratio > 1e-6
    ident = ((awr + 1) * np.sqrt(ratio[ok]) - (awr - 1) / np.sqrt(ratio[ok])) / 2
    assert np.allclose(mu[ok], ident, rtol=0, atol=1e-9)
    # the end points: forward (xi -> 1) keeps the energy, backward gives alpha
    assert oracle.elastic(awr, e0, 1.0)[0] == pytest.approx(e0, rel=1e-15)
    assert oracle.elastic(awr, e0, 0.0)[0] == pytest.approx(alpha * e0, rel=1e-12, abs=1e-9)


def test_rotation(oracle):
    """Unit norm, cosine to the old direction equal to mu, uniform azimuth,
    and the near-z branch."""
    rng = np.random.default_rng(16)
    phis = []
    for _ in range(3000):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        mu = rng.uniform(-1, 1)
        xi = rng.uniform()
        n = np.array(oracle.rotate(mu, xi, d))
        # 1 - w^2 loses relative accuracy eps / (1 - w^2) by cancellation
        tol = 1e-15 * (2 + 1 / (1 - d[2] ** 2))
        assert abs(np.linalg.norm(n) - 1) < tol
        assert abs(n @ d - mu) < tol
        # azimuth about d measured from a fixed perpendicular reference
        ref = np.cross(d, [0.0, 0.0, 1.0])
        ref /= np.linalg.norm(ref)
        ref2 = np.cross(d, ref)
        perp = n - (n @ d) * d
        if np.linalg.norm(perp) > 1e-8:
            phis.append(math.atan2(perp @ ref2, perp @ ref) % (2 * math.pi))
    assert stats.kstest(np.array(phis) / (2 * math.pi), "uniform").pvalue > 1e-3
    for w in (1.0, -1.0, math.sqrt(1 - 1e-11)):
        d = np.array([math.sqrt(max(0.0, 1 - w * w)), 0.0, w])
        for mu, xi in ((0.3, 0.1), (-0.7, 0.6), (1.0, 0.2)):
            n = np.array(oracle.rotate(mu, xi, d))
            assert abs(np.linalg.norm(n) - 1) < 1e-13
            assert abs(n @ d - mu) < 1e-12


def test_flat_infinite_medium_k(oracle):
    """Energy-independent cross sections in an infinite medium: k_inf =
    nu sigma_f / sigma_a whatever the slowing down (a heavy target, so no
    history reaches the cutoff); the absorption estimator is then exact in
    every generation."""
    ce = P.ce_flat(sig_s=8.0, sig_c=1.5, sig_f=1.0, awr=200.0, dens=0.05)
    prob = P.ce_homogeneous(ce, 4000, 12, 2, seed=21)
    r = oracle.run(prob)
    k_inf = P.NU_CE * 1.0 / 2.5
    km, ks = r["k_mean"], r["k_sigma"]
    for e in range(3):
        assert abs(km[e] - k_inf) < 4 * ks[e] + 1e-12, (e, km, ks)
    c = r["gen_counts"]
    assert np.all(c[:, 9] == 0)  # no cutoff
    # every absorption scores exactly nu sigma_f / sigma_a
    assert np.allclose(r["gen_k"][:, 2], k_inf, rtol=1e-12)


def test_pure_scatterer_slowing_down_to_cutoff(oracle):
    """Hydrogen-like target (A = 1), no absorption: ln(E/E') per collision is
    Exp(1), so the collisions from E0 to the cutoff number 1 + Poisson(L),
    L = ln(E0 / E_cut); every history ends at the cutoff."""
    ce = P.ce_flat(sig_s=10.0, sig_c=0.0, sig_f=0.0, awr=1.0, dens=0.1)
    n = 20000
    prob = P.ce_homogeneous(ce, n, 1, 0, seed=22, fixed_source=True)
    rng = np.random.default_rng(23)
    mu = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    s = np.sqrt(1 - mu * mu)
    e0 = 1e6
    ext = np.stack([rng.uniform(-1, 1, n) * 0.9 + 1.0, rng.uniform(-1, 1, n) * 0.9 + 1.0,
                    s * np.cos(phi), s * np.sin(phi), mu, np.full(n, e0)], axis=1)
    r = oracle.run(prob, ext_state=ext, records=True)
    c = r["gen_counts"][0]
    assert c[9] == n and c[5] == 0 and c[4] == 0
    L = math.log(e0 / ce["e_cut"])
    cols = r["records"][0]["n_col"].astype(float)
    assert abs(cols.mean() - (L + 1)) < 4 * math.sqrt(L / n)
    assert abs(cols.var() - L) < 0.1 * L
    assert np.all(r["records"][0]["e_final"] < ce["e_cut"])
    assert np.all(r["records"][0]["fate"] == 4)


def test_ce_pin_cell_balance_and_bank(oracle):
    """The continuous-energy pin cell: particle, event and site balance, and
    the bank size against k_col / k_used."""
    prob = P.ce_pin_cell(n_per_gen=3000, n_gen=4, n_inactive=1)
    r = oracle.run(prob, records=True, bank_cap=10000)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, *_ = r["gen_counts"].T
    assert np.all(ab + leak + killed + cut == n)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    assert np.all(killed == 0) and np.all(leak == 0)
    k_used = np.concatenate([[1.0], r["gen_k"][:-1, 0]])
    expect = n * r["gen_k"][:, 0] / k_used
    assert np.all(np.abs(sites - expect) < 4 * np.sqrt(col / 4.0) + 5)
    rec = r["records"]
    assert np.array_equal(rec["n_seg"].sum(1), seg)
    e = rec["e_final"]
    assert np.all((e > 0) & (e <= P.CE_E_MAX))
    bank = r["bank"]
    assert np.all((bank[:, 2] > 0) & (bank[:, 2] <= P.CE_E_MAX))


def test_ce_thread_count_does_not_change_results(oracle):
    prob = P.ce_pin_cell(n_per_gen=2500, n_gen=3, n_inactive=1)
    a = oracle.run(prob, n_threads=1, records=True, per_gen_tallies=True)
    b = oracle.run(prob, n_threads=6, records=True, per_gen_tallies=True)
    for k in ("gen_k", "gen_entropy", "gen_counts", "gen_flux", "records"):
        assert np.array_equal(a[k], b[k]), k
