"""Pins of whole oracle runs against closed forms and exact invariants.

Statistical checks use fixed seeds (each passes or fails reproducibly) and
compare with the run's own standard deviation.  Closed forms:

* one-group infinite medium: k = nu_sig_f / sig_a; collisions per history are
  geometric with mean sig_t / sig_a;
* multigroup infinite medium: k_inf = nu_sig_f^T A^-1 chi, A = diag(sig_t) -
  sig_s^T, and the track-length flux per source particle is A^-1 chi;
* a pin cell whose two regions hold the same material is an infinite medium,
  and its flux splits by region area;
* a reflective lattice of identical pins is the reflective single pin;
* pure-absorber slab transmission: exp(-tau) at normal incidence, E2(tau) for
  a uniform cosine, 2 E3(tau) for a cosine-weighted (isotropic-flux) source.
"""
import math

import numpy as np
import pytest
from scipy.special import expn

from paper_2501_05440_amd import problems as P


def z(x, mean, sigma):
    return abs(x - mean) / sigma


def fuel_of_pin_cell():
    xs = P.pin_cell()["xs"]
    return {k: v[0] for k, v in xs.items()}


def kinf(m):
    return P.mg_kinf(m["sig_t"], m["sig_s"], m["nu_sig_f"], m["chi"])


def group_flux(m):
    a = np.diag(m["sig_t"]) - m["sig_s"].T
    return np.linalg.solve(a, m["chi"])


def test_one_group_infinite_medium(oracle):
    mat = P.one_group(1.0, 0.6, 0.5)
    prob = P.homogeneous(mat, 20000, 25, 5, seed=11)
    r = oracle.run(prob)
    k_exact = 0.5 / 0.4
    for e in range(2):
        assert z(r["k_mean"][e], k_exact, r["k_sigma"][e]) < 3, (e, r["k_mean"], r["k_sigma"])
    # every history is absorbed once in a reflective one-group cell, scoring
    # nu_sig_f / sig_a: the absorption estimator has zero variance
    assert r["k_mean"][2] == pytest.approx(k_exact, rel=1e-14)
    assert r["k_sigma"][2] < 1e-13
    c = r["gen_counts"]
    n, g = prob["run"]["n_per_gen"], prob["run"]["n_gen"]
    # geometric number of collisions: mean sig_t / sig_a, variance (1 - p) / p^2
    p = 0.4
    mean_col = c[:, 1].sum() / (n * g)
    assert z(mean_col, 1 / p, math.sqrt((1 - p) / p**2 / (n * g))) < 3
    # each collision scores nu_sig_f / sig_t = 0.5 exactly
    np.testing.assert_allclose(r["gen_k"][:, 0], 0.5 * c[:, 1] / n, rtol=1e-13)
    # every history is absorbed (reflective cell)
    assert np.all(c[:, 5] == n) and np.all(c[:, 4] == 0)


def test_multigroup_infinite_medium_keff(oracle):
    fuel = fuel_of_pin_cell()
    k_exact = kinf(fuel)
    assert abs(k_exact - 1.2) < 1e-12
    r = oracle.run(P.homogeneous(fuel, 20000, 25, 5, seed=12))
    for e in range(3):
        assert z(r["k_mean"][e], k_exact, r["k_sigma"][e]) < 3, (e, r["k_mean"], r["k_sigma"])


def test_multigroup_fixed_source_flux_and_production(oracle):
    fuel = fuel_of_pin_cell()
    prob = P.homogeneous(fuel, 20000, 20, 0, seed=13, fixed_source=True)
    r = oracle.run(prob, per_gen_tallies=True)
    G = len(fuel["sig_t"])
    phi = group_flux(fuel)
    # bins of a one-cell, ring-less geometry: (region 0 or 1) x group; region 1 unused
    flux_g = r["gen_flux"].reshape(20, -1, G).sum(axis=1)
    prod_g = r["gen_prod"].reshape(20, -1, G).sum(axis=1)
    m, s = flux_g.mean(axis=0), flux_g.std(axis=0, ddof=1) / math.sqrt(20)
    for g in range(G):
        assert z(m[g], phi[g], s[g]) < 4, (g, m[g], phi[g], s[g])
    tot = prod_g.sum(axis=1)
    assert z(tot.mean(), float(fuel["nu_sig_f"] @ phi), tot.std(ddof=1) / math.sqrt(20)) < 3
    # no fission banking in fixed-source mode
    assert np.all(r["gen_counts"][:, 7] == 0)


def test_pin_cell_of_one_material_is_infinite_medium(oracle):
    fuel = fuel_of_pin_cell()
    prob = P.pin_cell_same_material(fuel, 20000, 25, 5, seed=14)
    r = oracle.run(prob, per_gen_tallies=True)
    assert z(r["k_mean"][0], kinf(fuel), r["k_sigma"][0]) < 3
    # flux splits by region area: region 0 is the disc of radius 0.54
    G = len(fuel["sig_t"])
    fl = r["gen_flux"][5:].reshape(20, 2, G).sum(axis=2)
    frac = fl[:, 0] / fl.sum(axis=1)
    area = math.pi * 0.54**2 / 1.26**2
    assert z(frac.mean(), area, frac.std(ddof=1) / math.sqrt(len(frac))) < 3
    # the total flux per source particle is the infinite-medium one
    tot = fl.sum(axis=1)
    assert z(tot.mean(), group_flux(fuel).sum(), tot.std(ddof=1) / math.sqrt(len(tot))) < 3


def test_reflective_lattice_equals_single_pin(oracle):
    base = P.pin_cell(n_per_gen=20000, n_gen=25, n_inactive=5, seed=15)
    r1 = oracle.run(base)
    geo = P.lattice_geometry(3, 3, P.PIN_PITCH, [([P.PIN_RADIUS], [0, 1])],
                             np.zeros((3, 3), int), [P.REFLECT] * 4)
    lat = P.make_problem("lattice3", geo, base["xs"], dict(base["run"], seed=16))
    r3 = oracle.run(lat)
    d = r1["k_mean"][0] - r3["k_mean"][0]
    s = math.hypot(r1["k_sigma"][0], r3["k_sigma"][0])
    assert abs(d) < 3 * s, (r1["k_mean"], r3["k_mean"], s)


@pytest.mark.parametrize("mode", ["normal", "uniform_cosine", "cosine_weighted"])
def test_pure_absorber_slab(oracle, mode):
    sig_t, L, n = 1.0, 1.5, 100000
    tau = sig_t * L
    rng = np.random.default_rng({"normal": 1, "uniform_cosine": 2, "cosine_weighted": 3}[mode])
    if mode == "normal":
        mu = np.ones(n)
        t_exact = math.exp(-tau)
        tl_exact = (1 - math.exp(-tau)) / sig_t
    elif mode == "uniform_cosine":
        mu = 1.0 - rng.uniform(size=n)  # (0, 1]
        t_exact = expn(2, tau)
        tl_exact = None
    else:
        mu = np.sqrt(1.0 - rng.uniform(size=n))
        t_exact = 2 * expn(3, tau)
        tl_exact = None
    phi = rng.uniform(0, 2 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1 - mu * mu))
    st = np.zeros((n, 6))
    st[:, 0] = 0.0
    st[:, 1] = 0.0
    st[:, 2] = mu
    st[:, 3] = s * np.cos(phi)
    st[:, 4] = s * np.sin(phi)
    prob = P.slab(L, sig_t, n, seed=17)
    r = oracle.run(prob, records=True, ext_state=st)
    rec = r["records"][0]
    leaked = rec["fate"] == 2
    # a pure absorber leaks only through the far face
    assert np.all(np.abs(rec["x_final"][leaked] - L) < 1e-12)
    assert np.all(rec["fate"][~leaked] == 1)
    frac = leaked.mean()
    assert z(frac, t_exact, math.sqrt(t_exact * (1 - t_exact) / n)) < 3, (frac, t_exact)
    if tl_exact is not None:
        tl = rec["tl_sum"]
        assert z(tl.mean(), tl_exact, tl.std() / math.sqrt(n)) < 3


def _c0(n=10000, gens=30, inactive=10):
    return P.pin_cell(n_per_gen=n, n_gen=gens, n_inactive=inactive)


def test_balance_and_records(oracle):
    prob = _c0(5000, 8, 2)
    r = oracle.run(prob, records=True, per_gen_tallies=True)
    n = prob["run"]["n_per_gen"]
    c = r["gen_counts"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cutoff, *_ = c.T
    assert np.all(ab + leak + killed == n)
    assert np.all(killed == 0)
    assert np.all(col == scat + ab)
    assert np.all(seg == col + cross)
    rec = r["records"]
    assert np.array_equal(rec["n_seg"].sum(axis=1), seg)
    assert np.array_equal(rec["n_col"].sum(axis=1), col)
    assert np.array_equal(rec["n_sites"].sum(axis=1), sites)
    assert np.array_equal(rec["n_refl"].sum(axis=1), refl)
    # per-history sums agree with the generation estimators
    np.testing.assert_allclose(rec["kcol_sum"].sum(axis=1) / n, r["gen_k"][:, 0], rtol=1e-12)
    np.testing.assert_allclose(rec["tl_sum"].sum(axis=1) / n, r["gen_flux"].sum(axis=1),
                               rtol=1e-12)
    # draws: 2 for the birth direction, 1 per segment, 1 per collision for the
    # scatter test, 3 per scatter, 1 per banked site, plus one fission draw per
    # collision in the fuel
    n_scat = rec["n_col"] - (rec["fate"] == 1)
    base = 2 + rec["n_seg"] + rec["n_col"] + 3 * n_scat + rec["n_sites"]
    extra = rec["ctr_final"].astype(np.int64) - base
    assert np.all(extra >= 0) and np.all(extra <= rec["n_col"])
    # the reflective pin cell never leaks; every history ends absorbed
    assert np.all(rec["fate"] == 1)


def test_thread_count_independence(oracle):
    prob = _c0(3000, 6, 2)
    a = oracle.run(prob, n_threads=1, records=True, per_gen_tallies=True)
    b = oracle.run(prob, n_threads=7, records=True, per_gen_tallies=True)
    for k in ("gen_k", "gen_entropy", "gen_counts", "gen_flux", "gen_prod", "records"):
        assert np.array_equal(a[k], b[k]), k


def test_estimators_agree(oracle):
    r = oracle.run(_c0())
    km, ks = r["k_mean"], r["k_sigma"]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(km[a] - km[b]) < 3 * math.hypot(ks[a], ks[b]), (km, ks)


def test_d4_symmetry(oracle):
    # 5x5 vacuum lattice with a D4-symmetric pin map
    n = 5
    ii, jj = np.meshgrid(np.arange(n), np.arange(n))
    ring = np.minimum(np.minimum(ii, n - 1 - ii), np.minimum(jj, n - 1 - jj))
    pin_map = (ring % 3).astype(int)
    # fixed-source batches are independent, so the batch spread is an honest
    # standard deviation (power-iteration generations are correlated)
    base = P.lattice_17x17(n_per_gen=20000, n_gen=20, n_inactive=0, seed=18)
    geo = P.lattice_geometry(n, n, P.PIN_PITCH, [([P.PIN_RADIUS], [f, 3]) for f in range(3)],
                             pin_map, [P.VACUUM] * 4)
    prob = P.make_problem("d4", geo, base["xs"],
                          dict(base["run"], ent_nx=5, ent_ny=5, fixed_source=True))
    r = oracle.run(prob)
    G = prob["xs"]["sig_t"].shape[1]
    pin = r["flux_mean"].reshape(n, n, 2 * G).sum(axis=2)
    sig = np.sqrt((r["flux_sigma"].reshape(n, n, 2 * G) ** 2).sum(axis=2))
    for j in range(n):
        for i in range(n):
            orbit = {(j, i), (i, j), (j, n - 1 - i), (n - 1 - i, j), (n - 1 - j, i),
                     (i, n - 1 - j), (n - 1 - j, n - 1 - i), (n - 1 - i, n - 1 - j)}
            vals = [pin[a, b] for a, b in orbit]
            m = np.mean(vals)
            assert abs(pin[j, i] - m) < 4 * sig[j, i], (j, i, pin[j, i], m, sig[j, i])


def test_event_guard_kills(oracle):
    prob = P.with_run(_c0(2000, 3, 1), max_events=3)
    r = oracle.run(prob, records=True)
    c = r["gen_counts"]
    assert np.all(c[:, 6] > 0)
    assert np.all(c[:, 4] + c[:, 5] + c[:, 6] == 2000)
    rec = r["records"]
    assert np.all(rec["n_seg"] <= 3)
    killed = rec["fate"] == 3
    assert np.all(rec["n_seg"][killed] == 3)
    assert not np.any(killed & (rec["n_seg"] < 3))


def test_extinct_population_is_an_error(oracle):
    fuel = fuel_of_pin_cell()
    fuel = dict(fuel, nu_sig_f=fuel["nu_sig_f"] * 1e-12)
    prob = P.homogeneous(fuel, 50, 3, 1, seed=19)
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(prob)
    assert e.value.code == -7


@pytest.mark.parametrize("bad", ["neg_xs", "radius", "pin_map"])
def test_invalid_inputs(oracle, bad):
    prob = _c0(100, 2, 1)
    if bad == "neg_xs":
        xs = dict(prob["xs"])
        xs["sig_t"] = xs["sig_t"].copy()
        xs["sig_t"][1, 2] = -1.0
        prob = dict(prob, xs=xs)
    elif bad == "radius":
        geo = dict(prob["geometry"])
        geo["radii"] = np.array([[0.7]])
        prob = dict(prob, geometry=geo)
    else:
        geo = dict(prob["geometry"])
        geo["pin_map"] = np.array([[3]], np.int32)
        prob = dict(prob, geometry=geo)
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(prob)
    assert e.value.code == -1


def test_fission_bank_size_follows_k_used(oracle):
    # conditional on the collisions, each banks floor(nu_sig_f / (sig_t k_used) + xi)
    # sites, whose mean is nu_sig_f / (sig_t k_used): M_g - N k_col,g / k_used,g is a
    # sum of independent zero-mean terms of variance <= 1/4 per fissile collision
    prob = _c0(20000, 6, 1)
    r = oracle.run(prob)
    n = prob["run"]["n_per_gen"]
    k_used = np.concatenate([[1.0], r["gen_k"][:-1, 0]])
    m = r["gen_counts"][:, 7]
    expect = n * r["gen_k"][:, 0] / k_used
    bound = 4 * np.sqrt(r["gen_counts"][:, 1] / 4.0)
    assert np.all(np.abs(m - expect) < bound), (m, expect, bound)


def test_event_log_is_consistent_with_records(oracle):
    """The per-flight event log of the oracle: as many flights as the record
    counts, flight lengths summing to the track length, one collision entry
    per collision, the last entry at the final position, leaks only last,
    and consecutive flights in the same or a neighbouring lattice cell."""
    for prob in (P.lattice_17x17(n_per_gen=300, n_gen=2, n_inactive=1),
                 P.ce_pin_cell(n_per_gen=200, n_gen=2, n_inactive=1)):
        cap = 4096
        r = oracle.run(prob, records=True, events=cap)
        ev, rec = r["events"], r["records"]
        nx = prob["geometry"]["nx"]
        for g in range(ev.shape[0]):
            for h in range(ev.shape[1]):
                rh = rec[g, h]
                n = int(rh["n_seg"])
                assert n <= cap
                e = ev[g, h, :n]
                assert np.all(ev[g, h, n:]["type"] == 0)
                assert np.all(e["type"] > 0)
                assert abs(e["d"].sum() - rh["tl_sum"]) <= 1e-12 * rh["tl_sum"]
                assert int((e["type"] == 1).sum()) == rh["n_col"]
                assert int((e["type"] != 1).sum()) == rh["n_cross"]
                assert e[-1]["x"] == rh["x_final"] and e[-1]["y"] == rh["y_final"]
                assert np.all(e[:-1]["type"] != 3)
                assert (e[-1]["type"] == 3) == (rh["fate"] == 2)
                ci, cj = e["cell"] % nx, e["cell"] // nx
                assert np.all(np.abs(np.diff(ci)) <= 1) and np.all(np.abs(np.diff(cj)) <= 1)
