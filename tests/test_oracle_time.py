"""Pins of the oracle's time-dependent fixed-source mode (Sec. 1 lists MC/DC's
fully time-dependent mode; here a source pulse at t = 0 with fission treated
as capture).  Closed forms: in an infinite medium the neutron density per
source particle obeys dn/dt = -A V n with A = diag(sig_t) - S^T and V the
group speeds, so the track length in the time bin [a, b] is
A^-1 (exp(-A V a) - exp(-A V b)) chi, and the census fraction at T is
1^T exp(-A V T) chi.  One group: (exp(-sig_a v a) - exp(-sig_a v b)) / sig_a.
"""
import math

import numpy as np
from scipy.linalg import expm

from paper_2501_05440_amd import problems as P


def time_flux(r, prob):
    """Flux per source particle summed over space: [group][time bin]."""
    nt = len(prob["time"]["t_edges"]) - 1
    g = prob["xs"]["sig_t"].shape[1]
    return (r["flux_mean"].reshape(-1, g, nt).sum(0), r["flux_sigma"].reshape(-1, g, nt))


def test_one_group_time_bins_and_census(oracle):
    xs = P.one_group(1.0, 0.3, 0.1)  # sig_a = 0.7 (fission counts as capture)
    v = 1.0e5
    edges = np.array([0.0, 1e-6, 3e-6, 1e-5, 3e-5])
    n, batches = 20000, 10
    prob = P.with_time(P.homogeneous(xs, n, batches, 0, seed=31, fixed_source=True), edges,
                       speed=[v])
    r = oracle.run(prob, records=True)
    fl, sg = time_flux(r, prob)
    sig = np.sqrt((sg ** 2).sum(0))[0]
    sa = 0.7
    want = (np.exp(-sa * v * edges[:-1]) - np.exp(-sa * v * edges[1:])) / sa
    assert np.all(np.abs(fl[0] - want) < 4 * sig + 1e-12), (fl[0], want, sig)
    cen = r["gen_counts"][:, 10].sum() / (n * batches)
    p = math.exp(-sa * v * edges[-1])
    assert abs(cen - p) < 4 * math.sqrt(p * (1 - p) / (n * batches))
    c = r["gen_counts"]
    assert np.all(c[:, 5] + c[:, 10] == n)  # absorbed or census
    rec = r["records"]
    t_max = edges[-1]
    assert np.all(rec["t_final"][rec["fate"] == 5] == t_max)
    assert np.all(rec["t_final"][rec["fate"] == 1] < t_max)
    assert np.all(rec["t_final"] > 0)


def test_multigroup_time_dependent_flux_matches_matrix_exponential(oracle):
    rng = np.random.default_rng(1000)
    fuel = P.mg_material(rng, fissile=True)
    edges = np.concatenate([[0.0], np.geomspace(1e-8, 2e-5, 7)])
    n, batches = 20000, 12
    prob = P.with_time(P.homogeneous(fuel, n, batches, 0, seed=32, fixed_source=True), edges)
    r = oracle.run(prob)
    fl, sg = time_flux(r, prob)
    sig = np.sqrt((sg ** 2).sum(0))
    st, ss, chi = fuel["sig_t"], fuel["sig_s"], fuel["chi"]
    V = np.diag(prob["time"]["speed"])
    A = np.diag(st) - ss.T
    Ainv = np.linalg.inv(A)
    E = [expm(-A @ V * t) @ chi for t in edges]
    want = np.stack([Ainv @ (E[k] - E[k + 1]) for k in range(len(edges) - 1)], axis=1)
    z = np.abs(fl - want) / np.maximum(sig, 1e-300)
    ok = want > 1e-6 * want.max()
    assert np.all(z[ok] < 4.5), np.max(z[ok])
    cen = r["gen_counts"][:, 10].sum() / (n * batches)
    p = float(E[-1].sum())
    assert abs(cen - p) < 4 * math.sqrt(p * (1 - p) / (n * batches)) + 1e-12


def test_time_dependent_lattice_balance_and_event_log(oracle):
    """Leakage and census together; the event log ends with a census entry
    exactly for the census histories."""
    prob = P.pulsed_lattice(n_per_gen=400, n_gen=2)
    cap = 2048
    r = oracle.run(prob, records=True, events=cap)
    n = prob["run"]["n_per_gen"]
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = r["gen_counts"].T
    assert np.all(ab + leak + killed + cut + cen == n)
    assert np.all(sites == 0)
    rec, ev = r["records"], r["events"]
    for g in range(rec.shape[0]):
        for h in range(n):
            k = int(rec[g, h]["n_seg"])
            assert (ev[g, h, k - 1]["type"] == 4) == (rec[g, h]["fate"] == 5)
            assert abs(ev[g, h, :k]["d"].sum() - rec[g, h]["tl_sum"]) <= 1e-12 * rec[g, h]["tl_sum"]


# ---------------------------------------------------------------------------
# continuous energy (the paper's time-dependent pin cell, Sec. 4): speed
# from the energy, neutron density tallied as time spent per bin
# ---------------------------------------------------------------------------

def test_neutron_speed_gives_back_the_kinetic_energy(oracle):
    """E = m v^2 / 2 with m c^2 = 939.56542052 MeV and c = 2.99792458e10 cm/s."""
    mc2, c = 939.56542052e6, 2.99792458e10
    for e in (1e-5, 0.0253, 1.0, 6.67e3, 1e6, 14e6, 2e7):
        v = oracle.speed(e)
        assert 0.5 * mc2 * (v / c) ** 2 == __import__("pytest").approx(e, rel=4e-16)
    # 2200 m/s at 0.0253 eV, the thermal reference speed
    assert abs(oracle.speed(0.0253) - 2.2e5) < 0.002 * 2.2e5


def ce_time_flat(sig_s, sig_c, sig_f, e0, edges, n, batches, seed, awr=1e12):
    """A continuous-energy infinite medium of one nuclide with flat cross
    sections and a target so heavy that scattering keeps the energy (and the
    speed): the one-group closed forms hold at v = speed(e0)."""
    ce = dict(P.ce_flat(sig_s, sig_c, sig_f, awr), src_energy=e0)
    prob = P.ce_homogeneous(ce, n, batches, 0, seed=seed, fixed_source=True)
    return P.with_time(prob, edges)


def test_ce_heavy_target_decay_matches_one_group_closed_form(oracle):
    e0 = 1.0e6
    sig_s, sig_c, sig_f = 3.0, 0.4, 0.1  # barns; density 1 atom / (b cm): 1/cm
    sa = sig_c + sig_f
    v = oracle.speed(e0)
    edges = np.array([0.0, 2e-10, 5e-10, 1e-9, 2e-9, 4e-9])
    n, batches = 20000, 10
    prob = ce_time_flat(sig_s, sig_c, sig_f, e0, edges, n, batches, seed=41)
    r = oracle.run(prob, records=True)
    nt = len(edges) - 1
    flux = r["flux_mean"].reshape(-1, nt).sum(0)
    fsig = np.sqrt((r["flux_sigma"].reshape(-1, nt) ** 2).sum(0))
    dens = r["prod_mean"].reshape(-1, nt).sum(0)
    dsig = np.sqrt((r["prod_sigma"].reshape(-1, nt) ** 2).sum(0))
    decay = np.exp(-sa * v * edges[:-1]) - np.exp(-sa * v * edges[1:])
    assert np.all(np.abs(flux - decay / sa) < 4 * fsig), (flux, decay / sa, fsig)
    assert np.all(np.abs(dens - decay / (sa * v)) < 4 * dsig), (dens, decay / (sa * v), dsig)
    # flux and density of a bin differ by the (constant) speed
    np.testing.assert_allclose(flux, v * dens, rtol=1e-9)
    cen = r["gen_counts"][:, 10].sum() / (n * batches)
    p = math.exp(-sa * v * edges[-1])
    assert abs(cen - p) < 4 * math.sqrt(p * (1 - p) / (n * batches))
    rec = r["records"]
    assert np.all(rec["t_final"][rec["fate"] == 5] == edges[-1])


def test_ce_density_sums_to_the_time_alive(oracle):
    """The density tally of a history adds up the time it spent before its
    end (census, absorption or cutoff), bin by bin: summed over every bin it
    equals the mean final time of the records, to rounding."""
    prob = P.ce_pulsed_pin_cell(n_per_gen=3000, n_gen=2)
    r = oracle.run(prob, records=True, per_gen_tallies=True, events=1)
    n = prob["run"]["n_per_gen"]
    for g in range(2):
        tot = r["gen_prod"][g].sum()
        want = r["records"][g]["t_final"].mean()
        assert abs(tot - want) <= 1e-12 * want, (tot, want)
    seg, col, cross, refl, leak, ab, killed, sites, scat, cut, cen = r["gen_counts"].T
    assert np.all(ab + leak + killed + cut + cen == n) and np.all(killed == 0)
    assert np.all(sites == 0)
    # every history starts at 14 MeV: the first flight's energy
    assert np.all(r["events"][:, :, 0]["e"] == P.SOURCE_14MEV)
    # a census ends exactly at the last time edge
    rec = r["records"]
    assert np.all(rec["t_final"][rec["fate"] == 5] == prob["time"]["t_edges"][-1])
    assert np.all(rec["t_final"][rec["fate"] != 5] < prob["time"]["t_edges"][-1])


def test_ce_with_a_monoenergetic_source_and_no_time_grid(oracle):
    """src_energy alone (no time grid): a fixed-source run whose histories
    all start at that energy, drawing no Watt numbers from the source stream."""
    ce = dict(P.ce_data(), src_energy=2.0e6)
    prob = P.with_run(P.ce_pin_cell(n_per_gen=500, n_gen=1, n_inactive=0, data=ce),
                      fixed_source=True)
    r = oracle.run(prob, events=1)
    assert np.all(r["events"][0, :, 0]["e"] == 2.0e6)
