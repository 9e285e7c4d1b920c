"""Pins of four oracle parts that the closed-form physics tests do not reach.

* source acceptance (Sec. 1, k-eigenvalue power iteration: the first
  generation is spread over the fissile volume): every generation-0 site lies
  in a fissile region, the sites are uniform in area there, their count per
  fissile region follows its area, and their group follows the fission
  spectrum of the material they sit in;
* the standard deviation of the active-generation mean: z-scores of whole
  runs against closed forms have the spread of a Student t with A - 1
  degrees of freedom (a sigma without the 1/sqrt(A), or of the wrong kind,
  fails it);
* the Shannon-entropy mesh binning: meshes aligned with fissile pins give
  exactly known entropies (0 when every site falls in one bin, 1 or 2 bits
  for symmetric splits, log2 B for a uniform medium), and transposing x and
  y changes them;
* the corner rule of the surface crossing (every plane hit at the boundary
  distance is crossed in the same event; any vacuum outer side crossed
  leaks, otherwise every crossed outer side reflects): rays aimed exactly at
  lattice corners with mixed vacuum and reflective sides end as computed by
  hand.
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2501_05440_amd import problems as P


def _mat(seed, fissile=True):
    return P.mg_material(np.random.default_rng(seed), fissile=fissile)


# ---------------------------------------------------------------------------
# source acceptance
# ---------------------------------------------------------------------------

def _cell_centres(geo, x, y):
    i = np.floor((x - geo["x0"]) / geo["pitch"]).astype(int)
    j = np.floor((y - geo["y0"]) / geo["pitch"]).astype(int)
    cx = geo["x0"] + (i + 0.5) * geo["pitch"]
    cy = geo["y0"] + (j + 0.5) * geo["pitch"]
    return i, j, x - cx, y - cy


def test_pin_cell_source_is_uniform_over_the_fuel_disc(oracle):
    prob = P.pin_cell(n_per_gen=40000, n_gen=1, n_inactive=0)
    s = oracle.run(prob, source=True)["source"][0]
    geo = prob["geometry"]
    _, _, dx, dy = _cell_centres(geo, s[:, 0], s[:, 1])
    rr = dx * dx + dy * dy
    R = P.PIN_RADIUS
    assert np.all(rr < R * R), "a source site outside the fuel disc"
    # uniform in area: (r / R)^2 is uniform on [0, 1); the angle is uniform
    cnt, _ = np.histogram(rr / (R * R), bins=20, range=(0.0, 1.0))
    assert stats.chisquare(cnt).pvalue > 1e-3
    cnt, _ = np.histogram(np.arctan2(dy, dx), bins=16, range=(-math.pi, math.pi))
    assert stats.chisquare(cnt).pvalue > 1e-3
    # the group follows the fuel's fission spectrum
    chi = prob["xs"]["chi"][0]
    obs = np.bincount(s[:, 2].astype(int), minlength=len(chi))
    nz = chi > 0
    assert np.all(obs[~nz] == 0)
    assert stats.chisquare(obs[nz], chi[nz] / chi[nz].sum() * len(s)).pvalue > 1e-3


def test_lattice_source_fills_every_pin_equally(oracle):
    prob = P.lattice_17x17(n_per_gen=289 * 150, n_gen=1, n_inactive=0)
    s = oracle.run(prob, source=True)["source"][0]
    geo = prob["geometry"]
    i, j, dx, dy = _cell_centres(geo, s[:, 0], s[:, 1])
    assert np.all(dx * dx + dy * dy < P.PIN_RADIUS ** 2)
    cnt = np.bincount(j * 17 + i, minlength=289)
    assert stats.chisquare(cnt).pvalue > 1e-3


def test_source_only_in_fissile_regions_of_mixed_pins(oracle):
    """2x2 lattice: a standard pin (fuel 1 inside the ring), a pin of
    moderator only, and an inverted pin (moderator inside, fuel 2 outside).
    Sites appear only in fissile regions, in proportion to their areas, with
    the group spectrum of the fuel they sit in."""
    f1, mod, f2 = _mat(11), _mat(12, fissile=False), _mat(13)
    # make the two spectra clearly different
    f2 = dict(f2, chi=np.array([0.1, 0.2, 0.7, 0, 0, 0, 0]))
    f1 = dict(f1, chi=np.array([0.7, 0.2, 0.1, 0, 0, 0, 0]))
    R = 0.5
    univ = [([R], [0, 1]), ([R], [1, 1]), ([R], [1, 2])]
    pin_map = [[0, 1], [2, 0]]  # row j = 0: (0, 1); row j = 1: (2, 0)
    geo = P.lattice_geometry(2, 2, P.PIN_PITCH, univ, pin_map, [P.REFLECT] * 4)
    N = 60000
    prob = P.make_problem("mixed", geo, P.stack_materials([f1, mod, f2]),
                          P.run_params(21, N, 1, 0, ent=(2, 2)))
    s = oracle.run(prob, source=True)["source"][0]
    i, j, dx, dy = _cell_centres(geo, s[:, 0], s[:, 1])
    inside = dx * dx + dy * dy < R * R
    univ_of = np.asarray(pin_map)[j, i]
    # moderator-only pin: nothing; standard pins: inside only; inverted: outside only
    assert not np.any(univ_of == 1)
    assert np.all(inside[univ_of == 0])
    assert not np.any(inside[univ_of == 2])
    # counts follow the fissile areas: two discs and one square minus a disc
    a_in = math.pi * R * R
    a_out = P.PIN_PITCH ** 2 - a_in
    p_out = a_out / (2 * a_in + a_out)
    n_out = int(np.sum(univ_of == 2))
    assert abs(n_out - N * p_out) < 4 * math.sqrt(N * p_out * (1 - p_out))
    # the two standard pins share their sites evenly
    n00 = int(np.sum((univ_of == 0) & (j == 0)))
    n_std = int(np.sum(univ_of == 0))
    assert abs(n00 - n_std / 2) < 4 * math.sqrt(n_std / 4)
    # groups follow the spectrum of the material at the site
    for sel, chi in ((univ_of == 0, f1["chi"]), (univ_of == 2, f2["chi"])):
        obs = np.bincount(s[sel, 2].astype(int), minlength=7)
        assert np.all(obs[3:] == 0)
        assert stats.chisquare(obs[:3], chi[:3] * sel.sum()).pvalue > 1e-3


# ---------------------------------------------------------------------------
# standard deviation of the active mean
# ---------------------------------------------------------------------------

def _t_ks(z, dof):
    return stats.kstest(z, stats.t(dof).cdf).pvalue


def test_sigma_of_the_mean_has_student_t_coverage_fixed_source(oracle):
    """Fixed-source one-group infinite medium: the flux per source particle
    is 1 / sig_a (the small nu_sig_f only makes the medium a source region;
    fission is capture here).  Over many independent runs of A batches,
    (mean - exact) / sigma follows Student's t with A - 1 degrees of freedom."""
    mat = P.one_group(1.0, 0.6, 0.1)
    A, n = 10, 600
    z = []
    for k in range(200):
        prob = P.homogeneous(mat, n, A, 0, seed=50000 + k, fixed_source=True)
        r = oracle.run(prob, n_threads=2)
        z.append((r["flux_mean"].sum() - 1.0 / 0.4) / math.sqrt((r["flux_sigma"] ** 2).sum()))
    z = np.array(z)
    assert _t_ks(z, A - 1) > 1e-3, z
    # the test has the power to see a sigma without 1/sqrt(A) or with an
    # extra one
    assert _t_ks(z * math.sqrt(A), A - 1) < 1e-6
    assert _t_ks(z / math.sqrt(A), A - 1) < 1e-6


def test_sigma_of_the_mean_has_student_t_coverage_keff(oracle):
    """k-eigenvalue one-group infinite medium: every estimator's generation
    values are independent draws around nu_sig_f / sig_a = 1.25 (no spatial
    dependence), so the active mean's z-score follows Student's t."""
    mat = P.one_group(1.0, 0.6, 0.5)
    ng, ni = 12, 2
    z = []
    for k in range(200):
        prob = P.homogeneous(mat, 500, ng, ni, seed=60000 + k)
        r = oracle.run(prob, n_threads=2)
        z.append((r["k_mean"][0] - 1.25) / r["k_sigma"][0])
    z = np.array(z)
    assert _t_ks(z, ng - ni - 1) > 1e-3, z
    assert _t_ks(z * math.sqrt(ng - ni), ng - ni - 1) < 1e-6


def test_sigma_is_over_the_active_generations_only(oracle):
    """The reported mean and sigma cover generations n_inactive .. n_gen - 1:
    a run whose inactive generations hold a different k (the first one is
    banked with k_used = 1) still has every z within the spread above, and
    the sigma matches the active values (sample standard deviation of the
    mean, the definition the coverage tests pin)."""
    prob = P.pin_cell(n_per_gen=2000, n_gen=12, n_inactive=4)
    r = oracle.run(prob, per_gen_tallies=True)
    act = r["gen_k"][4:]
    np.testing.assert_allclose(r["k_mean"], act.mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(r["k_sigma"], act.std(axis=0, ddof=1) / math.sqrt(8), rtol=1e-12)
    f = r["gen_flux"][4:]
    np.testing.assert_allclose(r["flux_sigma"], f.std(axis=0, ddof=1) / math.sqrt(8),
                               rtol=1e-10, atol=1e-300)


# ---------------------------------------------------------------------------
# entropy mesh binning
# ---------------------------------------------------------------------------

def test_entropy_of_a_uniform_medium_is_log2_bins(oracle):
    """Fission sites of a homogeneous reflective medium are uniform over the
    cell: H = log2(64) up to the multinomial deficit, about (B - 1) / (2 M ln 2)
    times the clustering of sites from one history."""
    mat = P.one_group(1.0, 0.6, 0.5)
    prob = P.homogeneous(mat, 100000, 3, 1, seed=71)
    prob["run"].update(ent_nx=8, ent_ny=8)
    r = oracle.run(prob)
    deficit = 6.0 - r["gen_entropy"]
    M = r["gen_counts"][:, 7]
    assert np.all(deficit > 0), deficit
    assert np.all(deficit < 10 * 63 / (2 * M * math.log(2))), (deficit, M)


def _row_lattice(fissile_col, ent, bc=None):
    """3 x 1 lattice of r = 0.54 pins: only the pin in column fissile_col
    has fuel; the others hold moderator in both regions."""
    fuel, mod = _mat(31), _mat(32, fissile=False)
    univ = [([P.PIN_RADIUS], [0, 1]), ([P.PIN_RADIUS], [1, 1])]
    pin_map = [[0 if c == fissile_col else 1 for c in range(3)]]
    geo = P.lattice_geometry(3, 1, P.PIN_PITCH, univ, pin_map, bc or [P.REFLECT] * 4)
    return P.make_problem("row", geo, P.stack_materials([fuel, mod]),
                          P.run_params(33, 20000, 3, 1, ent=ent))


def test_entropy_mesh_aligned_with_the_only_fissile_pin_is_zero(oracle):
    for col in range(3):
        r = oracle.run(_row_lattice(col, (3, 1)))
        assert np.all(r["gen_entropy"] == 0.0), (col, r["gen_entropy"])
        # one bin over the whole lattice: 0 as well
        r = oracle.run(_row_lattice(col, (1, 1)))
        assert np.all(r["gen_entropy"] == 0.0)


def test_entropy_mesh_halving_the_fissile_pin_is_one_bit(oracle):
    """A 6 x 1 mesh puts the middle pin's disc into two bins split at its
    centre line; the reflective row is symmetric about that line, so each
    bin holds half the sites."""
    r = oracle.run(_row_lattice(1, (6, 1)))
    M = r["gen_counts"][:, 7]
    # 1 - H = 2 / ln 2 (p - 1/2)^2 to leading order, p - 1/2 ~ 1 / (2 sqrt M)
    assert np.all(r["gen_entropy"] <= 1.0 + 1e-12)
    assert np.all(1.0 - r["gen_entropy"] < 25 * 2 / math.log(2) / (4 * M)), r["gen_entropy"]


def test_entropy_mesh_is_not_transposed(oracle):
    """A 1 x 3 mesh cuts the same row lattice along y: every bin is crossed
    by the fuel disc, so the entropy is far from 0; the 3 x 1 mesh (x cuts)
    gives exactly 0."""
    r = oracle.run(_row_lattice(0, (1, 3)))
    assert np.all(r["gen_entropy"] > 1.2), r["gen_entropy"]
    assert np.all(r["gen_entropy"] <= math.log2(3) + 1e-12)


def test_entropy_of_a_thin_pin_on_a_4x4_mesh_is_two_bits(oracle):
    """A fuel disc of radius 0.3 < pitch / 4 lies inside the four central
    bins of a 4 x 4 mesh and is shared evenly between them (D4 symmetry of a
    reflective pin cell): H = 2 bits up to the multinomial deficit."""
    fuel, mod = _mat(41), _mat(42, fissile=False)
    geo = P.lattice_geometry(1, 1, P.PIN_PITCH, [([0.3], [0, 1])], [[0]], [P.REFLECT] * 4)
    prob = P.make_problem("thin", geo, P.stack_materials([fuel, mod]),
                          P.run_params(43, 40000, 3, 1, ent=(4, 4)))
    r = oracle.run(prob)
    M = r["gen_counts"][:, 7]
    d = 2.0 - r["gen_entropy"]
    assert np.all(d >= -1e-12)
    assert np.all(d < 25 * 3 / (2 * M * math.log(2))), (d, M)


# ---------------------------------------------------------------------------
# corner crossings with mixed boundary conditions
# ---------------------------------------------------------------------------

V, R_ = P.VACUUM, P.REFLECT


def _corner_run(oracle, nx, ny, bc, starts, max_events=100000):
    """Fixed-source runs of a ring-less nx x ny lattice of a near-void
    material (no collision within the cells) from explicit start states."""
    geo = P.lattice_geometry(nx, ny, P.PIN_PITCH, [([], [0])], np.zeros((ny, nx), int), bc)
    xs = P.stack_materials([P.one_group(1e-9, 0.0, 0.0)])
    prob = P.make_problem("corner", geo, xs,
                          P.run_params(81, len(starts), 1, 0, fixed_source=True, ent=(1, 1),
                                       max_events=max_events))
    st = np.zeros((len(starts), 6))
    for k, (x, y, u, v) in enumerate(starts):
        st[k] = (x, y, u, v, math.sqrt(1.0 - u * u - v * v), 0)
    r = oracle.run(prob, ext_state=st, records=True, events=4)
    return geo, r["records"][0], r["events"][0]


A = 0.6  # in-plane direction components: u = v exactly, so the two plane distances tie


def test_corner_with_one_vacuum_side_leaks(oracle):
    # 1 x 1 cell centred on the origin, ray to the (xmax, ymax) corner
    for bc in ([R_, V, R_, R_], [R_, R_, R_, V], [R_, V, R_, V]):
        _, rec, ev = _corner_run(oracle, 1, 1, bc, [(0.0, 0.0, A, A)])
        assert rec["fate"][0] == 2 and rec["n_cross"][0] == 1 and rec["n_refl"][0] == 0, bc
        assert ev[0, 0]["type"] == 3
        assert rec["x_final"][0] == pytest.approx(0.63, abs=1e-12)
        assert rec["y_final"][0] == pytest.approx(0.63, abs=1e-12)


def test_reflective_corner_reflects_both_sides(oracle):
    # (xmax, ymax) reflective on both sides: the ray comes straight back to
    # the opposite corner, whose x side is vacuum
    _, rec, ev = _corner_run(oracle, 1, 1, [V, R_, R_, R_], [(0.0, 0.0, A, A)])
    assert rec["fate"][0] == 2
    assert rec["n_cross"][0] == 2 and rec["n_refl"][0] == 1 and rec["n_seg"][0] == 2
    assert list(ev[0, :2]["type"]) == [2, 3]
    # corner to corner: in-plane length 1.26 sqrt(2) at in-plane speed A sqrt(2)
    assert ev[0, 1]["d"] == pytest.approx(1.26 / A, rel=1e-12)
    assert rec["x_final"][0] == pytest.approx(-0.63, abs=1e-12)
    assert rec["y_final"][0] == pytest.approx(-0.63, abs=1e-12)


def test_all_reflective_corners_bounce_until_the_guard(oracle):
    _, rec, _ = _corner_run(oracle, 1, 1, [R_] * 4, [(0.0, 0.0, A, A)], max_events=50)
    assert rec["fate"][0] == 3
    assert rec["n_seg"][0] == 50 and rec["n_cross"][0] == 50 and rec["n_refl"][0] == 50


def test_interior_corner_steps_diagonally(oracle):
    # 2 x 2 lattice: from the centre of cell (0, 0) through the shared corner
    # into cell (1, 1), then out through its vacuum (xmax, ymax) corner
    _, rec, ev = _corner_run(oracle, 2, 2, [R_, V, R_, R_], [(-0.63, -0.63, A, A)])
    assert rec["fate"][0] == 2 and rec["n_cross"][0] == 2 and rec["n_refl"][0] == 0
    assert list(ev[0, :2]["cell"]) == [0, 3]
    assert list(ev[0, :2]["type"]) == [2, 3]


def test_corner_of_an_inner_face_and_an_outer_side(oracle):
    # 2 x 1 lattice: the first corner joins the inner x face and the
    # reflective top side (step right and reflect v in one event); the second
    # is cell (1, 0)'s (xmax, ymin) corner, whose y side is vacuum
    _, rec, ev = _corner_run(oracle, 2, 1, [R_, R_, V, R_], [(-0.63, 0.0, A, A)])
    assert rec["fate"][0] == 2 and rec["n_cross"][0] == 2 and rec["n_refl"][0] == 1
    assert list(ev[0, :2]["cell"]) == [0, 1]
    assert list(ev[0, :2]["type"]) == [2, 3]
    assert rec["x_final"][0] == pytest.approx(1.26, abs=1e-12)
    assert rec["y_final"][0] == pytest.approx(-0.63, abs=1e-12)
    # with a vacuum top side the first corner already leaks
    _, rec, _ = _corner_run(oracle, 2, 1, [R_, R_, R_, V], [(-0.63, 0.0, A, A)])
    assert rec["fate"][0] == 2 and rec["n_cross"][0] == 1 and rec["n_refl"][0] == 0
