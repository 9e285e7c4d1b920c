"""Seeded synthetic problem generators.

This module builds the inputs that both the HIP transport path and the CPU
oracle consume: lattice geometry, multigroup cross sections and run
parameters.  It holds none of the transport arithmetic (no sampling, no
tracking, no estimators); it only draws problem data from numpy generators
with fixed seeds.

The paper's workloads (a 3D C5G7 multigroup k-eigenvalue benchmark and an
OpenMC-data continuous-energy pin cell; Sec. 4) need data that is not
available here.  The problems below are synthetic stand-ins with the same
shapes: a 7-group pin cell, a 17x17 lattice of such pins, a batch of small
fixed-source pin cells, plus closed-form test problems (homogeneous media,
a pure-absorber slab).

A problem is a plain dict:

    geometry:  nx, ny, pitch, x0, y0, bc[4] (xmin, xmax, ymin, ymax;
               0 = vacuum, 1 = reflective), n_rings[n_univ],
               radii[n_univ, max_rings], mats[n_univ, max_rings + 1],
               pin_map[ny, nx]
    xs:        sig_t[M, G], sig_s[M, G, G] (row g = scatter out of group g),
               nu_sig_f[M, G], chi[M, G]
    run:       seed, n_per_gen, n_gen, n_inactive, fixed_source, problem_id,
               ent_nx, ent_ny, max_events
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

VACUUM = 0
REFLECT = 1

PIN_PITCH = 1.26
PIN_RADIUS = 0.54
N_GROUPS = 7


# ---------------------------------------------------------------------------
# cross sections
# ---------------------------------------------------------------------------

def _removal_matrix(sig_t, sig_s):
    """diag(sig_t) - sig_s^T: the infinite-medium group balance operator."""
    return np.diag(sig_t) - sig_s.T


def mg_kinf(sig_t, sig_s, nu_sig_f, chi):
    """Infinite-medium multiplication of one material, nu_sig_f^T A^-1 chi.

    Used here only to scale generated fuels to a target k_inf; it is the
    dominant (and only nonzero) eigenvalue of the rank-one fission operator.
    """
    a = _removal_matrix(np.asarray(sig_t, float), np.asarray(sig_s, float))
    return float(np.asarray(nu_sig_f, float) @ np.linalg.solve(a, np.asarray(chi, float)))


def mg_material(rng, n_groups=N_GROUPS, fissile=True, k_target=1.2):
    """One synthetic multigroup material.

    total XS ~ U[0.2, 1.5]/cm per group; scattering ratio ~ U[0.5, 0.95];
    the out-scatter of group g is spread over groups g' >= g with U[0,1]
    weights (last group: self-scatter only).  Fissile materials get a fission
    spectrum in the first three groups and nu_sig_f = r_g * sig_a_g with
    r_g ~ U[0.5, 1.5], rescaled so that the material's own k_inf equals
    k_target; draws are repeated while any nu_sig_f_g exceeds 2.5 sig_a_g.
    """
    g_n = n_groups
    sig_t = rng.uniform(0.2, 1.5, g_n)
    ratio = rng.uniform(0.5, 0.95, g_n)
    sig_s = np.zeros((g_n, g_n))
    for g in range(g_n):
        if g == g_n - 1:
            w = np.ones(1)
        else:
            w = rng.uniform(0.0, 1.0, g_n - g)
        sig_s[g, g:] = ratio[g] * sig_t[g] * w / w.sum()
    sig_a = sig_t - sig_s.sum(axis=1)
    chi = np.zeros(g_n)
    nu_sig_f = np.zeros(g_n)
    if fissile:
        n_chi = min(3, g_n)
        chi[:n_chi] = rng.uniform(0.0, 1.0, n_chi)
        chi /= chi.sum()
        for _ in range(1000):
            r = rng.uniform(0.5, 1.5, g_n)
            nu_sig_f = r * sig_a
            nu_sig_f *= k_target / mg_kinf(sig_t, sig_s, nu_sig_f, chi)
            if np.all(nu_sig_f <= 2.5 * sig_a):
                break
        else:  # pragma: no cover - the bound is loose enough in practice
            raise RuntimeError("could not draw a fissile material within bounds")
    return dict(sig_t=sig_t, sig_s=sig_s, nu_sig_f=nu_sig_f, chi=chi)


def stack_materials(mats):
    return dict(
        sig_t=np.ascontiguousarray(np.stack([m["sig_t"] for m in mats]), dtype=np.float64),
        sig_s=np.ascontiguousarray(np.stack([m["sig_s"] for m in mats]), dtype=np.float64),
        nu_sig_f=np.ascontiguousarray(np.stack([m["nu_sig_f"] for m in mats]), dtype=np.float64),
        chi=np.ascontiguousarray(np.stack([m["chi"] for m in mats]), dtype=np.float64),
    )


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def lattice_geometry(nx, ny, pitch, universes, pin_map, bc, x0=None, y0=None):
    """Rectangular lattice of pin universes.

    universes: list of (radii, mats) with len(mats) == len(radii) + 1; region
    r of a pin is inside ring r (r < len(radii)) or outside every ring.
    The lattice is centred on the origin unless x0/y0 are given.
    """
    max_rings = max(1, max(len(r) for r, _ in universes))
    n_univ = len(universes)
    n_rings = np.zeros(n_univ, np.int32)
    radii = np.zeros((n_univ, max_rings), np.float64)
    mats = np.full((n_univ, max_rings + 1), -1, np.int32)
    for u, (rr, mm) in enumerate(universes):
        assert len(mm) == len(rr) + 1
        n_rings[u] = len(rr)
        radii[u, : len(rr)] = rr
        mats[u, : len(mm)] = mm
        mats[u, len(mm):] = mm[-1]
    pin_map = np.ascontiguousarray(np.asarray(pin_map, np.int32).reshape(ny, nx))
    if x0 is None:
        x0 = -0.5 * nx * pitch
    if y0 is None:
        y0 = -0.5 * ny * pitch
    return dict(nx=int(nx), ny=int(ny), pitch=float(pitch), x0=float(x0), y0=float(y0),
                bc=[int(b) for b in bc], n_rings=n_rings, radii=radii, mats=mats,
                pin_map=pin_map)


def run_params(seed, n_per_gen, n_gen, n_inactive, fixed_source=False, problem_id=0,
               ent=(8, 8), max_events=100000):
    return dict(seed=int(seed), n_per_gen=int(n_per_gen), n_gen=int(n_gen),
                n_inactive=int(n_inactive), fixed_source=bool(fixed_source),
                problem_id=int(problem_id), ent_nx=int(ent[0]), ent_ny=int(ent[1]),
                max_events=int(max_events))


def make_problem(name, geometry, xs, run):
    return dict(name=name, geometry=geometry, xs=xs, run=run)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def pin_cell(n_per_gen=10_000, n_gen=30, n_inactive=10, seed=1, xs_seed=1000):
    """7-group pin cell: r = 0.54 cm fuel pin in a 1.26 cm reflective square."""
    rng = np.random.default_rng(xs_seed)
    fuel = mg_material(rng, fissile=True)
    mod = mg_material(rng, fissile=False)
    geo = lattice_geometry(1, 1, PIN_PITCH, [([PIN_RADIUS], [0, 1])], [[0]],
                           [REFLECT] * 4)
    return make_problem("pin_cell_7g", geo, stack_materials([fuel, mod]),
                        run_params(seed, n_per_gen, n_gen, n_inactive, ent=(8, 8)))


def lattice_17x17(n_per_gen=1_000_000, n_gen=60, n_inactive=20, seed=2):
    """17x17 lattice of the pin cell: 3 fuels + moderator, seeded pin map, vacuum."""
    fuels = [mg_material(np.random.default_rng(1001 + f), fissile=True) for f in range(3)]
    mod = mg_material(np.random.default_rng(1004), fissile=False)
    pin_map = np.random.default_rng(2001).integers(0, 3, size=(17, 17))
    univ = [([PIN_RADIUS], [f, 3]) for f in range(3)]
    geo = lattice_geometry(17, 17, PIN_PITCH, univ, pin_map, [VACUUM] * 4)
    return make_problem("lattice_17x17_7g", geo, stack_materials(fuels + [mod]),
                        run_params(seed, n_per_gen, n_gen, n_inactive, ent=(17, 17)))


def batch_pin_cells(n_problems=512, batch_seed=3001, n_min=1_000, n_max=1_000_000):
    """Independent fixed-source pin cells with their own XS, radius and size."""
    rng = np.random.default_rng(batch_seed)
    radii = rng.uniform(0.3, 0.6, n_problems)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_problems)))
    probs = []
    for p in range(n_problems):
        r = np.random.default_rng(10000 + p)
        fuel = mg_material(r, fissile=True)
        mod = mg_material(r, fissile=False)
        geo = lattice_geometry(1, 1, PIN_PITCH, [([float(radii[p])], [0, 1])], [[0]],
                               [REFLECT] * 4)
        run = run_params(100000 + p, int(sizes[p]), 1, 0, fixed_source=True,
                         problem_id=p, ent=(8, 8))
        probs.append(make_problem(f"batch_pin_{p}", geo, stack_materials([fuel, mod]), run))
    return probs


# ---------------------------------------------------------------------------
# closed-form test problems
# ---------------------------------------------------------------------------

def homogeneous(xs_material, n_per_gen, n_gen, n_inactive, seed, fixed_source=False,
                pitch=2.0):
    """Infinite medium: one reflective cell of a single material, no rings."""
    geo = lattice_geometry(1, 1, pitch, [([], [0])], [[0]], [REFLECT] * 4)
    return make_problem("homogeneous", geo, stack_materials([xs_material]),
                        run_params(seed, n_per_gen, n_gen, n_inactive,
                                   fixed_source=fixed_source, ent=(4, 4)))


def one_group(sig_t, sig_s, nu_sig_f):
    return dict(sig_t=np.array([sig_t], float), sig_s=np.array([[sig_s]], float),
                nu_sig_f=np.array([nu_sig_f], float),
                chi=np.array([1.0 if nu_sig_f > 0 else 0.0]))


def pin_cell_same_material(xs_material, n_per_gen, n_gen, n_inactive, seed, radius=PIN_RADIUS,
                           fixed_source=False):
    """Pin cell whose fuel and moderator are the same material (two copies)."""
    geo = lattice_geometry(1, 1, PIN_PITCH, [([radius], [0, 1])], [[0]], [REFLECT] * 4)
    return make_problem("pin_same", geo, stack_materials([xs_material, xs_material]),
                        run_params(seed, n_per_gen, n_gen, n_inactive,
                                   fixed_source=fixed_source, ent=(8, 8)))


def slab(thickness, sig_t, n_per_gen, seed):
    """Pure absorber slab: one cell of width `thickness`, vacuum in x,
    reflective in y.  Used with explicitly supplied start states."""
    geo = lattice_geometry(1, 1, thickness, [([], [0])], [[0]],
                           [VACUUM, VACUUM, REFLECT, REFLECT], x0=0.0,
                           y0=-0.5 * thickness)
    xs = stack_materials([one_group(sig_t, 0.0, 0.0)])
    return make_problem("slab", geo, xs,
                        run_params(seed, n_per_gen, 1, 0, fixed_source=True, ent=(1, 1)))


# ---------------------------------------------------------------------------
# continuous-energy data (input tables only: pointwise values on a grid)
# ---------------------------------------------------------------------------

CE_E_MIN, CE_E_MAX = 1e-5, 2e7     # eV
WATT_A, WATT_B = 0.988e6, 2.249e-6  # eV, 1/eV
NU_CE = 2.43


def _resonances(rng, e, n_res, channels):
    """Sum of n_res single-level resonance shapes
    s0 (G/2)^2 / ((E - Er)^2 + (G/2)^2) sqrt(Er / E), each split over the
    channels by Dirichlet fractions; returns [channels][len(e)]."""
    out = np.zeros((channels, len(e)))
    er = np.exp(rng.uniform(math.log(1.0), math.log(1e5), n_res))
    gam = np.exp(rng.uniform(math.log(1e-2), math.log(1.0), n_res))
    s0 = np.exp(rng.uniform(math.log(10.0), math.log(1e4), n_res))
    frac = rng.dirichlet(np.ones(channels), n_res)
    for k in range(n_res):
        h = 0.5 * gam[k]
        shape = s0[k] * h * h / ((e - er[k]) ** 2 + h * h) * np.sqrt(er[k] / e)
        out += frac[k][:, None] * shape[None, :]
    return out


def _ce_tables(seed, n_nuc, n_pts, n_res):
    rng = np.random.default_rng(seed)
    e = np.geomspace(CE_E_MIN, CE_E_MAX, n_pts)
    awr = np.sort(rng.uniform(1.0, 240.0, n_nuc))
    n_fissile = 2
    sig_s = np.zeros((n_nuc, n_pts))
    sig_c = np.zeros((n_nuc, n_pts))
    sig_f = np.zeros((n_nuc, n_pts))
    inv_v = np.sqrt(0.0253 / e)
    for n in range(n_nuc):
        fissile = n >= n_nuc - n_fissile
        sig_s[n] = rng.uniform(2.0, 20.0)
        if fissile:
            sig_c[n] = rng.uniform(20.0, 100.0) * inv_v
            sig_f[n] = rng.uniform(200.0, 600.0) * inv_v
            res = _resonances(rng, e, n_res, 3)
            sig_s[n] += res[0]
            sig_c[n] += res[1]
            sig_f[n] += res[2]
        else:
            sig_c[n] = rng.uniform(0.1, 5.0) * inv_v
            res = _resonances(rng, e, n_res, 2)
            sig_s[n] += res[0]
            sig_c[n] += res[1]
    sig_t = sig_s + sig_c + sig_f
    return e, awr, sig_t, sig_s, sig_f


_CE_CACHE = {}


def ce_data(seed=4001, n_nuc=10, n_pts=50_000, n_res=200, n_ebins=100):
    """10 synthetic nuclides on a 50,000-point log grid, 1e-5 eV .. 20 MeV:
    1/v capture and fission backgrounds plus 200 seeded resonances each,
    constant potential scattering; target masses A ~ U[1, 240] sorted, the
    five lightest make the moderator, the five heaviest the fuel, whose two
    heaviest are fissile.  Material 0 = fuel, 1 = moderator."""
    key = (seed, n_nuc, n_pts, n_res, n_ebins)
    if key not in _CE_CACHE:
        e, awr, sig_t, sig_s, sig_f = _ce_tables(seed, n_nuc, n_pts, n_res)
        rng = np.random.default_rng(seed + 1)
        half = n_nuc // 2
        fuel = np.arange(half, n_nuc)
        mod = np.arange(0, half)
        mat_nuc = np.stack([fuel, mod]).astype(np.int32)
        mat_dens = np.stack([rng.uniform(1e-3, 2e-2, len(fuel)),
                             rng.uniform(1e-2, 5e-2, len(mod))])
        _CE_CACHE[key] = dict(
            e_grid=e, sig_t=sig_t, sig_s=sig_s, sig_f=sig_f, awr=awr, nu=NU_CE,
            mat_n=np.array([len(fuel), len(mod)], np.int32), mat_nuc=mat_nuc,
            mat_dens=mat_dens, watt_a=WATT_A, watt_b=WATT_B, e_max=CE_E_MAX,
            e_cut=CE_E_MIN, e_edges=np.geomspace(CE_E_MIN, CE_E_MAX, n_ebins + 1))
    return _CE_CACHE[key]


def ce_pin_cell(n_per_gen=1_000_000, n_gen=50, n_inactive=10, seed=4, data=None):
    """Continuous-energy pin cell (r = 0.54 cm in a 1.26 cm reflective
    square: an infinite lattice), flux tallied per region on 100 log bins."""
    ce = ce_data() if data is None else data
    geo = lattice_geometry(1, 1, PIN_PITCH, [([PIN_RADIUS], [0, 1])], [[0]], [REFLECT] * 4)
    return dict(name="ce_pin_cell", geometry=geo, ce=ce,
                run=run_params(seed, n_per_gen, n_gen, n_inactive, ent=(8, 8)))


def ce_flat(sig_s, sig_c, sig_f, awr, dens=1.0, n_pts=2, n_ebins=10, e_cut=CE_E_MIN):
    """One nuclide with energy-independent cross sections (barns) in one
    material: the continuous-energy code path with closed-form answers."""
    e = np.array([CE_E_MIN, CE_E_MAX]) if n_pts == 2 else np.geomspace(CE_E_MIN, CE_E_MAX, n_pts)
    row = np.ones(len(e))
    return dict(e_grid=e, sig_t=((sig_s + sig_c + sig_f) * row)[None, :],
                sig_s=(sig_s * row)[None, :], sig_f=(sig_f * row)[None, :],
                awr=np.array([float(awr)]), nu=NU_CE, mat_n=np.array([1], np.int32),
                mat_nuc=np.array([[0]], np.int32), mat_dens=np.array([[float(dens)]]),
                watt_a=WATT_A, watt_b=WATT_B, e_max=CE_E_MAX, e_cut=e_cut,
                e_edges=np.geomspace(CE_E_MIN, CE_E_MAX, n_ebins + 1))


def ce_homogeneous(ce, n_per_gen, n_gen, n_inactive, seed, fixed_source=False, pitch=2.0):
    """Infinite medium of continuous-energy material 0."""
    geo = lattice_geometry(1, 1, pitch, [([], [0])], [[0]], [REFLECT] * 4)
    return dict(name="ce_homogeneous", geometry=geo, ce=ce,
                run=run_params(seed, n_per_gen, n_gen, n_inactive, fixed_source=fixed_source,
                               ent=(4, 4)))


# ---------------------------------------------------------------------------
# time-dependent fixed source (input tables only)
# ---------------------------------------------------------------------------

# speeds of the 7 groups, fast to thermal (cm/s): log-spaced from about
# 2 MeV neutrons (2e9 cm/s) to thermal ones (2.2e5 cm/s)
GROUP_SPEEDS_7 = np.geomspace(2.0e9, 2.2e5, N_GROUPS)


def with_time(problem, t_edges, speed=None):
    """Copy of a fixed-source problem with a time grid: a pulse at t = 0,
    flux tallied per time bin, census at the last edge.  Multigroup problems
    take one speed per group; continuous-energy problems take none (the
    speed follows from the energy)."""
    p = dict(problem)
    if "ce" in problem:
        assert speed is None
        v = None
    else:
        g = problem["xs"]["sig_t"].shape[1]
        v = GROUP_SPEEDS_7 if speed is None else np.asarray(speed, float)
        assert len(v) == g
    p["time"] = dict(t_edges=np.asarray(t_edges, float), speed=v)
    p["run"] = dict(problem["run"], fixed_source=True)
    return p


SOURCE_14MEV = 14.0e6  # eV


def ce_pulsed_pin_cell(n_per_gen=1_000_000, n_gen=10, seed=7, data=None):
    """The continuous-energy pin cell as a time-dependent fixed-source
    problem, the shape of the paper's second benchmark (Sec. 4): every
    history starts at t = 0 with 14 MeV, uniform over the fuel, fission
    treated as capture; flux and neutron density per region, energy bin and
    time bin (0, then 24 log bins from 1e-10 s to 1e-5 s), census at 10 us
    (the synthetic resonances absorb most histories within a microsecond)."""
    ce = dict(ce_data() if data is None else data, src_energy=SOURCE_14MEV)
    prob = ce_pin_cell(n_per_gen=n_per_gen, n_gen=n_gen, n_inactive=0, seed=seed, data=ce)
    prob = with_run(prob, fixed_source=True)
    edges = np.concatenate([[0.0], np.geomspace(1e-10, 1e-5, 25)])
    return with_time(prob, edges)


def pulsed_lattice(n_per_gen=1_000_000, n_gen=10, seed=6):
    """The 17x17 lattice driven by a source pulse at t = 0 (fission as
    capture): flux per pin, group and time bin (0, then 11 log bins from
    1e-9 s to 1e-5 s), census at 10 us, where about a quarter of the
    histories are still flying."""
    lat = lattice_17x17(n_per_gen=n_per_gen, n_gen=n_gen, n_inactive=0, seed=seed)
    lat = with_run(lat, fixed_source=True)
    edges = np.concatenate([[0.0], np.geomspace(1e-9, 1e-5, 12)])
    return with_time(lat, edges)


def with_run(problem, **kw):
    """Copy of a problem with some run parameters replaced."""
    p = dict(problem)
    p["run"] = dict(problem["run"])
    p["run"].update(kw)
    return p


def n_bins(problem):
    geo = problem["geometry"]
    per = (len(problem["ce"]["e_edges"]) - 1 if "ce" in problem
           else problem["xs"]["sig_t"].shape[1])
    if "time" in problem:
        per *= len(problem["time"]["t_edges"]) - 1
    return geo["nx"] * geo["ny"] * (geo["radii"].shape[1] + 1) * per


def digest(problem):
    """sha256 over every array and scalar of a problem (records the inputs)."""
    h = hashlib.sha256()
    for part in ("geometry", "xs", "ce", "time", "run"):
        if part not in problem:
            continue
        d = problem[part]
        for k in sorted(d):
            v = d[k]
            h.update(k.encode())
            h.update(np.ascontiguousarray(np.asarray(v)).tobytes())
    return h.hexdigest()
