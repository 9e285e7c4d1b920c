"""ctypes wrapper of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.  It marshals a problem dict (see
paper_2501_05440_amd/problems.py) into the oracle's own C structs and returns
numpy arrays; all transport arithmetic lives in oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

COUNT_NAMES = ["seg", "col", "cross", "refl", "leak", "abs", "killed", "sites", "scat", "cutoff",
               "census"]
FATE = {"alive": 0, "absorbed": 1, "leaked": 2, "killed": 3, "cutoff": 4, "census": 5}
TAG_SRC, TAG_TRANSPORT, TAG_RESAMPLE = 1, 2, 3


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", SRC_PATH,
           "-lquadmath", "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("pitch", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("bc", C.c_int32 * 4),
        ("n_univ", C.c_int32), ("max_rings", C.c_int32),
        ("n_rings", C.c_void_p), ("radii", C.c_void_p), ("mats", C.c_void_p),
        ("pin_map", C.c_void_p),
        ("n_mat", C.c_int32), ("n_grp", C.c_int32),
        ("sig_t", C.c_void_p), ("sig_s", C.c_void_p), ("nu_sig_f", C.c_void_p),
        ("chi", C.c_void_p),
        ("seed", C.c_uint64), ("n_per_gen", C.c_int64),
        ("n_gen", C.c_int32), ("n_inactive", C.c_int32),
        ("fixed_source", C.c_int32), ("problem_id", C.c_uint64),
        ("ent_nx", C.c_int32), ("ent_ny", C.c_int32),
        ("max_events", C.c_int64), ("n_threads", C.c_int32),
        ("ext_state", C.c_void_p),
        ("ce", C.c_void_p),
        ("time", C.c_void_p),
    ]


class _Time(C.Structure):
    _fields_ = [("n_tbins", C.c_int32), ("t_edges", C.c_void_p), ("speed", C.c_void_p)]


class _CE(C.Structure):
    _fields_ = [
        ("n_nuc", C.c_int32), ("n_pts", C.c_int32),
        ("e_grid", C.c_void_p), ("sig_t", C.c_void_p), ("sig_s", C.c_void_p),
        ("sig_f", C.c_void_p), ("awr", C.c_void_p), ("nu", C.c_double),
        ("max_nuc", C.c_int32), ("mat_n", C.c_void_p), ("mat_nuc", C.c_void_p),
        ("mat_dens", C.c_void_p), ("watt_a", C.c_double), ("watt_b", C.c_double),
        ("e_max", C.c_double), ("e_cut", C.c_double), ("n_ebins", C.c_int32),
        ("e_edges", C.c_void_p), ("src_energy", C.c_double),
    ]


RECORD_DTYPE = np.dtype([
    ("n_seg", "<i4"), ("n_col", "<i4"), ("n_cross", "<i4"), ("n_refl", "<i4"),
    ("fate", "<i4"), ("n_sites", "<i4"), ("g_final", "<i4"), ("ctr_final", "<u4"),
    ("tl_sum", "<f8"), ("kcol_sum", "<f8"), ("x_final", "<f8"), ("y_final", "<f8"),
    ("e_final", "<f8"), ("t_final", "<f8"),
])


class _Record(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_seg", "n_col", "n_cross", "n_refl", "fate",
                                          "n_sites", "g_final")] + [
        ("ctr_final", C.c_uint32), ("tl_sum", C.c_double), ("kcol_sum", C.c_double),
        ("x_final", C.c_double), ("y_final", C.c_double), ("e_final", C.c_double),
        ("t_final", C.c_double)]


EVENT_DTYPE = np.dtype([
    ("x", "<f8"), ("y", "<f8"), ("d", "<f8"), ("e", "<f8"),
    ("cell", "<i4"), ("region", "<i4"), ("group", "<i4"), ("type", "<i4"),
])


class _Output(C.Structure):
    _fields_ = [
        ("gen_k", C.c_void_p), ("gen_entropy", C.c_void_p), ("gen_counts", C.c_void_p),
        ("k_mean", C.c_double * 3), ("k_sigma", C.c_double * 3),
        ("flux_mean", C.c_void_p), ("flux_sigma", C.c_void_p),
        ("prod_mean", C.c_void_p), ("prod_sigma", C.c_void_p),
        ("gen_flux", C.c_void_p), ("gen_prod", C.c_void_p),
        ("records", C.c_void_p),
        ("bank", C.c_void_p), ("bank_cap", C.c_int64), ("bank_len", C.c_int64),
        ("events", C.c_void_p), ("event_cap", C.c_int32),
        ("source", C.c_void_p),
        ("errmsg", C.c_char * 256),
    ]


assert C.sizeof(_Record) == RECORD_DTYPE.itemsize == 80

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Output)]
        L.orc_run.restype = C.c_int
        L.orc_histories.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int64,
                                    C.POINTER(_Output)]
        L.orc_histories.restype = C.c_int
        L.orc_n_bins.argtypes = [C.POINTER(_Problem)]
        L.orc_n_bins.restype = C.c_int64
        L.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        L.orc_philox4x64_10.restype = None
        L.orc_uniform.argtypes = [C.c_uint64]
        L.orc_uniform.restype = C.c_double
        L.orc_stream_uniform.argtypes = [C.c_uint64] * 5 + [C.c_uint32]
        L.orc_stream_uniform.restype = C.c_double
        L.orc_dist_plane.argtypes = [C.c_double] * 4
        L.orc_dist_plane.restype = C.c_double
        L.orc_dist_cylinder.argtypes = [C.c_double] * 5 + [C.c_int]
        L.orc_dist_cylinder.restype = C.c_double
        L.orc_cr_log.argtypes = [C.c_double]
        L.orc_cr_log.restype = C.c_double
        L.orc_cr_cossin_2pi.argtypes = [C.c_double, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.orc_cr_cossin_2pi.restype = None
        L.orc_isotropic.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.orc_isotropic.restype = None
        L.orc_sample_cdf.argtypes = [C.c_double, C.POINTER(C.c_double), C.c_int]
        L.orc_sample_cdf.restype = C.c_int
        L.orc_comb.argtypes = [C.c_int64, C.c_int64, C.c_double, C.POINTER(C.c_int64)]
        L.orc_comb.restype = None
        L.orc_entropy.argtypes = [C.POINTER(C.c_int64), C.c_int64, C.c_int64]
        L.orc_entropy.restype = C.c_double
        L.orc_neumaier.argtypes = [C.POINTER(C.c_double), C.c_int64]
        L.orc_neumaier.restype = C.c_double
        L.orc_ce_interval.argtypes = [C.POINTER(C.c_double), C.c_int, C.c_double]
        L.orc_ce_interval.restype = C.c_int
        L.orc_ce_macro.argtypes = [C.POINTER(_CE), C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.orc_ce_macro.restype = None
        L.orc_watt_attempt.argtypes = [C.c_double] * 6
        L.orc_watt_attempt.restype = C.c_double
        L.orc_elastic.argtypes = [C.c_double] * 3 + [C.POINTER(C.c_double)]
        L.orc_elastic.restype = C.c_double
        L.orc_rotate.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.orc_rotate.restype = None
        L.orc_speed.argtypes = [C.c_double]
        L.orc_speed.restype = C.c_double
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def uniform(word):
    return lib().orc_uniform(int(word) & (2**64 - 1))


def stream_uniform(seed, tag, pid, gen, prob, draw):
    return lib().orc_stream_uniform(seed, tag, pid, gen, prob, draw)


def dist_plane(x, lo, hi, u):
    return lib().orc_dist_plane(x, lo, hi, u)


def dist_cylinder(dx, dy, u, v, radius, inside):
    return lib().orc_dist_cylinder(dx, dy, u, v, radius, int(bool(inside)))


def cr_log(x):
    return lib().orc_cr_log(float(x))


def cr_cossin_2pi(t):
    c, s = C.c_double(), C.c_double()
    lib().orc_cr_cossin_2pi(float(t), C.byref(c), C.byref(s))
    return c.value, s.value


def isotropic(xi_mu, xi_phi):
    o = (C.c_double * 3)()
    lib().orc_isotropic(xi_mu, xi_phi, o)
    return tuple(o)


def sample_cdf(xi, weights):
    w = np.ascontiguousarray(weights, dtype=np.float64)
    return lib().orc_sample_cdf(xi, w.ctypes.data_as(C.POINTER(C.c_double)), len(w))


def comb(n, m, xi0):
    out = np.zeros(n, np.int64)
    lib().orc_comb(n, m, xi0, out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out


def entropy(counts, m):
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return lib().orc_entropy(c.ctypes.data_as(C.POINTER(C.c_int64)), len(c), int(m))


def neumaier(values):
    v = np.ascontiguousarray(values, dtype=np.float64)
    return lib().orc_neumaier(v.ctypes.data_as(C.POINTER(C.c_double)), len(v))


def ce_interval(grid, e):
    g = np.ascontiguousarray(grid, dtype=np.float64)
    return lib().orc_ce_interval(g.ctypes.data_as(C.POINTER(C.c_double)), len(g), float(e))


def ce_macro(ce, m, e):
    """(Sigma_t, Sigma_s, Sigma_f) of material m at energy e."""
    keep = []
    S = _ce_struct(ce, keep)
    o = (C.c_double * 3)()
    lib().orc_ce_macro(C.byref(S), int(m), float(e), o)
    return tuple(o)


def speed(e):
    """Neutron speed in cm/s at energy e in eV."""
    return lib().orc_speed(float(e))


def watt_attempt(a, b, x1, x2, x3, x4):
    return lib().orc_watt_attempt(a, b, x1, x2, x3, x4)


def elastic(awr, e, xi_mu):
    mu = C.c_double()
    e_out = lib().orc_elastic(awr, e, xi_mu, C.byref(mu))
    return e_out, mu.value


def rotate(mu, xi_phi, direction):
    d = (C.c_double * 3)(*[float(v) for v in direction])
    lib().orc_rotate(mu, xi_phi, d)
    return tuple(d)


def _ce_struct(ce, keep):
    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    S = _CE()
    sig_t = np.asarray(ce["sig_t"])
    S.n_nuc, S.n_pts = sig_t.shape
    S.e_grid = arr(ce["e_grid"], np.float64)
    S.sig_t = arr(ce["sig_t"], np.float64)
    S.sig_s = arr(ce["sig_s"], np.float64)
    S.sig_f = arr(ce["sig_f"], np.float64)
    S.awr = arr(ce["awr"], np.float64)
    S.nu = ce["nu"]
    mat_nuc = np.asarray(ce["mat_nuc"])
    S.max_nuc = mat_nuc.shape[1]
    S.mat_n = arr(ce["mat_n"], np.int32)
    S.mat_nuc = arr(mat_nuc, np.int32)
    S.mat_dens = arr(ce["mat_dens"], np.float64)
    S.watt_a, S.watt_b = ce["watt_a"], ce["watt_b"]
    S.e_max, S.e_cut = ce["e_max"], ce["e_cut"]
    edges = np.asarray(ce["e_edges"])
    S.n_ebins = len(edges) - 1
    S.e_edges = arr(edges, np.float64)
    S.src_energy = float(ce.get("src_energy", 0.0))
    return S


# ---------------------------------------------------------------------------
# full runs
# ---------------------------------------------------------------------------

class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data


def _problem(problem, n_threads=None, ext_state=None):
    """The orc_problem of a problem dict, and the arrays it points into."""
    geo, rp = problem["geometry"], problem["run"]
    ce = problem.get("ce")
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    n_rings = arr(geo["n_rings"], np.int32)
    radii = arr(geo["radii"], np.float64)
    mats = arr(geo["mats"], np.int32)
    pin_map = arr(geo["pin_map"], np.int32)
    if ce is None:
        xs = problem["xs"]
        sig_t = arr(xs["sig_t"], np.float64)
        sig_s = arr(xs["sig_s"], np.float64)
        nusf = arr(xs["nu_sig_f"], np.float64)
        chi = arr(xs["chi"], np.float64)
        n_mat, n_grp = sig_t.shape
        assert sig_s.shape == (n_mat, n_grp, n_grp)
    else:
        sig_t = sig_s = nusf = chi = None
        n_mat, n_grp = len(ce["mat_n"]), 0
        ce_s = _ce_struct(ce, keep)
        keep.append(ce_s)
    ext = None if ext_state is None else arr(ext_state, np.float64)
    if ext is not None:
        assert ext.shape == (rp["n_per_gen"], 6)

    P = _Problem()
    P.nx, P.ny = geo["nx"], geo["ny"]
    P.pitch, P.x0, P.y0 = geo["pitch"], geo["x0"], geo["y0"]
    P.bc = (C.c_int32 * 4)(*geo["bc"])
    P.n_univ = len(n_rings)
    P.max_rings = radii.shape[1]
    P.n_rings, P.radii, P.mats, P.pin_map = (_ptr(n_rings), _ptr(radii), _ptr(mats),
                                             _ptr(pin_map))
    P.n_mat, P.n_grp = n_mat, n_grp
    P.sig_t, P.sig_s, P.nu_sig_f, P.chi = _ptr(sig_t), _ptr(sig_s), _ptr(nusf), _ptr(chi)
    P.seed = rp["seed"]
    P.n_per_gen = rp["n_per_gen"]
    P.n_gen, P.n_inactive = rp["n_gen"], rp["n_inactive"]
    P.fixed_source = int(rp["fixed_source"])
    P.problem_id = rp["problem_id"]
    P.ent_nx, P.ent_ny = rp["ent_nx"], rp["ent_ny"]
    P.max_events = rp["max_events"]
    P.n_threads = n_threads if n_threads else (os.cpu_count() or 1)
    P.ext_state = _ptr(ext)
    P.ce = None if ce is None else C.addressof(ce_s)
    tm = problem.get("time")
    if tm is not None:
        t_s = _Time()
        edges = arr(tm["t_edges"], np.float64)
        t_s.n_tbins = len(edges) - 1
        t_s.t_edges = edges.ctypes.data
        t_s.speed = None if tm.get("speed") is None else arr(tm["speed"], np.float64).ctypes.data
        keep.append(t_s)
        P.time = C.addressof(t_s)
    return P, keep


def run(problem, n_threads=None, records=False, per_gen_tallies=False, bank_cap=0,
        ext_state=None, events=0, source=False):
    """Run the oracle on a problem dict; returns a dict of numpy arrays."""
    rp = problem["run"]
    P, keep = _problem(problem, n_threads, ext_state)
    L = lib()
    nb = L.orc_n_bins(C.byref(P))
    G, N = rp["n_gen"], rp["n_per_gen"]
    res = dict(
        gen_k=np.zeros((G, 3)), gen_entropy=np.zeros(G),
        gen_counts=np.zeros((G, len(COUNT_NAMES)), np.int64),
        flux_mean=np.zeros(nb), flux_sigma=np.zeros(nb),
        prod_mean=np.zeros(nb), prod_sigma=np.zeros(nb),
    )
    O = _Output()
    O.gen_k, O.gen_entropy, O.gen_counts = (_ptr(res["gen_k"]), _ptr(res["gen_entropy"]),
                                            _ptr(res["gen_counts"]))
    O.flux_mean, O.flux_sigma = _ptr(res["flux_mean"]), _ptr(res["flux_sigma"])
    O.prod_mean, O.prod_sigma = _ptr(res["prod_mean"]), _ptr(res["prod_sigma"])
    if per_gen_tallies:
        res["gen_flux"] = np.zeros((G, nb))
        res["gen_prod"] = np.zeros((G, nb))
        O.gen_flux, O.gen_prod = _ptr(res["gen_flux"]), _ptr(res["gen_prod"])
    if records:
        res["records"] = np.zeros((G, N), RECORD_DTYPE)
        O.records = _ptr(res["records"])
    if bank_cap:
        res["bank"] = np.zeros((bank_cap, 3))
        O.bank = _ptr(res["bank"])
        O.bank_cap = bank_cap
    if events:
        res["events"] = np.zeros((G, N, events), EVENT_DTYPE)
        O.events = _ptr(res["events"])
        O.event_cap = events
    if source:
        res["source"] = np.zeros((G, N, 3))
        O.source = _ptr(res["source"])
    rc = L.orc_run(C.byref(P), C.byref(O))
    if rc != 0:
        raise OracleError(rc, O.errmsg.decode())
    res["k_mean"] = np.array(O.k_mean[:])
    res["k_sigma"] = np.array(O.k_sigma[:])
    if bank_cap:
        res["bank"] = res["bank"][: min(bank_cap, O.bank_len)]
    res["bank_len"] = int(O.bank_len)
    res["n_bins"] = int(nb)
    del keep
    return res


def histories(problem, ids, ext_state=None):
    """Records of the first-generation histories ids (any ids below the
    problem's n_per_gen), as run() gives them, without running the rest of
    the generation (orc_histories)."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    P, keep = _problem(problem, 1, ext_state)
    out = np.zeros(len(ids), RECORD_DTYPE)
    O = _Output()
    O.records = _ptr(out)
    rc = lib().orc_histories(C.byref(P), _ptr(ids), len(ids), C.byref(O))
    if rc != 0:
        raise OracleError(rc, O.errmsg.decode())
    del keep
    return out
