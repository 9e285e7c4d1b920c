"""Python binding of libmcx (include/mcx.h): argument marshalling only.

Every step of the transport runs in the library's HIP kernels.  PyTorch
provides the device workspace (one uint8 tensor) and the stream.  There is
no fallback: if libmcx.so is missing the import of the library fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcx.so")

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, ELOST, EGUARD, EEXTINCT, EOVERFLOW = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FP64, FP32_MIXED = 0, 1
ENGINE_EVENT, ENGINE_PERSISTENT, ENGINE_MONOLITHIC, ENGINE_ASYNC = 0, 1, 2, 3
ENGINES = {"event": ENGINE_EVENT, "persistent": ENGINE_PERSISTENT,
           "monolithic": ENGINE_MONOLITHIC, "async": ENGINE_ASYNC}
N_CNT = 11
COUNT_NAMES = ["seg", "col", "cross", "refl", "leak", "abs", "killed", "sites", "scat", "cutoff",
               "census"]

# every function the header declares
EXPORTS = [
    "mcx_create", "mcx_load_geometry", "mcx_load_mg_xs", "mcx_seed_source",
    "mcx_workspace_size", "mcx_bind_workspace", "mcx_run_generations", "mcx_get_keff",
    "mcx_get_generation_stats", "mcx_get_tallies", "mcx_get_generation_tallies",
    "mcx_get_records", "mcx_get_bank", "mcx_get_timing", "mcx_diag_math", "mcx_host_math",
    "mcx_diag_philox", "mcx_last_error", "mcx_destroy", "mcx_load_batch", "mcx_run_batch",
    "mcx_get_batch_results", "mcx_get_batch_tallies", "mcx_autotune", "mcx_load_ce_xs",
    "mcx_continue_generations", "mcx_checkpoint", "mcx_restore", "mcx_get_event_log",
    "mcx_load_time_grid", "mcx_run_generations_noalloc",
]


class MCXError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmcx error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
                ("block_size", C.c_int32), ("tail_threshold", C.c_int32),
                ("lookahead", C.c_int32), ("max_events", C.c_int64),
                ("record_histories", C.c_int32), ("time_kernels", C.c_int32),
                ("engine", C.c_int32), ("p_block", C.c_int32), ("p_slots", C.c_int32),
                ("p_grid", C.c_int32), ("p_tau", C.c_double), ("p_sort", C.c_int32),
                ("flights", C.c_int32), ("event_log", C.c_int32),
                ("time_stride", C.c_int32), ("rounds", C.c_int32),
                ("lds_tally_min", C.c_int32), ("lt_flights", C.c_int32)]


class Geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("pitch", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("bc", C.c_int32 * 4),
                ("n_univ", C.c_int32), ("max_rings", C.c_int32), ("n_rings", C.c_void_p),
                ("radii", C.c_void_p), ("mats", C.c_void_p), ("pin_map", C.c_void_p)]


class Source(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_per_gen", C.c_int64), ("fixed_source", C.c_int32),
                ("problem_id", C.c_uint64), ("ent_nx", C.c_int32), ("ent_ny", C.c_int32)]


class Timing(C.Structure):
    _fields_ = [("run_ms", C.c_double), ("n_iterations", C.c_int64),
                ("n_tail_launches", C.c_int64), ("advance_ms", C.c_double),
                ("collide_ms", C.c_double), ("tail_ms", C.c_double),
                ("n_advance", C.c_int64), ("n_collide", C.c_int64),
                ("advance_items", C.c_int64), ("collide_items", C.c_int64),
                ("persistent_ms", C.c_double), ("n_persistent", C.c_int64),
                ("advance_segments", C.c_int64)]


class CEData(C.Structure):
    _fields_ = [("n_nuc", C.c_int32), ("n_pts", C.c_int32), ("e_grid", C.c_void_p),
                ("sig_t", C.c_void_p), ("sig_s", C.c_void_p), ("sig_f", C.c_void_p),
                ("awr", C.c_void_p), ("nu", C.c_double), ("n_mat", C.c_int32),
                ("max_nuc", C.c_int32), ("mat_n", C.c_void_p), ("mat_nuc", C.c_void_p),
                ("mat_dens", C.c_void_p), ("watt_a", C.c_double), ("watt_b", C.c_double),
                ("e_max", C.c_double), ("e_cut", C.c_double), ("n_ebins", C.c_int32),
                ("e_edges", C.c_void_p), ("src_energy", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("geo", Geometry), ("n_mat", C.c_int32), ("n_grp", C.c_int32),
                ("sig_t", C.c_void_p), ("sig_s", C.c_void_p), ("nu_sig_f", C.c_void_p),
                ("chi", C.c_void_p), ("seed", C.c_uint64), ("n_hist", C.c_int64),
                ("problem_id", C.c_uint64)]


class Tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("slots", C.c_int32), ("grid", C.c_int32),
                ("tau", C.c_double), ("ms", C.c_double), ("sort", C.c_int32),
                ("flights", C.c_int32), ("lt_flights", C.c_int32), ("tail", C.c_int32)]


EVENT_DTYPE = np.dtype([
    ("x", "<f8"), ("y", "<f8"), ("d", "<f8"), ("e", "<f8"),
    ("cell", "<i4"), ("region", "<i4"), ("group", "<i4"), ("type", "<i4"),
])

RECORD_DTYPE = np.dtype([
    ("n_seg", "<i4"), ("n_col", "<i4"), ("n_cross", "<i4"), ("n_refl", "<i4"),
    ("fate", "<i4"), ("n_sites", "<i4"), ("g_final", "<i4"), ("ctr_final", "<u4"),
    ("tl_sum", "<f8"), ("kcol_sum", "<f8"), ("x_final", "<f8"), ("y_final", "<f8"),
    ("e_final", "<f8"), ("t_final", "<f8"),
])

_lib = None


def lib():
    """Load libmcx.so (built by paper_2501_05440_amd/build.py); no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2501_05440_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "mcx_create": ([C.POINTER(vp), C.POINTER(Options)], C.c_int),
        "mcx_load_geometry": ([vp, C.POINTER(Geometry)], C.c_int),
        "mcx_load_mg_xs": ([vp, i32, i32, dp, dp, dp, dp], C.c_int),
        "mcx_seed_source": ([vp, C.POINTER(Source)], C.c_int),
        "mcx_workspace_size": ([vp, i32, C.POINTER(C.c_size_t)], C.c_int),
        "mcx_bind_workspace": ([vp, vp, C.c_size_t, i32], C.c_int),
        "mcx_run_generations": ([vp, i32, i32], C.c_int),
        "mcx_run_generations_noalloc": ([vp, i32, i32], C.c_int),
        "mcx_get_keff": ([vp, dp, dp, dp], C.c_int),
        "mcx_get_generation_stats": ([vp, dp, dp], C.c_int),
        "mcx_get_tallies": ([vp, dp, dp, dp, dp, i64], C.c_int),
        "mcx_get_generation_tallies": ([vp, i32, dp, dp, i64], C.c_int),
        "mcx_get_records": ([vp, i32, dp, i64], C.c_int),
        "mcx_get_bank": ([vp, dp, i64, C.POINTER(i64)], C.c_int),
        "mcx_get_timing": ([vp, C.POINTER(Timing)], C.c_int),
        "mcx_diag_math": ([vp, i32, dp, dp, i64], C.c_int),
        "mcx_host_math": ([i32, dp, dp, i64], C.c_int),
        "mcx_diag_philox": ([vp, dp, dp, i64], C.c_int),
        "mcx_last_error": ([vp], C.c_char_p),
        "mcx_destroy": ([vp], None),
        "mcx_load_batch": ([vp, i32, C.POINTER(Problem)], C.c_int),
        "mcx_run_batch": ([vp], C.c_int),
        "mcx_get_batch_results": ([vp, dp, dp], C.c_int),
        "mcx_get_batch_tallies": ([vp, i32, dp, dp, i64], C.c_int),
        "mcx_autotune": ([vp, C.c_char_p, C.POINTER(Tune)], C.c_int),
        "mcx_load_ce_xs": ([vp, C.POINTER(CEData)], C.c_int),
        "mcx_continue_generations": ([vp, i32], C.c_int),
        "mcx_checkpoint": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "mcx_restore": ([vp, vp, C.c_size_t], C.c_int),
        "mcx_get_event_log": ([vp, i32, dp, i64], C.c_int),
        "mcx_load_time_grid": ([vp, i32, dp, dp, i32], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def host_math(which, values):
    """The library's ln / cos,sin(2 pi t) / sqrt / uniform mapping on the host."""
    x = np.ascontiguousarray(values, dtype=np.float64)
    out = np.zeros(2 * len(x) if which == 1 else len(x))
    rc = lib().mcx_host_math(which, x.ctypes.data, out.ctypes.data, len(x))
    if rc:
        raise MCXError(rc, "mcx_host_math")
    return out.reshape(-1, 2) if which == 1 else out


def _arr(a, dt, keep):
    a = np.ascontiguousarray(a, dtype=dt)
    keep.append(a)
    return a


def _geometry(geo, keep):
    n_rings = _arr(geo["n_rings"], np.int32, keep)
    radii = _arr(geo["radii"], np.float64, keep)
    mats = _arr(geo["mats"], np.int32, keep)
    pin_map = _arr(geo["pin_map"], np.int32, keep)
    g = Geometry()
    g.nx, g.ny = geo["nx"], geo["ny"]
    g.pitch, g.x0, g.y0 = geo["pitch"], geo["x0"], geo["y0"]
    g.bc = (C.c_int32 * 4)(*geo["bc"])
    g.n_univ, g.max_rings = len(n_rings), radii.shape[1]
    g.n_rings, g.radii = n_rings.ctypes.data, radii.ctypes.data
    g.mats, g.pin_map = mats.ctypes.data, pin_map.ctypes.data
    return g


def _ce(ce, keep):
    d = CEData()
    sig_t = _arr(ce["sig_t"], np.float64, keep)
    d.n_nuc, d.n_pts = sig_t.shape
    d.e_grid = _arr(ce["e_grid"], np.float64, keep).ctypes.data
    d.sig_t = sig_t.ctypes.data
    d.sig_s = _arr(ce["sig_s"], np.float64, keep).ctypes.data
    d.sig_f = _arr(ce["sig_f"], np.float64, keep).ctypes.data
    d.awr = _arr(ce["awr"], np.float64, keep).ctypes.data
    d.nu = ce["nu"]
    mat_nuc = _arr(ce["mat_nuc"], np.int32, keep)
    d.n_mat, d.max_nuc = mat_nuc.shape
    d.mat_n = _arr(ce["mat_n"], np.int32, keep).ctypes.data
    d.mat_nuc = mat_nuc.ctypes.data
    d.mat_dens = _arr(ce["mat_dens"], np.float64, keep).ctypes.data
    d.watt_a, d.watt_b = ce["watt_a"], ce["watt_b"]
    d.e_max, d.e_cut = ce["e_max"], ce["e_cut"]
    edges = _arr(ce["e_edges"], np.float64, keep)
    d.n_ebins = len(edges) - 1
    d.e_edges = edges.ctypes.data
    d.src_energy = float(ce.get("src_energy", 0.0))
    return d


def _xs(xs, keep):
    arrs = [_arr(xs[k], np.float64, keep) for k in ("sig_t", "sig_s", "nu_sig_f", "chi")]
    return arrs[0].shape, [a.ctypes.data for a in arrs]


def _options(o, precision, device, stream, engine, persistent):
    if precision not in ("fp64", "fp32"):
        raise ValueError("precision is 'fp64' or 'fp32' (FP32-mixed)")
    if engine not in ENGINES:
        raise ValueError(f"engine is one of {sorted(ENGINES)}")
    o.precision = FP64 if precision == "fp64" else FP32_MIXED
    o.device = device
    o.stream = stream.cuda_stream
    o.engine = ENGINES[engine]
    p = persistent or {}
    o.p_block = p.get("block", 0)
    o.p_slots = p.get("slots", 0)
    o.p_grid = p.get("grid", 0)
    o.p_tau = p.get("tau", 0.0)
    o.p_sort = p.get("sort", 0)


class Context:
    """One libmcx context bound to a torch-allocated workspace on one GPU."""

    def __init__(self, problem, device=0, record=False, block_size=0, tail_threshold=0,
                 lookahead=0, max_events=None, time_kernels=False, n_gen_max=None,
                 stream=None, precision="fp64", engine="event", persistent=None, flights=0,
                 event_log=0, time_stride=0, rounds=0, lds_tally_min=0, lt_flights=0,
                 workspace=True):
        import torch

        self.problem = problem
        self.device = device
        L = lib()
        self.L = L
        self._keep = []
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        rp = problem["run"]
        o = Options()
        _options(o, precision, device, self.stream, engine, persistent)
        o.block_size = block_size
        o.tail_threshold = tail_threshold
        o.lookahead = lookahead
        o.max_events = rp["max_events"] if max_events is None else max_events
        o.record_histories = int(bool(record))
        o.flights = flights
        o.event_log = event_log
        o.time_stride = time_stride
        o.rounds = rounds
        o.lds_tally_min = lds_tally_min
        o.lt_flights = lt_flights
        self.event_log = event_log
        # True / 1: every event kernel; "advance" / 2: the advance kernels only
        o.time_kernels = 2 if time_kernels in ("advance", 2) else int(bool(time_kernels))
        h = C.c_void_p()
        self._check(L.mcx_create(C.byref(h), C.byref(o)), None)
        self.h = h
        geo = problem["geometry"]
        k = self._keep
        g = _geometry(geo, k)
        self._check(L.mcx_load_geometry(h, C.byref(g)))
        if "ce" in problem:
            d = _ce(problem["ce"], k)
            self._check(L.mcx_load_ce_xs(h, C.byref(d)))
            n_grp = d.n_ebins
        else:
            (n_mat, n_grp), ptrs = _xs(problem["xs"], k)
            self._check(L.mcx_load_mg_xs(h, n_mat, n_grp, *ptrs))
        n_t = 1
        if "time" in problem:
            edges = _arr(problem["time"]["t_edges"], np.float64, k)
            n_t = len(edges) - 1
            if problem["time"].get("speed") is None:
                self._check(L.mcx_load_time_grid(h, n_t, edges.ctypes.data, None, 0))
            else:
                speed = _arr(problem["time"]["speed"], np.float64, k)
                self._check(L.mcx_load_time_grid(h, n_t, edges.ctypes.data, speed.ctypes.data,
                                                 len(speed)))
        s = Source()
        s.seed, s.n_per_gen = rp["seed"], rp["n_per_gen"]
        s.fixed_source, s.problem_id = int(rp["fixed_source"]), rp["problem_id"]
        s.ent_nx, s.ent_ny = rp["ent_nx"], rp["ent_ny"]
        self._check(L.mcx_seed_source(h, C.byref(s)))
        self.n_gen_max = n_gen_max or rp["n_gen"]
        self.workspace = None
        if workspace:
            nbytes = C.c_size_t()
            self._check(L.mcx_workspace_size(h, self.n_gen_max, C.byref(nbytes)))
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8,
                                         device=f"cuda:{device}")
            self._check(L.mcx_bind_workspace(h, self.workspace.data_ptr(), nbytes.value,
                                             self.n_gen_max))
        self.n_bins = geo["nx"] * geo["ny"] * (g.max_rings + 1) * n_grp * n_t
        self.n_per_gen = rp["n_per_gen"]
        self.n_gen = None

    def _check(self, rc, h="self"):
        if rc != 0:
            msg = "" if h is None else self.L.mcx_last_error(self.h).decode()
            raise MCXError(rc, msg)

    def run(self, n_gen=None, n_inactive=None, check=True):
        rp = self.problem["run"]
        n_gen = rp["n_gen"] if n_gen is None else n_gen
        n_inactive = rp["n_inactive"] if n_inactive is None else n_inactive
        rc = self.L.mcx_run_generations(self.h, n_gen, n_inactive)
        self.n_gen = n_gen
        if check:
            self._check(rc)
        return rc

    def run_noalloc(self, n_gen=None, n_inactive=None, check=True):
        """mcx_run_generations_noalloc: the run's workspace in the library's
        static scratch array (no device allocation)."""
        rp = self.problem["run"]
        n_gen = rp["n_gen"] if n_gen is None else n_gen
        n_inactive = rp["n_inactive"] if n_inactive is None else n_inactive
        rc = self.L.mcx_run_generations_noalloc(self.h, n_gen, n_inactive)
        self.n_gen = n_gen
        if check:
            self._check(rc)
        return rc

    def continue_run(self, n_more, check=True):
        rc = self.L.mcx_continue_generations(self.h, n_more)
        if rc in (OK, EGUARD):
            self.n_gen = (self.n_gen or 0) + n_more
        if check:
            self._check(rc)
        return rc

    def checkpoint(self):
        """Bytes of a checkpoint of the last completed run."""
        n = C.c_size_t()
        self._check(self.L.mcx_checkpoint(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.L.mcx_checkpoint(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def restore(self, data, n_gen):
        buf = C.create_string_buffer(bytes(data), len(data))
        self._check(self.L.mcx_restore(self.h, buf, len(data)))
        self.n_gen = n_gen

    def keff(self):
        m, s = np.zeros(3), np.zeros(3)
        pg = np.zeros((self.n_gen, 3))
        self._check(self.L.mcx_get_keff(self.h, m.ctypes.data, s.ctypes.data, pg.ctypes.data))
        return m, s, pg

    def generation_stats(self):
        h = np.zeros(self.n_gen)
        c = np.zeros((self.n_gen, N_CNT), np.int64)
        self._check(self.L.mcx_get_generation_stats(self.h, h.ctypes.data, c.ctypes.data))
        return h, c

    def tallies(self):
        nb = self.n_bins
        out = {k: np.zeros(nb) for k in ("flux_mean", "flux_sigma", "prod_mean", "prod_sigma")}
        self._check(self.L.mcx_get_tallies(self.h, out["flux_mean"].ctypes.data,
                                           out["flux_sigma"].ctypes.data,
                                           out["prod_mean"].ctypes.data,
                                           out["prod_sigma"].ctypes.data, nb))
        return out

    def generation_tallies(self, gen):
        f, p = np.zeros(self.n_bins), np.zeros(self.n_bins)
        self._check(self.L.mcx_get_generation_tallies(self.h, gen, f.ctypes.data, p.ctypes.data,
                                                      self.n_bins))
        return f, p

    def records(self, gen):
        r = np.zeros(self.n_per_gen, RECORD_DTYPE)
        self._check(self.L.mcx_get_records(self.h, gen, r.ctypes.data, self.n_per_gen))
        return r

    def events(self, gen):
        n = self.n_per_gen * self.event_log
        e = np.zeros(n, EVENT_DTYPE)
        self._check(self.L.mcx_get_event_log(self.h, gen, e.ctypes.data, n))
        return e.reshape(self.n_per_gen, self.event_log)

    def bank(self, cap=None):
        n = C.c_int64()
        self._check(self.L.mcx_get_bank(self.h, None, 0, C.byref(n)))
        cap = n.value if cap is None else min(cap, n.value)
        out = np.zeros((cap, 3))
        self._check(self.L.mcx_get_bank(self.h, out.ctypes.data if cap else None, cap,
                                        C.byref(n)))
        return out

    def timing(self):
        t = Timing()
        self._check(self.L.mcx_get_timing(self.h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in Timing._fields_}

    def autotune(self, cache_path=None):
        """Launch configuration with the shortest measured run (persistent
        engine: block, slots, grid, tau, sort; event engine: block, flights,
        lt_flights, tail), swept in the library, optionally cached in a text
        file."""
        t = Tune()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.L.mcx_autotune(self.h, path, C.byref(t)))
        return {name: getattr(t, name) for name, _ in Tune._fields_}

    def diag_math(self, which, values):
        import torch
        x = torch.as_tensor(np.ascontiguousarray(values, dtype=np.float64)).to(
            f"cuda:{self.device}")
        out = torch.empty(2 * len(x) if which == 1 else len(x), dtype=torch.float64,
                          device=x.device)
        self._check(self.L.mcx_diag_math(self.h, which, x.data_ptr(), out.data_ptr(), len(x)))
        o = out.cpu().numpy()
        return o.reshape(-1, 2) if which == 1 else o

    def diag_philox(self, ctr_key):
        import torch
        a = np.ascontiguousarray(ctr_key, dtype=np.uint64).reshape(-1, 6)
        x = torch.as_tensor(a.view(np.int64)).to(f"cuda:{self.device}")
        out = torch.empty((len(a), 4), dtype=torch.int64, device=x.device)
        self._check(self.L.mcx_diag_philox(self.h, x.data_ptr(), out.data_ptr(), len(a)))
        return out.cpu().numpy().view(np.uint64)

    def close(self):
        if getattr(self, "h", None):
            self.L.mcx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(problem, device=0, record=False, per_gen_tallies=False, bank=False, **kw):
    """Run a problem on the GPU; returns a dict shaped like the oracle's."""
    ctx = Context(problem, device=device, record=record, **kw)
    try:
        rc = ctx.run(check=False)
        if rc not in (OK, EGUARD):
            ctx._check(rc)
        m, s, pg = ctx.keff()
        h, c = ctx.generation_stats()
        res = dict(gen_k=pg, gen_entropy=h, gen_counts=c, k_mean=m, k_sigma=s, rc=rc,
                   n_bins=ctx.n_bins, timing=ctx.timing())
        res.update(ctx.tallies())
        G = ctx.n_gen
        if per_gen_tallies:
            res["gen_flux"] = np.zeros((G, ctx.n_bins))
            res["gen_prod"] = np.zeros((G, ctx.n_bins))
            for g in range(G):
                res["gen_flux"][g], res["gen_prod"][g] = ctx.generation_tallies(g)
        if record:
            res["records"] = np.stack([ctx.records(g) for g in range(G)])
        if kw.get("event_log"):
            res["events"] = np.stack([ctx.events(g) for g in range(G)])
        if bank:
            res["bank"] = ctx.bank()
        return res
    finally:
        ctx.close()


class Batch(Context):
    """A batch of independent fixed-source problems run in one persistent
    (or asynchronous-engine) launch (mcx_load_batch / mcx_run_batch)."""

    def __init__(self, problems, device=0, max_events=None, stream=None, precision="fp64",
                 persistent=None, engine="persistent", flights=0):
        import torch

        self.problems = problems
        self.device = device
        L = lib()
        self.L = L
        self._keep = []
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        o = Options()
        if engine not in ("persistent", "async"):
            raise ValueError("a batch runs on the persistent or the asynchronous engine")
        _options(o, precision, device, self.stream, engine, persistent)
        o.flights = flights
        o.max_events = problems[0]["run"]["max_events"] if max_events is None else max_events
        h = C.c_void_p()
        self._check(L.mcx_create(C.byref(h), C.byref(o)), None)
        self.h = h
        arr = (Problem * len(problems))()
        self.n_bins_of = []
        for q, prob in zip(arr, problems):
            rp = prob["run"]
            q.geo = _geometry(prob["geometry"], self._keep)
            (n_mat, n_grp), ptrs = _xs(prob["xs"], self._keep)
            q.n_mat, q.n_grp = n_mat, n_grp
            q.sig_t, q.sig_s, q.nu_sig_f, q.chi = ptrs
            q.seed, q.n_hist, q.problem_id = rp["seed"], rp["n_per_gen"], rp["problem_id"]
            self.n_bins_of.append(q.geo.nx * q.geo.ny * (q.geo.max_rings + 1) * n_grp)
        self._check(L.mcx_load_batch(h, len(problems), arr))
        nbytes = C.c_size_t()
        self._check(L.mcx_workspace_size(h, 1, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=f"cuda:{device}")
        self._check(L.mcx_bind_workspace(h, self.workspace.data_ptr(), nbytes.value, 1))
        self.n_probs = len(problems)

    def run(self, check=True):
        rc = self.L.mcx_run_batch(self.h)
        if check:
            self._check(rc)
        return rc

    def results(self):
        """k[p] = (collision, track-length, absorption) per source particle,
        counts[p][MCX_N_CNT]."""
        k = np.zeros((self.n_probs, 3))
        c = np.zeros((self.n_probs, N_CNT), np.int64)
        self._check(self.L.mcx_get_batch_results(self.h, k.ctypes.data, c.ctypes.data))
        return k, c

    def tallies_of(self, p):
        nb = self.n_bins_of[p]
        f, q = np.zeros(nb), np.zeros(nb)
        self._check(self.L.mcx_get_batch_tallies(self.h, p, f.ctypes.data, q.ctypes.data, nb))
        return f, q
