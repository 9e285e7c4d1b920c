#!/usr/bin/env python3
"""Throughput of the event-based Monte Carlo k-eigenvalue path on one MI355X.

One step is one full power iteration of the 17x17-pin, 7-group lattice at
1e7 histories per generation (60 generations, 20 inactive) in FP64 on the
event engine, with the problem data and workspace resident on the GPU.
Prints one JSON line with histories/s (value), events/s, the roofline of
the dominant event kernel (the advance kernel, timed with HIP events on the
run's stream around its launches in the timed steps), the copy-kernel
bandwidth of the device, and the CPU oracle timed on a bounded sample of the
same workload.  Beside them: the same lattice at 1e6 histories per
generation; the FP32-mixed form at 1e7 histories (k difference in pcm with
its paired sigma); the engines side by side (decomposed event kernels, the
paper's monolithic one-segment kernel, the asynchronous global-queue engine,
the persistent LDS-slot engine); the 512-problem fixed-source batch in one
launch against the same problems one at a time; the continuous-energy pin
cell in FP64 and FP32-mixed; and the time-dependent forms (the pulsed
lattice and the 14 MeV pulsed continuous-energy pin cell).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIME_STRIDE = 4  # the timed steps time the advance launches of every 4th generation
# algorithmic bytes of the advance kernel per flight segment (the minimum
# state one flight moves, FP64 multigroup): reads x, y, u, v, w, group, cell,
# counter (52 B), writes x, y, counter, event (24 B), queue traffic 8 B
SEGMENT_BYTES = 84
# the kernel's own accounting per processed particle: the 52-byte bank entry
# read and written (the flux words of the large launches stay in LDS until
# one add per bin and block; the small launches add 16 B per flight)
STATE_BYTES = 52
COUNTERS = os.path.join(ROOT, "profiles", "k_advance_lattice17x17_1e7_counters.md")
KERNEL_SOURCES = ["paper_2501_05440_amd/csrc/mcx_kernels.hip",
                  "paper_2501_05440_amd/csrc/mcx_kernels_common.hpp",
                  "paper_2501_05440_amd/csrc/mcx_device.hpp",
                  "paper_2501_05440_amd/csrc/mcx_math.hpp"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic_per_item():
    """HBM bytes per advanced particle from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line)
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_item"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-per-gen", type=int, default=10_000_000)
    ap.add_argument("--n-gen", type=int, default=60)
    ap.add_argument("--n-inactive", type=int, default=20)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tail", type=int, default=0)
    ap.add_argument("--flights", type=int, default=0,
                    help="flights per particle per advance launch (0 = library default)")
    ap.add_argument("--rounds", type=int, default=0,
                    help="particles per thread of an advance block, refilled lanes "
                         "(0 = library default)")
    ap.add_argument("--lds-tally-min", type=int, default=0,
                    help="live-count bound from which an advance launch stages its flux tally "
                         "in LDS (0 = library default, negative = never)")
    ap.add_argument("--lt-flights", type=int, default=0,
                    help="flights per particle of the LDS-staged advance launches "
                         "(0 = library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="headline: the event engine's launch configuration from the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-gens", type=int, default=4,
                    help="generations of the headline lattice the CPU oracle runs (about 10 s)")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-engines", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-ce", action="store_true")
    ap.add_argument("--no-time", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: a fresh one per run)")
    return ap.parse_args()


def sync():
    import torch
    torch.cuda.synchronize()


def timed_runs(ctx, steps, warmup=1):
    for _ in range(warmup):
        ctx.run()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run()
    sync()
    return (time.perf_counter() - t0) / steps


def copy_peak_gbps():
    """Device-to-device copy of 1 GiB (the copy kernel of the runtime), best
    of 5, counted as bytes read plus bytes written."""
    import torch
    a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = math.inf
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2 * 1024 ** 3 / best / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_breakdown(mcx, prob, **kw):
    """Per-kernel times of one more run with every event kernel timed (the
    events between launches slow a run a little, so the timed runs go
    without them)."""
    ctx = mcx.Context(prob, time_kernels=True, **kw)
    ctx.run()
    t = ctx.timing()
    ctx.close()
    return t


def paired(g32, g64, ni):
    d = g32[ni:, 0] - g64[ni:, 0]
    return float(d.std(ddof=1) / math.sqrt(len(d)))


def engine_leg(mcx, prob, engine, steps=1, **kw):
    ctx = mcx.Context(prob, engine=engine, **kw)
    tune = ctx.autotune() if engine == "persistent" else None
    sec = timed_runs(ctx, steps)
    km, _, _ = ctx.keff()
    _, c = ctx.generation_stats()
    ctx.close()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    out = {"histories_per_s": round(n / sec, 1), "events_per_s": round(float(c[:, 0].sum()) / sec, 1),
           "ms_per_step": round(sec * 1e3, 2), "k_col": round(float(km[0]), 7)}
    if tune:
        out["tuned"] = {k: tune[k] for k in ("block", "slots", "grid", "tau", "sort")}
    return out


def engines_comparison(P, mcx, big):
    """The same problems on every engine (identical histories): decomposed
    event kernels, the paper's monolithic one-segment kernel, the
    asynchronous engine with global per-event-type queues, and the
    persistent engine."""
    out = {}
    c1 = P.lattice_17x17()
    out["lattice_1e6"] = {e: engine_leg(mcx, c1, e) for e in ("event", "monolithic", "async",
                                                              "persistent")}
    log("engines: lattice 1e7 monolithic")
    out["lattice_1e7_monolithic"] = engine_leg(mcx, big, "monolithic")
    c4 = P.ce_pin_cell()
    log("engines: continuous-energy pin cell")
    out["ce_pin_cell"] = {e: engine_leg(mcx, c4, e) for e in ("event", "monolithic")}
    for key, legs in (("lattice_1e6", out["lattice_1e6"]), ("ce_pin_cell", out["ce_pin_cell"])):
        ev = legs["event"]["histories_per_s"]
        for e, r in legs.items():
            r["relative_to_event"] = round(r["histories_per_s"] / ev, 3)
    out["note"] = ("histories per second of each engine on the same problem; every engine gives "
                   "the same histories bit for bit (k_col equal)")
    return out


def batch_comparison(P, mcx, tune_cache, steps):
    """512 fixed-source pin cells in one persistent launch (autotuned) and
    in one asynchronous-engine launch, against the same problems run one at
    a time with the FP64 event engine."""
    import numpy as np
    probs = P.batch_pin_cells()
    n = np.array([q["run"]["n_per_gen"] for q in probs])
    out = {}
    for eng in ("persistent", "async"):
        b = mcx.Batch(probs, engine=eng)
        tune = b.autotune(tune_cache) if eng == "persistent" else None
        b.run()
        sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.run()
        sync()
        sec = (time.perf_counter() - t0) / steps
        k, cnt = b.results()
        b.close()
        out[eng] = {"histories_per_s": round(n.sum() / sec, 1),
                    "events_per_s": round(float(cnt[:, 0].sum()) / sec, 1),
                    "ms_per_batch": round(sec * 1e3, 2), "killed": int(cnt[:, 6].sum())}
        if tune:
            out[eng]["tuned"] = {kk: tune[kk] for kk in ("block", "slots", "grid", "tau", "sort")}
        log(f"batch ({eng}): {sec * 1e3:.1f} ms per launch")
    ctxs = [mcx.Context(q) for q in probs]
    for c in ctxs[:4]:
        c.run()
    sync()
    t0 = time.perf_counter()
    for c in ctxs:
        c.run()
    sync()
    base = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    out["workload"] = ("512 fixed-source 7-group pin cells, own XS and radius each, "
                       f"{int(n.min())}..{int(n.max())} histories (total {int(n.sum())}), one "
                       "launch in a HIP graph, FP64")
    out["one_at_a_time_event_fp64"] = {"histories_per_s": round(n.sum() / base, 1),
                                       "ms": round(base * 1e3, 1)}
    out["speedup_over_one_at_a_time"] = round(base / (out["persistent"]["ms_per_batch"] * 1e-3), 3)
    out["async_speedup_over_one_at_a_time"] = round(base / (out["async"]["ms_per_batch"] * 1e-3), 3)
    return out


def ce_measurement(P, mcx):
    """Continuous-energy pin cell, 1e6 histories x 50 generations (10
    inactive), event engine, FP64 and FP32-mixed on the same streams; the
    per-kernel times come from a separate fully timed run."""
    prob = P.ce_pin_cell()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    ni = prob["run"]["n_inactive"]
    out, gk = {}, {}
    for prec in ("fp64", "fp32"):
        ctx = mcx.Context(prob, precision=prec)
        sec = timed_runs(ctx, 1)
        km, ks, pg = ctx.keff()
        _, c = ctx.generation_stats()
        ctx.close()
        t = kernel_breakdown(mcx, prob, precision=prec)
        gk[prec] = (km, ks, pg)
        out[prec] = {"histories_per_s": round(n / sec, 1),
                     "events_per_s": round(float(c[:, 0].sum()) / sec, 1),
                     "ms_per_step": round(sec * 1e3, 2),
                     "segments_per_history": round(float(c[:, 0].sum()) / n, 3),
                     "k_col": round(float(km[0]), 7), "sigma": round(float(ks[0]), 7),
                     "kernel_ms_per_step": {"advance": round(t["advance_ms"], 2),
                                            "collide": round(t["collide_ms"], 2),
                                            "tail": round(t["tail_ms"], 2)}}
    out["dk_pcm"] = round(float(gk["fp32"][0][0] - gk["fp64"][0][0]) * 1e5, 3)
    out["paired_sigma_pcm"] = round(paired(gk["fp32"][2], gk["fp64"][2], ni) * 1e5, 3)
    out["within_10_pcm"] = abs(out["dk_pcm"]) <= 10.0
    out["speedup_fp32_over_fp64"] = round(out["fp32"]["histories_per_s"] /
                                          out["fp64"]["histories_per_s"], 3)
    out["workload"] = ("continuous-energy pin cell: 10 nuclides x 50,000-point grid, "
                       "1e6 histories/gen x 50 gens (10 inactive), event engine")
    return out


def time_dependent_measurement(P, mcx, cpu):
    """The pulsed 17x17 lattice (1e6 histories x 10 batches, 12 time bins,
    census at 10 us) and the 14 MeV pulsed continuous-energy pin cell (1e6
    histories x 10 batches, 25 time bins, census at 10 us, neutron density
    per bin): FP64 event engine; the oracle on one batch of each."""
    import numpy as np
    out = {}
    for key, prob in (("pulsed_lattice", P.pulsed_lattice()),
                      ("ce_pulsed_pin_cell", P.ce_pulsed_pin_cell())):
        n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
        ctx = mcx.Context(prob)
        sec = timed_runs(ctx, 1)
        _, c = ctx.generation_stats()
        tl = ctx.tallies()
        ctx.close()
        t = kernel_breakdown(mcx, prob)
        r = {"histories_per_s": round(n / sec, 1),
             "events_per_s": round(float(c[:, 0].sum()) / sec, 1),
             "ms_per_step": round(sec * 1e3, 2),
             "segments_per_history": round(float(c[:, 0].sum()) / n, 3),
             "census_fraction": round(float(c[:, 10].sum()) / n, 5),
             "kernel_ms_per_step": {"advance": round(t["advance_ms"], 2),
                                    "collide": round(t["collide_ms"], 2),
                                    "tail": round(t["tail_ms"], 2)}}
        if key == "ce_pulsed_pin_cell":
            nt = len(prob["time"]["t_edges"]) - 1
            dens = tl["prod_mean"].reshape(-1, nt).sum(0)
            r["density_per_time_bin"] = [float(f"{v:.4e}") for v in dens]
            r["time_edges_s"] = [float(f"{v:.4e}") for v in prob["time"]["t_edges"]]
            r["workload"] = ("continuous-energy pin cell driven by a 14 MeV pulse, fission as "
                             "capture, 1e6 histories x 10 batches, 25 time bins to 10 us, "
                             "flux and neutron density per bin, FP64 event engine")
        else:
            r["leak_fraction"] = round(float(c[:, 4].sum()) / n, 5)
            r["workload"] = ("pulsed lattice_17x17_7g: source pulse at t = 0, fission as capture, "
                             "1e6 histories x 10 batches, 12 time bins to 10 us, FP64 event engine")
        if cpu:
            from oracle import oracle as O
            cores = os.cpu_count() or 1
            c0 = time.perf_counter()
            O.run(P.with_run(prob, n_gen=1), n_threads=cores)
            dt = time.perf_counter() - c0
            r["cpu_oracle"] = {"histories_per_s": round(prob["run"]["n_per_gen"] / dt, 1),
                               "cores": cores, "sample": "first batch (1e6 histories)"}
        out[key] = r
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): sharding histories over "
              "several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2501_05440_amd import mcx
    from paper_2501_05440_amd import problems as P

    if not os.path.exists(mcx.LIB_PATH):
        from paper_2501_05440_amd import build as B
        B.build()
    N, G, NI = a.n_per_gen, a.n_gen, a.n_inactive
    prob = P.lattice_17x17(n_per_gen=N, n_gen=G, n_inactive=NI)
    log(f"lattice 17x17, {N} histories x {G} generations, steps={a.steps} warmup={a.warmup}")
    # the timed steps record HIP events around the advance launches of every
    # TIME_STRIDE-th generation (each event between two launches delays the
    # next one a little); the generations are statistically alike
    ctx = mcx.Context(prob, device=0, block_size=a.block, tail_threshold=a.tail,
                      time_kernels="advance", time_stride=TIME_STRIDE, flights=a.flights,
                      rounds=a.rounds, lds_tally_min=a.lds_tally_min, lt_flights=a.lt_flights)
    tuned = None
    if a.autotune:
        tuned = ctx.autotune(a.tune_cache)
        log(f"autotuned: {tuned}")
    for w in range(a.warmup):
        ctx.run()
        log(f"warmup {w + 1}/{a.warmup} done")
    tot = dict(advance_ms=0.0, n_advance=0, advance_items=0, advance_segments=0,
               n_iterations=0)
    segs = 0
    sync()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ctx.run()
        t = ctx.timing()
        for key in tot:
            tot[key] += t[key]
        _, c = ctx.generation_stats()
        segs += int(c[:, 0].sum())
    sync()
    elapsed = time.perf_counter() - t0
    log(f"timed {a.steps} steps: {elapsed / a.steps * 1e3:.1f} ms per step")
    km, ks, g64 = ctx.keff()
    ctx.close()
    histories = a.steps * N * G
    value = histories / elapsed

    # per-kernel breakdown: one more step, outside the timed region, with every
    # event kernel timed
    bctx = mcx.Context(prob, device=0, block_size=a.block, tail_threshold=a.tail,
                       time_kernels=True, flights=a.flights, rounds=a.rounds,
                       lds_tally_min=a.lds_tally_min, lt_flights=a.lt_flights)
    bctx.run()
    brk = bctx.timing()
    bctx.close()

    # roofline of the dominant event kernel, the advance kernel, over the
    # timed steps: algorithmic bytes = 84 B per flight segment x the
    # segments of an average launch
    adv_avg_ms = tot["advance_ms"] / max(1, tot["n_advance"])
    segs_per_launch = tot["advance_segments"] / max(1, tot["n_iterations"])  # every launch
    items_per_launch = tot["advance_items"] / max(1, tot["n_iterations"])
    flights = tot["advance_segments"] / max(1, tot["advance_items"])
    per_launch = SEGMENT_BYTES * segs_per_launch
    achieved = per_launch / (adv_avg_ms * 1e-3) / 1e9 if adv_avg_ms > 0 else 0.0
    own = items_per_launch * 2 * STATE_BYTES
    own_gbs = own / (adv_avg_ms * 1e-3) / 1e9 if adv_avg_ms > 0 else 0.0
    copy_gbs = copy_peak_gbps()
    traffic = None
    tpi = measured_traffic_per_item()
    if tpi is not None:
        traffic = round(tpi * items_per_launch)  # HBM bytes per launch
    roofline = {"bound": "hbm", "kernel": "k_advance_lt / k_advance (the advance step)",
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "bytes_per_segment": SEGMENT_BYTES,
                "segments_per_launch": round(segs_per_launch, 1),
                "avg_launch_us": round(adv_avg_ms * 1e3, 2),
                "timed_launches": int(tot["n_advance"]),
                "timed_generation_stride": TIME_STRIDE,
                "frac_of_copy_peak": round(achieved / copy_gbs, 4),
                "copy_peak_GBps": round(copy_gbs, 1),
                "kernel_accounting": {"bytes_per_item": 2 * STATE_BYTES,
                                      "items_per_launch": round(items_per_launch, 1),
                                      "flights_per_item": round(flights, 4),
                                      "achieved_GBps": round(own_gbs, 1),
                                      "frac": round(own_gbs / HBM_PEAK_GBS, 4)},
                "segments_per_s_in_advance": round(segs_per_launch / (adv_avg_ms * 1e-3), 1)
                if adv_avg_ms > 0 else 0.0,
                "iterations_per_generation": round(tot["n_iterations"] / (a.steps * G), 2),
                "kernel_ms_per_step": {"advance": round(brk["advance_ms"], 2),
                                       "collide": round(brk["collide_ms"], 2),
                                       "tail": round(brk["tail_ms"], 2),
                                       "note": "one extra step with every event kernel timed"}}

    cpu = None
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        cores = os.cpu_count() or 1
        sample = P.with_run(prob, n_gen=a.cpu_gens, n_inactive=a.cpu_gens - 1)
        log(f"cpu oracle: {a.cpu_gens} generations of {N} histories on {cores} threads")
        c0 = time.perf_counter()
        O.run(sample, n_threads=cores)
        dt = time.perf_counter() - c0
        cpu = {"value": round(a.cpu_gens * N / dt, 1), "unit": "histories/s",
               "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"first {a.cpu_gens} generations of the same lattice problem "
                         f"({a.cpu_gens * N} histories, {dt:.1f} s)"}

    import tempfile
    tune_cache = a.tune_cache or os.path.join(tempfile.mkdtemp(), "mcx_tune.txt")
    extras = not a.no_extras
    lat1 = fp32 = engines = batch = ce = td = None
    if extras:
        log("lattice at 1e6 histories per generation")
        c1 = P.lattice_17x17(n_gen=G, n_inactive=NI)
        lat1 = engine_leg(mcx, c1, "event", steps=3)
        lat1["workload"] = f"lattice_17x17_7g, 1e6 histories/gen x {G} gens ({NI} inactive)"
    if extras and not a.no_fp32:
        log(f"FP32-mixed at {N} histories/gen")
        c32 = mcx.Context(prob, precision="fp32")
        sec = timed_runs(c32, 1)
        km32, ks32, g32 = c32.keff()
        c32.close()
        h32 = N * G / sec
        fp32 = {"histories_per_s": round(h32, 1), "ms_per_step": round(sec * 1e3, 2),
                "k_col": round(float(km32[0]), 7),
                "dk_pcm": round(float(km32[0] - km[0]) * 1e5, 3),
                "paired_sigma_pcm": round(paired(g32, g64, NI) * 1e5, 3),
                "speedup_over_fp64": round(h32 / value, 3)}
        fp32["within_10_pcm"] = abs(fp32["dk_pcm"]) <= 10.0
    if extras and not a.no_engines:
        log("engines side by side")
        engines = engines_comparison(P, mcx, prob)
    if extras and not a.no_batch:
        log("512-problem batch")
        batch = batch_comparison(P, mcx, tune_cache, a.steps)
    if extras and not a.no_ce:
        log("continuous-energy pin cell")
        ce = ce_measurement(P, mcx)
    if extras and not a.no_time:
        log("time-dependent forms")
        td = time_dependent_measurement(P, mcx, not a.no_cpu_baseline)

    out = {
        "metric": "histories/s and events/s per MI355X (FP64 vs FP32-mixed, batched) at <=10 pcm "
                  "k-eff error",
        "value": round(value, 1),
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"lattice_17x17_7g: 17x17 pin cells, 3 fuels + moderator, 7 groups, "
                               f"vacuum boundary, {N} histories/gen x {G} gens ({NI} inactive), "
                               f"FP64 event-based",
                   "histories_per_step": N * G, "block_size": a.block or 512,
                   "tail_threshold": a.tail or min(131072, max(4096, N // 8)),
                   "lds_tally_min": a.lds_tally_min or 524288,
                   "flights_per_advance_launch": a.flights or 8,
                   "flights_per_lds_staged_launch": a.lt_flights or min(a.flights or 8, 5)},
        "events_per_s": round(segs / elapsed, 1),
        "segments_per_history": round(segs / histories, 4),
        "k_eff": {"collision": round(float(km[0]), 6), "sigma": round(float(ks[0]), 6)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "lattice_1e6": lat1,
        "fp32_mixed": fp32,
        "engines": engines,
        "batch": batch,
        "continuous_energy": ce,
        "time_dependent": td,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
