#!/usr/bin/env python3
"""Throughput of the event-based Monte Carlo k-eigenvalue path on one MI355X.

One step is one full power iteration of the 17x17-pin, 7-group lattice
(1e6 histories per generation, 60 generations, 20 inactive) in FP64 with the
event engine, with the problem data and workspace resident on the GPU.
Prints one JSON line with histories/s (value), events/s, the roofline of the
dominant event kernel (the advance kernel, timed with HIP events on the
run's stream around each of its launches in the timed steps) and the CPU
oracle timed on a bounded sample of the same workload; beside them the same
lattice on the persistent engine and as one history-based kernel per
generation, the FP64 / FP32-mixed comparison at 1e7 histories per
generation, the 512-problem fixed-source batch in one persistent launch
against the same problems run one at a time, the continuous-energy pin cell
and the pulsed (time-dependent) lattice.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIME_STRIDE = 4  # the timed steps time the advance launches of every 4th generation
# algorithmic bytes per processed particle (FP64 bank entry: x, y, u, v as f64,
# cell, group|sites, draw counter, id, flight count as u32 = 52 B)
STATE_BYTES = 52
TALLY_BYTES_ADV = 16  # one 64-bit fixed-point flux atomic (read-modify-write) per flight
COUNTERS = os.path.join(ROOT, "profiles", "k_advance_lattice17x17_counters.md")
KERNEL_SOURCES = ["paper_2501_05440_amd/csrc/mcx_kernels.hip",
                  "paper_2501_05440_amd/csrc/mcx_kernels_common.hpp",
                  "paper_2501_05440_amd/csrc/mcx_device.hpp",
                  "paper_2501_05440_amd/csrc/mcx_math.hpp"]


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
    ap.add_argument("--n-per-gen", type=int, default=1_000_000)
    ap.add_argument("--n-gen", type=int, default=60)
    ap.add_argument("--n-inactive", type=int, default=20)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tail", type=int, default=0)
    ap.add_argument("--flights", type=int, default=0,
                    help="flights per particle per advance launch (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-gens", type=int, default=40,
                    help="generations of the lattice the CPU oracle runs (about 10-15 s)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the 1e7-history FP64 / FP32-mixed comparison")
    ap.add_argument("--n-fp32", type=int, default=10_000_000)
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-problem batch")
    ap.add_argument("--no-ce", action="store_true", help="skip the continuous-energy pin cell")
    ap.add_argument("--no-time", action="store_true", help="skip the pulsed (time-dependent) lattice")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the lattice on the persistent engine")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: a fresh one per run)")
    return ap.parse_args()


def timed_runs(ctx, steps):
    import torch
    ctx.run()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def fp32_mixed_comparison(P, mcx, n, n_gen, n_inactive):
    """Lattice at n histories per generation: FP64 and FP32-mixed throughput
    and the k-eff difference (pcm) with its standard deviation, and the
    per-pin flux differences."""
    import math

    import numpy as np
    prob = P.lattice_17x17(n_per_gen=n, n_gen=n_gen, n_inactive=n_inactive)
    geo = prob["geometry"]
    cells, per_cell = geo["ny"] * geo["nx"], (geo["radii"].shape[1] + 1) * prob["xs"]["sig_t"].shape[1]
    out = {}
    res = {}
    pins = {}
    for prec in ("fp64", "fp32"):
        ctx = mcx.Context(prob, precision=prec, time_kernels=True)
        sec = timed_runs(ctx, 1)
        km, ks, pg = ctx.keff()
        t = ctx.timing()
        res[prec] = (km, ks, pg)
        # per-pin flux (all rings and groups of a lattice cell) and its sigma
        tl = ctx.tallies()
        pins[prec] = (tl["flux_mean"].reshape(cells, per_cell).sum(axis=1),
                      np.sqrt((tl["flux_sigma"].reshape(cells, per_cell) ** 2).sum(axis=1)))
        ctx.close()
        out[prec] = {"histories_per_s": round(n * n_gen / sec, 1), "ms_per_step": round(sec * 1e3, 2),
                     "k_col": round(float(km[0]), 7), "sigma": round(float(ks[0]), 7)}
        # the advance kernel at this size (direction cosines are binary32 in FP32-mixed)
        state = STATE_BYTES if prec == "fp64" else STATE_BYTES - 8
        items = t["advance_items"] / max(1, t["n_advance"])
        fl = t["advance_segments"] / max(1, t["advance_items"])
        avg_ms = t["advance_ms"] / max(1, t["n_advance"])
        ach = items * (2 * state + TALLY_BYTES_ADV * fl) / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
        out[prec]["k_advance_roofline"] = {"achieved_GBps": round(ach, 1),
                                           "frac": round(ach / HBM_PEAK_GBS, 4),
                                           "items_per_launch": round(items, 1),
                                           "avg_launch_us": round(avg_ms * 1e3, 2)}
    dk = res["fp32"][0][0] - res["fp64"][0][0]
    sig = math.hypot(res["fp32"][1][0], res["fp64"][1][0])
    d = res["fp32"][2][n_inactive:, 0] - res["fp64"][2][n_inactive:, 0]
    out["dk_pcm"] = round(dk * 1e5, 3)
    out["sigma_pcm"] = round(sig * 1e5, 3)
    out["paired_sigma_pcm"] = round(float(d.std(ddof=1) / math.sqrt(len(d))) * 1e5, 3)
    out["speedup_fp32_over_fp64"] = round(out["fp32"]["histories_per_s"] / out["fp64"]["histories_per_s"], 3)
    (f64, s64), (f32, s32) = pins["fp64"], pins["fp32"]
    rel = np.abs(f32 - f64) / f64
    out["pin_flux"] = {"max_rel_diff": float(f"{rel.max():.3e}"),
                       "rms_rel_diff": float(f"{np.sqrt(np.mean(rel ** 2)):.3e}"),
                       "max_rel_sigma_fp64": float(f"{(s64 / f64).max():.3e}"),
                       "mean_abs_diff_over_sigma": round(float(np.mean(np.abs(f32 - f64) / np.hypot(s32, s64))), 3),
                       "pins": int(cells)}
    out["workload"] = f"lattice_17x17_7g, {n} histories/gen x {n_gen} gens ({n_inactive} inactive)"
    return out


def persistent_comparison(P, mcx, prob, event_hps, tune_cache):
    """The lattice on the persistent engine (autotuned): histories/s."""
    ctx = mcx.Context(prob, engine="persistent")
    tune = ctx.autotune(tune_cache)
    sec = timed_runs(ctx, 1)
    km, ks, _ = ctx.keff()
    ctx.close()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    return {"histories_per_s": round(n / sec, 1), "ms_per_step": round(sec * 1e3, 2),
            "speedup_over_event_engine": round(n / sec / event_hps, 3),
            "k_col": round(float(km[0]), 7),
            "tuned": {k: tune[k] for k in ("block", "slots", "grid", "tau", "sort")}}


def monolithic_comparison(P, mcx, prob, event_hps):
    """The paper's monolithic form for comparison: every history of a
    generation run by one history-based kernel (the tail kernel from the
    first flight)."""
    ctx = mcx.Context(prob, tail_threshold=1 << 30)
    sec = timed_runs(ctx, 1)
    ctx.close()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    return {"histories_per_s": round(n / sec, 1), "ms_per_step": round(sec * 1e3, 2),
            "event_engine_speedup": round(event_hps / (n / sec), 3)}


def batch_comparison(P, mcx, tune_cache, steps):
    """512 fixed-source pin cells in one persistent launch (autotuned) against
    the same problems run one at a time with the FP64 event engine."""
    import numpy as np
    import torch
    probs = P.batch_pin_cells()
    n = np.array([q["run"]["n_per_gen"] for q in probs])
    b = mcx.Batch(probs)
    tune = b.autotune(tune_cache)
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    k, cnt = b.results()
    b.close()
    print(f"[bench] batch: {sec * 1e3:.1f} ms per launch; one-at-a-time baseline", file=sys.stderr,
          flush=True)
    ctxs = [mcx.Context(q) for q in probs]
    for c in ctxs[:4]:
        c.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in ctxs:
        c.run()
    torch.cuda.synchronize()
    base = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    return {"workload": "512 fixed-source 7-group pin cells, own XS and radius each, "
                        f"{int(n.min())}..{int(n.max())} histories (total {int(n.sum())}), one "
                        "persistent launch in a HIP graph, FP64",
            "histories_per_s": round(n.sum() / sec, 1),
            "events_per_s": round(float(cnt[:, 0].sum()) / sec, 1),
            "ms_per_batch": round(sec * 1e3, 2),
            "one_at_a_time_event_fp64": {"histories_per_s": round(n.sum() / base, 1),
                                         "ms": round(base * 1e3, 1)},
            "speedup_over_one_at_a_time": round(base / sec, 3),
            "tuned": {kk: tune[kk] for kk in ("block", "slots", "grid", "tau", "sort")},
            "killed": int(cnt[:, 6].sum())}


def ce_measurement(P, mcx, steps):
    """Continuous-energy pin cell, 1e6 histories x 50 generations (10
    inactive), event engine, FP64 and FP32-mixed."""
    import math
    import torch
    prob = P.ce_pin_cell()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    ni = prob["run"]["n_inactive"]
    out, gk = {}, {}
    for prec in ("fp64", "fp32"):
        ctx = mcx.Context(prob, time_kernels=True, precision=prec)
        ctx.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        t = ctx.timing()
        km, ks, pg = ctx.keff()
        _, c = ctx.generation_stats()
        ctx.close()
        gk[prec] = (km, ks, pg)
        out[prec] = {"histories_per_s": round(n / sec, 1),
                     "events_per_s": round(float(c[:, 0].sum()) / sec, 1),
                     "ms_per_step": round(sec * 1e3, 2),
                     "segments_per_history": round(float(c[:, 0].sum()) / n, 3),
                     "k_col": round(float(km[0]), 7), "sigma": round(float(ks[0]), 7),
                     "kernel_ms_per_step": {"advance": round(t["advance_ms"], 2),
                                            "collide": round(t["collide_ms"], 2),
                                            "tail": round(t["tail_ms"], 2)}}
    d = gk["fp32"][2][ni:, 0] - gk["fp64"][2][ni:, 0]
    out["dk_pcm"] = round(float(gk["fp32"][0][0] - gk["fp64"][0][0]) * 1e5, 3)
    out["sigma_pcm"] = round(math.hypot(gk["fp32"][1][0], gk["fp64"][1][0]) * 1e5, 3)
    out["paired_sigma_pcm"] = round(float(d.std(ddof=1) / math.sqrt(len(d))) * 1e5, 3)
    out["speedup_fp32_over_fp64"] = round(out["fp32"]["histories_per_s"] /
                                          out["fp64"]["histories_per_s"], 3)
    out["workload"] = ("continuous-energy pin cell: 10 nuclides x 50,000-point grid, "
                       "1e6 histories/gen x 50 gens (10 inactive), event engine")
    return out


def time_dependent_measurement(P, mcx, steps, cpu):
    """The pulsed 17x17 lattice (fixed source, fission as capture), 1e6
    histories x 10 batches, flux in 12 time bins, census at 10 us: FP64
    event engine, and the oracle on one batch."""
    import torch
    prob = P.pulsed_lattice()
    n = prob["run"]["n_per_gen"] * prob["run"]["n_gen"]
    ctx = mcx.Context(prob, time_kernels=True)
    ctx.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    t = ctx.timing()
    _, c = ctx.generation_stats()
    ctx.close()
    out = {"histories_per_s": round(n / sec, 1),
           "events_per_s": round(float(c[:, 0].sum()) / sec, 1),
           "ms_per_step": round(sec * 1e3, 2),
           "segments_per_history": round(float(c[:, 0].sum()) / n, 3),
           "census_fraction": round(float(c[:, 10].sum()) / n, 5),
           "leak_fraction": round(float(c[:, 4].sum()) / n, 5),
           "kernel_ms_per_step": {"advance": round(t["advance_ms"], 2),
                                  "collide": round(t["collide_ms"], 2),
                                  "tail": round(t["tail_ms"], 2)},
           "workload": "pulsed lattice_17x17_7g: source pulse at t = 0, fission as capture, "
                       "1e6 histories x 10 batches, 12 time bins to 10 us, FP64 event engine"}
    if cpu:
        from oracle import oracle as O
        cores = os.cpu_count() or 1
        c0 = time.perf_counter()
        O.run(P.with_run(prob, n_gen=1), n_threads=cores)
        dt = time.perf_counter() - c0
        out["cpu_oracle"] = {"histories_per_s": round(prob["run"]["n_per_gen"] / dt, 1),
                             "cores": cores, "sample": "first batch (1e6 histories)"}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): sharding histories over "
              "several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2501_05440_amd import mcx
    from paper_2501_05440_amd import problems as P

    if not os.path.exists(mcx.LIB_PATH):
        from paper_2501_05440_amd import build as B
        B.build()
    prob = P.lattice_17x17(n_per_gen=a.n_per_gen, n_gen=a.n_gen, n_inactive=a.n_inactive)
    N, G = a.n_per_gen, a.n_gen
    print(f"[bench] lattice 17x17, {N} histories x {G} generations, steps={a.steps} "
          f"warmup={a.warmup}", file=sys.stderr, flush=True)
    # the timed steps record HIP events around the advance launches of every
    # TIME_STRIDE-th generation (each event between two launches delays the
    # next one a little); the generations are statistically alike
    ctx = mcx.Context(prob, device=0, block_size=a.block, tail_threshold=a.tail,
                      time_kernels="advance", time_stride=TIME_STRIDE, flights=a.flights)
    for w in range(a.warmup):
        ctx.run()
        print(f"[bench] warmup {w + 1}/{a.warmup} done", file=sys.stderr, flush=True)
    tot = dict(advance_ms=0.0, collide_ms=0.0, tail_ms=0.0, n_advance=0, n_collide=0,
               advance_items=0, collide_items=0, advance_segments=0, n_iterations=0, run_ms=0.0)
    segs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ctx.run()
        t = ctx.timing()
        for key in tot:
            tot[key] += t[key]
        _, c = ctx.generation_stats()
        segs += int(c[:, 0].sum())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    km, ks, _ = ctx.keff()
    ctx.close()
    histories = a.steps * N * G
    value = histories / elapsed

    # per-kernel breakdown: one more step, outside the timed region, with every
    # event kernel timed
    bctx = mcx.Context(prob, device=0, block_size=a.block, tail_threshold=a.tail,
                       time_kernels=True, flights=a.flights)
    bctx.run()
    brk = bctx.timing()
    bctx.close()

    # roofline of the dominant event kernel, the advance kernel (the largest
    # summed time of the breakdown step), timed over the timed steps
    adv_avg_ms = tot["advance_ms"] / max(1, tot["n_advance"])
    adv_items = tot["advance_items"] / max(1, tot["n_iterations"])  # every launch
    adv_flights = tot["advance_segments"] / max(1, tot["advance_items"])
    adv_bytes = 2 * STATE_BYTES + TALLY_BYTES_ADV * adv_flights
    name, avg_ms, per_launch = "k_advance", adv_avg_ms, adv_items * adv_bytes
    per_item = adv_bytes
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = None
    tpi = measured_traffic_per_item()
    if tpi is not None:
        traffic = round(tpi * adv_items)  # HBM bytes per launch
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_item": round(per_item, 2),
                "items_per_launch": round(adv_items, 1),
                "avg_launch_us": round(avg_ms * 1e3, 2),
                "timed_launches": int(tot["n_advance"]),
                "timed_generation_stride": TIME_STRIDE,
                "flights_per_advance_item": round(adv_flights, 4),
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
        print(f"[bench] cpu oracle: {a.cpu_gens} generations of {N} histories on {cores} threads",
              file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        O.run(sample, n_threads=cores)
        c1 = time.perf_counter()
        cpu = {"value": round(a.cpu_gens * N / (c1 - c0), 1), "unit": "histories/s",
               "cores": cores, "kind": "oracle",
               "sample": f"first {a.cpu_gens} generations of the same lattice problem "
                         f"({a.cpu_gens * N} histories, {c1 - c0:.1f} s)"}

    import tempfile
    tune_cache = a.tune_cache or os.path.join(tempfile.mkdtemp(), "mcx_tune.txt")
    pers = None
    if not a.no_persistent:
        print("[bench] lattice on the persistent engine", file=sys.stderr, flush=True)
        pers = persistent_comparison(P, mcx, prob, value, tune_cache)
    mono = None
    if not a.no_persistent:
        print("[bench] lattice as one history-based kernel per generation", file=sys.stderr,
              flush=True)
        mono = monolithic_comparison(P, mcx, prob, value)
    batch = None
    if not a.no_batch:
        print("[bench] 512-problem batch", file=sys.stderr, flush=True)
        batch = batch_comparison(P, mcx, tune_cache, a.steps)

    ce = None
    if not a.no_ce:
        print("[bench] continuous-energy pin cell", file=sys.stderr, flush=True)
        ce = ce_measurement(P, mcx, 1)

    td = None
    if not a.no_time:
        print("[bench] pulsed lattice (time-dependent fixed source)", file=sys.stderr, flush=True)
        td = time_dependent_measurement(P, mcx, 1, not a.no_cpu_baseline)

    extra = None
    if not a.no_fp32:
        print(f"[bench] FP64 vs FP32-mixed at {a.n_fp32} histories/gen", file=sys.stderr, flush=True)
        extra = fp32_mixed_comparison(P, mcx, a.n_fp32, G, a.n_inactive)

    out = {
        "metric": "histories/s per MI355X (FP64 event-based, k-eigenvalue power iteration)",
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
                               f"vacuum boundary, {N} histories/gen x {G} gens ({a.n_inactive} "
                               f"inactive), FP64 event-based",
                   "histories_per_step": N * G, "block_size": a.block or 256,
                   "tail_threshold": a.tail or max(4096, N // 8),
                   "flights_per_advance_launch": a.flights or 8},
        "events_per_s": round(segs / elapsed, 1),
        "segments_per_history": round(segs / histories, 4),
        "k_eff": {"collision": round(float(km[0]), 6), "sigma": round(float(ks[0]), 6)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "persistent_engine": pers,
        "monolithic_history_kernel": mono,
        "fp32_mixed": extra,
        "batch": batch,
        "continuous_energy": ce,
        "time_dependent": td,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
