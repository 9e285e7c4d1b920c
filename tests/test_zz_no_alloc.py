"""GPU tests of the allocation-free entry point mcx_run_generations_noalloc:
the workspace lives in the library's static per-device scratch array.  Its
results must equal those of mcx_run_generations on a caller-bound
workspace, bit for bit, on consecutive calls (the second one smaller, so it
runs on what the first one left in the array), and it must refuse runs that
do not fit."""
import numpy as np
import pytest

from paper_2501_05440_amd import mcx
from paper_2501_05440_amd import problems as P

pytestmark = pytest.mark.gpu

KEYS = ("gen_k", "gen_entropy", "gen_counts")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def results(ctx, prob):
    m, s, pg = ctx.keff()
    h, c = ctx.generation_stats()
    out = dict(gen_k=pg, gen_entropy=h, gen_counts=c, k_mean=m, k_sigma=s)
    out.update(ctx.tallies())
    out["records"] = np.stack([ctx.records(g) for g in range(prob["run"]["n_gen"])])
    return out


def same(a, b):
    for k in KEYS + ("k_mean", "k_sigma", "flux_mean", "flux_sigma", "prod_mean", "prod_sigma"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["records"], b["records"])


def test_noalloc_equals_bound_workspace_on_consecutive_calls():
    """Two calls in a row through the C ABI, the second with fewer histories
    (and a different problem shape), each against the caller-bound run."""
    cases = [("lattice", P.lattice_17x17(n_per_gen=20000, n_gen=4, n_inactive=1)),
             ("pin cell", P.pin_cell(n_per_gen=3001, n_gen=3, n_inactive=1)),
             ("lattice fp32", P.lattice_17x17(n_per_gen=7000, n_gen=3, n_inactive=1))]
    for name, prob in cases:
        prec = "fp32" if "fp32" in name else "fp64"
        banner(f"noalloc {name} n={prob['run']['n_per_gen']} {prec}")
        ref_ctx = mcx.Context(prob, record=True, precision=prec)
        ref_ctx.run()
        ref = results(ref_ctx, prob)
        ref_ctx.close()
        ctx = mcx.Context(prob, record=True, precision=prec, workspace=False)
        ctx.run_noalloc()
        got = results(ctx, prob)
        ctx.close()
        same(ref, got)


def test_noalloc_refusals():
    """A run larger than the scratch array is refused with MCX_ENOMEM and the
    byte counts; kernel timing (which creates events) with MCX_EINVAL; a
    context whose run fits still runs afterwards."""
    banner("noalloc refusals")
    big = P.lattice_17x17(n_per_gen=1_000_000, n_gen=2, n_inactive=1)
    ctx = mcx.Context(big, workspace=False)
    rc = ctx.run_noalloc(check=False)
    assert rc == mcx.ENOMEM
    assert "static scratch" in ctx.L.mcx_last_error(ctx.h).decode()
    ctx.close()
    small = P.pin_cell(n_per_gen=2000, n_gen=2, n_inactive=1)
    ctx = mcx.Context(small, workspace=False, time_kernels=True)
    assert ctx.run_noalloc(check=False) == mcx.EINVAL
    ctx.close()
    ctx = mcx.Context(small, workspace=False)
    ctx.run_noalloc()
    k, _, _ = ctx.keff()
    assert np.isfinite(k[0]) and k[0] > 0
    ctx.close()
