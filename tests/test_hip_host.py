"""CPU checks of the HIP library: it loads, exports every declared symbol, and
its arithmetic (compiled for the host from the same source as the kernels)
gives the oracle's correctly rounded values."""
import os
import re

import numpy as np
import pytest

from paper_2501_05440_amd import mcx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "mcx.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(mcx_\w+)\(", text, re.M)))


def test_header_declarations_are_bound():
    assert declared() == sorted(mcx.EXPORTS)


def test_header_declarations_are_unique_and_cited():
    """Every entry point is declared once, and the comment in front of it
    cites the paper's passage that defines the operation, says that it is a
    project addition with no passage, or (the allocation-free variant) names
    the callers it is for, those that cannot allocate."""
    text = open(os.path.join(ROOT, "include", "mcx.h")).read()
    names = re.findall(r"^(?:int|void|const char\*)\s+(mcx_\w+)\(", text, re.M)
    assert len(names) == len(set(names)), sorted(n for n in names if names.count(n) > 1)
    decl = re.compile(r"^(?:int|void|const char\*)\s+(mcx_\w+)\(", re.M)
    prev_end = 0
    for m in decl.finditer(text):
        before = text[prev_end:m.start()]
        # the comment block right in front of the declaration
        k = before.rfind("*/")
        assert k >= 0 and before[k + 2:].strip() == "", f"{m.group(1)} has no comment"
        comment = " ".join(before[before.rfind("/*", 0, k):k].split())
        assert ("Sec." in comment or "roject addition" in comment or
                "cannot allocate" in comment), \
            f"{m.group(1)}: the comment cites no passage and is not marked a project addition"
        prev_end = text.index(";", m.end()) + 1


def test_library_exports_every_symbol():
    L = mcx.lib()
    for name in declared():
        assert hasattr(L, name), name


def test_host_math_matches_oracle(oracle):
    rng = np.random.default_rng(31)
    words = rng.integers(0, 2**63, 200000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    xi = ((words >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    got = mcx.host_math(0, xi)
    want = np.array([oracle.cr_log(x) for x in xi])
    assert np.array_equal(got, want)
    cs = mcx.host_math(1, xi)
    want_cs = np.array([oracle.cr_cossin_2pi(x) for x in xi])
    assert np.array_equal(cs, want_cs)
    # the uniform mapping of a 64-bit word
    u = mcx.host_math(3, words.view(np.float64))
    assert np.array_equal(u, np.array([oracle.uniform(int(w)) for w in words[:2000]] +
                                      list(xi[2000:])))


def test_host_math_edges(oracle):
    x = np.array([2.0**-53, 1 - 2.0**-53, 0.5, 0.25, 1e-300, 3.0, 1e300, 5e-324])
    assert np.array_equal(mcx.host_math(0, x), [oracle.cr_log(v) for v in x])
    t = np.array([0.0, 0.25, 0.5, 0.75, 0.125, 2.0**-53, 1 - 2.0**-53, 0.25 + 2.0**-54])
    assert np.array_equal(mcx.host_math(1, t), [oracle.cr_cossin_2pi(v) for v in t])


def test_host_log_next_to_one_and_table_knots(oracle):
    """Arguments 1 - k 2^-53 and 1 + k 2^-52 have logarithms within about
    2^-105 relative of a rounding midpoint; so do arguments next to the
    ends of the reduction interval."""
    k = np.arange(1, 4097, dtype=np.float64)
    x = np.concatenate([1 - k * 2.0**-53, 1 + k * 2.0**-52, 181 / 256 * (1 + k * 2.0**-52),
                        362 / 256 * (1 - k * 2.0**-53), 0.5 - k * 2.0**-54])
    assert np.array_equal(mcx.host_math(0, x), [oracle.cr_log(v) for v in x])


def test_host_math_rejects_bad_selector():
    with pytest.raises(mcx.MCXError):
        mcx.host_math(9, np.ones(3))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and
    says so, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
