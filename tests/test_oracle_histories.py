"""The oracle's first-generation histories of a list of ids (orc_histories).

A first-generation history depends on nothing but the problem, the seed and
its id (its source point is sampled from its own stream, and k_used is 1), so
each listed history must get exactly the record the whole run gives it: for
the multigroup lattice, the continuous-energy pin cell, given start states and
the pulsed lattice, with ids in any order, repeated, and the last one of the
generation.  This is what lets a run too large for the oracle be checked
history by history on a sample.
"""
import math

import numpy as np
import pytest

from paper_2501_05440_amd import problems as P


def _ids(n):
    return np.array([n - 1, 0, 7, n // 2, 1, 7, n - 2, 3 * n // 4, 123 % n], np.int64)


def _same(sub, full):
    assert sub.dtype == full.dtype
    for f in full.dtype.names:
        assert np.array_equal(sub[f], full[f]), f


def test_lattice_histories_match_the_whole_run(oracle):
    n = 3000
    prob = P.lattice_17x17(n_per_gen=n, n_gen=1, n_inactive=0, seed=31)
    full = oracle.run(prob, records=True)["records"][0]
    ids = _ids(n)
    _same(oracle.histories(prob, ids), full[ids])
    # a different seed gives different histories: the subset follows the seed
    other = oracle.histories(P.with_run(prob, seed=32), ids)
    assert not np.array_equal(other["n_seg"], full[ids]["n_seg"])


def test_continuous_energy_histories_match_the_whole_run(oracle):
    n = 600
    prob = P.ce_pin_cell(n_per_gen=n, n_gen=1, n_inactive=0, seed=33,
                         data=P.ce_data(n_pts=4000, n_res=40, n_ebins=20))
    full = oracle.run(prob, records=True)["records"][0]
    ids = _ids(n)
    _same(oracle.histories(prob, ids), full[ids])


def test_given_start_states_and_the_pulsed_lattice(oracle):
    n = 1000
    prob = P.pulsed_lattice(n_per_gen=n, n_gen=1, seed=34)
    full = oracle.run(prob, records=True)["records"][0]
    ids = _ids(n)
    _same(oracle.histories(prob, ids), full[ids])

    rng = np.random.default_rng(35)
    geo = prob["geometry"]
    w = geo["nx"] * geo["pitch"]
    mu = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    s = np.sqrt(1 - mu * mu)
    st = np.stack([geo["x0"] + rng.uniform(0.01, 0.99, n) * w,
                   geo["y0"] + rng.uniform(0.01, 0.99, n) * w,
                   s * np.cos(phi), s * np.sin(phi), mu,
                   rng.integers(0, 7, n).astype(float)], axis=1)
    lat = P.lattice_17x17(n_per_gen=n, n_gen=1, n_inactive=0, seed=36)
    full = oracle.run(lat, records=True, ext_state=st)["records"][0]
    _same(oracle.histories(lat, ids, ext_state=st), full[ids])


def test_bad_lists_are_refused(oracle):
    prob = P.lattice_17x17(n_per_gen=100, n_gen=1, n_inactive=0, seed=37)
    assert len(oracle.histories(prob, np.zeros(0, np.int64))) == 0
    for bad in ([100], [-1]):
        with pytest.raises(oracle.OracleError):
            oracle.histories(prob, bad)
