"""Pins of the oracle's building blocks against independent definitions.

Each block is checked against something other than itself: numpy's Philox
bit generator, 50-digit mpmath arithmetic, math.fsum, or a closed form.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

M64 = 2**64 - 1


def numpy_block(ctr, key):
    """Philox4x64-10 block at counter ctr from numpy.random.Philox.

    numpy advances its 256-bit counter before producing a block, so the block
    at counter C comes from a generator started at C - 1 (mod 2^256)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % 2**256
    words = [(c >> (64 * i)) & M64 for i in range(4)]
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                          counter=np.array(words, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def test_philox_known_answer(oracle):
    # the Random123 known-answer vector for a zero counter and key
    assert oracle.philox([0, 0, 0, 0], [0, 0]) == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_philox_matches_numpy(oracle):
    rng = np.random.default_rng(7)
    cases = [([0, 5, 3, 1], [1, 2]), ([M64, M64, M64, M64], [M64, M64]),
             ([1, 0, 0, 0], [0, 0])]
    for _ in range(300):
        cases.append(([int(v) for v in rng.integers(0, 2**63, 4, dtype=np.int64)],
                      [int(v) for v in rng.integers(0, 2**63, 2, dtype=np.int64)]))
    for ctr, key in cases:
        assert oracle.philox(ctr, key) == numpy_block(ctr, key), (ctr, key)


def test_uniform_mapping_edges(oracle):
    # (k + 1/2) 2^-52 for the top 52 bits k, exact as a rational number
    assert Fraction(oracle.uniform(0)) == Fraction(1, 2**53)
    assert Fraction(oracle.uniform(M64)) == 1 - Fraction(1, 2**53)
    assert oracle.uniform(M64) < 1.0
    assert Fraction(oracle.uniform(1 << 12)) == Fraction(3, 2**53)
    rng = np.random.default_rng(3)
    for w in rng.integers(0, 2**63, 400, dtype=np.int64):
        w = int(w) * 2 + 1
        assert Fraction(oracle.uniform(w)) == Fraction(2 * (w >> 12) + 1, 2**53)
        assert 0.0 < oracle.uniform(w) < 1.0


def test_stream_draws_are_block_words(oracle):
    seed, tag, pid, gen, prob = 12345, 2, 77, 4, 3
    for d in range(0, 13):
        block = numpy_block([d >> 2, pid, gen, prob], [seed, tag])
        want = float(Fraction(2 * (block[d & 3] >> 12) + 1, 2**53))
        assert oracle.stream_uniform(seed, tag, pid, gen, prob, d) == want


def _cr(x_mp):
    """Round an mpmath value (computed at high precision) to the nearest double."""
    return float(x_mp)


def test_cr_log_against_mpmath(oracle):
    mpmath.mp.prec = 300
    rng = np.random.default_rng(11)
    words = rng.integers(0, 2**63, 3000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    xs = [float(Fraction(2 * (int(w) >> 12) + 1, 2**53)) for w in words]
    xs += [2.0**-53, 1.0 - 2.0**-53, 0.5, 0.25 + 2.0**-53, 1e-300, 0.9999999]
    for x in xs:
        assert oracle.cr_log(x) == _cr(mpmath.log(mpmath.mpf(x))), x


def test_cr_cossin_against_mpmath(oracle):
    mpmath.mp.prec = 300
    rng = np.random.default_rng(12)
    ts = list(rng.uniform(0, 1, 2000)) + [2.0**-53, 0.25 + 2.0**-54, 0.25 - 2.0**-55,
                                           0.5 - 2.0**-53, 0.5 + 2.0**-53, 0.125,
                                           0.75 + 2.0**-53, 1.0 - 2.0**-53, 0.0]
    for t in ts:
        a = 2 * mpmath.pi * mpmath.mpf(t)
        c, s = oracle.cr_cossin_2pi(t)
        assert c == _cr(mpmath.cos(a)), t
        assert s == _cr(mpmath.sin(a)), t


def test_isotropic_direction(oracle):
    rng = np.random.default_rng(5)
    xm = rng.uniform(size=40000)
    xp = rng.uniform(size=40000)
    d = np.array([oracle.isotropic(a, b) for a, b in zip(xm, xp)])
    n = len(d)
    # unit vectors
    assert np.max(np.abs(np.sum(d * d, axis=1) - 1.0)) < 1e-15
    # first and second moments of an isotropic direction
    for k in range(3):
        assert abs(d[:, k].mean()) < 4 * math.sqrt(1 / 3 / n)
        assert abs((d[:, k] ** 2).mean() - 1 / 3) < 4 * math.sqrt(4 / 45 / n)
    # w is exactly 2 xi - 1 and the azimuth exactly 2 pi xi
    u, v, w = oracle.isotropic(0.75, 0.125)
    assert w == 0.5
    mpmath.mp.prec = 200
    c45 = float(mpmath.cos(mpmath.pi / 4))
    assert u == math.sqrt(0.75) * c45
    assert v == math.sqrt(0.75) * c45


def test_sample_cdf(oracle):
    w = np.array([0.1, 0.0, 0.3, 0.6, 0.0])
    rng = np.random.default_rng(9)
    xi = rng.uniform(size=60000)
    idx = np.array([oracle.sample_cdf(x, w) for x in xi])
    counts = np.bincount(idx, minlength=5)
    assert counts[1] == 0 and counts[4] == 0
    expect = w * len(xi)
    chi2 = sum((counts[j] - expect[j]) ** 2 / expect[j] for j in (0, 2, 3))
    assert chi2 < 13.8  # chi^2(2 dof) at p = 1e-3
    # boundaries: first index with xi * total < cum_j
    assert oracle.sample_cdf(2.0**-54, w) == 0
    assert oracle.sample_cdf(0.1, w) == 2  # 0.1 * 1.0 is not < 0.1
    assert oracle.sample_cdf(1.0 - 2.0**-54, w) == 3
    assert oracle.sample_cdf(0.5, np.array([0.0, 0.0, 2.0])) == 2


def test_comb(oracle):
    for n, m, xi0 in [(1000, 1000, 0.3), (1000, 437, 0.91), (1000, 2401, 0.05), (7, 1, 0.5)]:
        idx = oracle.comb(n, m, xi0)
        assert idx.min() >= 0 and idx.max() <= m - 1
        assert np.all(np.diff(idx) >= 0)
        if m <= n:
            c = np.bincount(idx, minlength=m)
            assert set(np.unique(c)) <= {n // m, -(-n // m)}
        else:
            assert len(np.unique(idx)) == n
    assert np.array_equal(oracle.comb(50, 50, 0.999), np.arange(50))


def test_entropy(oracle):
    assert oracle.entropy(np.full(64, 10), 640) == pytest.approx(6.0, abs=1e-15)
    assert oracle.entropy(np.array([0, 5, 0]), 5) == 0.0
    assert oracle.entropy(np.array([1, 1, 2]), 4) == pytest.approx(1.5, abs=1e-15)


def test_neumaier_against_fsum(oracle):
    rng = np.random.default_rng(2)
    v = np.concatenate([rng.uniform(0, 1, 10000) * 1e10, rng.uniform(0, 1, 10000) * 1e-6,
                        [1e16, 1.0, -1e16]])
    rng.shuffle(v)
    exact = math.fsum(v)
    got = oracle.neumaier(v)
    assert abs(got - exact) <= 2 * math.ulp(exact)


# ---------------------------------------------------------------------------
# distances
# ---------------------------------------------------------------------------

def test_dist_plane(oracle):
    inf = float("inf")
    assert oracle.dist_plane(0.2, 0.0, 1.0, 0.5) == (1.0 - 0.2) / 0.5
    assert oracle.dist_plane(0.2, 0.0, 1.0, -0.25) == (0.0 - 0.2) / -0.25
    assert oracle.dist_plane(0.2, 0.0, 1.0, 0.0) == inf
    assert oracle.dist_plane(1.0 + 1e-16, 0.0, 1.0, 0.3) == 0.0  # past the plane
    assert oracle.dist_plane(-1e-17, 0.0, 1.0, -0.3) == 0.0


def _cyl_exact(dx, dy, u, v, r, inside):
    """Smallest positive intersection distance in 60-digit arithmetic, with the
    same logical side convention (None = miss)."""
    mpmath.mp.dps = 60
    dx, dy, u, v, r = map(mpmath.mpf, (dx, dy, u, v, r))
    a = u * u + v * v
    if a == 0:
        return None
    k = dx * u + dy * v
    c = dx * dx + dy * dy - r * r
    c = min(c, 0) if inside else max(c, 0)
    disc = k * k - a * c
    if disc < 0:
        return None
    roots = [(-k - mpmath.sqrt(disc)) / a, (-k + mpmath.sqrt(disc)) / a]
    if inside:
        return max(roots[1], mpmath.mpf(0))
    pos = [t for t in roots if t >= 0]
    if k >= 0 or not pos:
        return None
    return min(pos)


def test_dist_cylinder_random_rays(oracle):
    rng = np.random.default_rng(21)
    r = 0.54
    worst = 0.0
    for _ in range(4000):
        inside = rng.uniform() < 0.5
        rad = r * math.sqrt(rng.uniform()) if inside else rng.uniform(r, 0.63 * math.sqrt(2))
        th = rng.uniform(0, 2 * math.pi)
        dx, dy = rad * math.cos(th), rad * math.sin(th)
        w = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * math.pi)
        s = math.sqrt(1 - w * w)
        u, v = s * math.cos(ph), s * math.sin(ph)
        got = oracle.dist_cylinder(dx, dy, u, v, r, inside)
        want = _cyl_exact(dx, dy, u, v, r, inside)
        if want is None:
            assert got == float("inf")
            continue
        want = float(want)
        assert math.isfinite(got)
        k = dx * u + dy * v
        c = dx * dx + dy * dy - r * r
        disc = k * k - (u * u + v * v) * c
        # first-order rounding bound: c carries ~3 ulp of r^2, divided by the
        # root's denominator sqrt(disc) (the near-surface, grazing cases)
        eps = 2.0**-53
        bound = 8 * eps * want + 4 * eps * (dx * dx + dy * dy + r * r) / max(math.sqrt(max(disc, 0.0)), 1e-300)
        assert abs(got - want) <= bound, (dx, dy, u, v, inside, got, want)
        # well-conditioned rays (away from the surface, not grazing): within 4 ulp
        if (dx * dx + dy * dy + r * r) < 2 * abs(c) and disc > 0.05:
            worst = max(worst, abs(got - want) / math.ulp(want))
    assert worst <= 4.0, worst


def test_dist_cylinder_adversarial(oracle):
    inf = float("inf")
    r = 0.54
    # axial flight: no intersection
    assert oracle.dist_cylinder(0.1, 0.2, 0.0, 0.0, r, True) == inf
    # on the surface, inside, moving outward: zero distance
    assert oracle.dist_cylinder(r, 0.0, 1.0, 0.0, r, True) == 0.0
    # on the surface, inside, moving inward: the chord 2r
    assert oracle.dist_cylinder(r, 0.0, -1.0, 0.0, r, True) == pytest.approx(2 * r, rel=1e-15)
    # on the surface, outside (logically), moving inward: zero distance
    assert oracle.dist_cylinder(r, 0.0, -1.0, 0.0, r, False) == 0.0
    # outside moving away: miss
    assert oracle.dist_cylinder(0.6, 0.0, 1.0, 0.0, r, False) == inf
    # outside, tangent ray: grazing hit at the tangent point or a miss, never negative
    t = oracle.dist_cylinder(-1.0, r, 1.0, 0.0, r, False)
    assert t == inf or abs(t - 1.0) < 1e-7
    # position rounded to the wrong side is clamped to its logical side
    eps = 1e-15
    t = oracle.dist_cylinder(r + eps, 0.0, 1.0, 0.0, r, True)
    assert t == 0.0
    t = oracle.dist_cylinder(r - eps, 0.0, -1.0, 0.0, r, False)
    assert t == 0.0
    # slanted 3D direction: path length scales with 1 / sqrt(u^2 + v^2)
    s = math.sqrt(1 - 0.8**2)
    t = oracle.dist_cylinder(0.0, 0.0, s, 0.0, r, True)
    assert t == pytest.approx(r / s, rel=1e-15)
