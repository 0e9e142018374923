"""Unit tests of the seeded input generators (graphs and fixed-point exponential shifts)."""
import math

import numpy as np
import pytest
import scipy.stats

import inputs


def check_csr(rp, ci):
    n = rp.size - 1
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size
    if ci.size:
        assert ci.min() >= 0 and ci.max() < n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert not np.any(src == ci), "self-loop"
    key = src * n + ci
    # sorted ascending within each row and no duplicates
    assert np.all(np.diff(key) > 0)
    # symmetric: the reversed arc set equals the arc set
    rkey = np.sort(ci.astype(np.int64) * n + src)
    assert np.array_equal(rkey, key)


def test_grid2d_counts():
    rp, ci = inputs.grid2d(64, 64)
    assert rp.size - 1 == 4096 and ci.size == 2 * 8064
    check_csr(rp, ci)
    rp, ci = inputs.grid2d(3, 5)
    assert ci.size // 2 == 3 * 4 + 5 * 2
    check_csr(rp, ci)


def test_grid3d_counts():
    rp, ci = inputs.grid3d(16, 16, 16)
    assert rp.size - 1 == 4096 and ci.size // 2 == 3 * 16 * 16 * 15
    check_csr(rp, ci)
    rp, ci = inputs.grid3d(2, 3, 4)
    assert ci.size // 2 == 1 * 3 * 4 + 2 * 2 * 4 + 2 * 3 * 3
    check_csr(rp, ci)


def test_rmat_structure_and_relabel_is_isomorphism():
    rp, ci = inputs.rmat(12, 16, seed=7, relabel=True)
    check_csr(rp, ci)
    rp0, ci0 = inputs.rmat(12, 16, seed=7, relabel=False)
    check_csr(rp0, ci0)
    assert rp.size == rp0.size == 4097
    # relabelling is a bijection of ids: same edge count and degree multiset
    assert ci.size == ci0.size
    assert np.array_equal(np.sort(np.diff(rp)), np.sort(np.diff(rp0)))
    # unrelabelled RMAT puts the heaviest vertex at id 0 (quadrant a is the most likely)
    assert np.argmax(np.diff(rp0)) == 0
    # at most edgefactor * 2^scale undirected edges survive clean-up
    assert ci.size // 2 <= 16 * 4096


def test_rmat_deterministic():
    a = inputs.rmat(10, 8, seed=3)
    b = inputs.rmat(10, 8, seed=3)
    c = inputs.rmat(10, 8, seed=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not (a[1].size == c[1].size and np.array_equal(a[1], c[1]))


def test_er_mean_degree():
    n = 20000
    rp, ci = inputs.er(n, 8.0, seed=11)
    check_csr(rp, ci)
    mean = ci.size / n
    # number of edges ~ Binomial(n(n-1)/2, p): sd of the mean degree is about sqrt(8/n)*sqrt(2)
    assert abs(mean - 8.0) < 6 * math.sqrt(2 * 8.0 / n)


def test_rgg_mean_degree():
    n = 20000
    rp, ci = inputs.rgg(n, 6.0, seed=5)
    check_csr(rp, ci)
    r = math.sqrt(6.0 / (math.pi * n))
    # expected area of a radius-r disk around a uniform point, clipped to the unit square
    area = math.pi * r * r - 8.0 * r ** 3 / 3.0 + r ** 4 / 2.0
    expect = (n - 1) * area
    assert abs(ci.size / n - expect) < 0.15


def test_from_edges_dedup_and_selfloops():
    rp, ci = inputs.from_edges(4, [0, 1, 1, 2, 3, 0], [1, 0, 1, 3, 2, 1])
    check_csr(rp, ci)
    assert ci.tolist() == [1, 0, 3, 2]
    assert rp.tolist() == [0, 1, 2, 3, 4]


def test_shifts_exponential_distribution():
    beta = 0.1
    s = inputs.make_shifts(200_000, beta, seed=1)
    assert s.dtype == np.int64 and s.min() >= 0
    x = (s.astype(np.float64) + 0.5) / inputs.FIX_ONE
    assert abs(x.mean() - 1 / beta) < 6 * (1 / beta) / math.sqrt(s.size)
    stat = scipy.stats.kstest(x, "expon", args=(0, 1 / beta))
    assert stat.pvalue > 1e-4


def test_shifts_integer_log_equals_inversion_formula():
    """The integer-only logarithm gives floor(2^20 * (-ln(1 - U)) / beta) for the stream's
    uniforms U: against libm's log1p in double, every value is within one fixed-point unit
    and nearly all are equal (they differ only where the real value lies within rounding of an
    integer)."""
    for beta, seed in ((0.05, 1), (0.3, 77), (1.7, 5)):
        n = 20000
        s = inputs.make_shifts(n, beta, seed)
        u = np.array([inputs.u01(seed, inputs.TAG_SHIFT, i) for i in range(n)])
        ref = np.floor(-np.log1p(-u) / beta * inputs.FIX_ONE).astype(np.int64)
        diff = s - ref
        assert np.abs(diff).max() <= 1
        assert np.count_nonzero(diff) <= 5


def test_shifts_deterministic_and_prefix_stable():
    a = inputs.make_shifts(1000, 0.05, seed=9)
    b = inputs.make_shifts(2000, 0.05, seed=9)
    assert np.array_equal(a, b[:1000])  # counter-based: draw i does not depend on n
    c = inputs.make_shifts(1000, 0.05, seed=10)
    assert not np.array_equal(a, c)
    # beta only scales: floor(2^20 * E/beta) from the same uniforms
    d = inputs.make_shifts(1000, 0.1, seed=9)
    assert np.all(np.abs(d * 2 - a) <= 2)


def test_batch_recipe_ranges():
    rec = inputs.batch_recipe(512, seed=1)
    assert len(rec) == 512
    ns = np.array([r[1] for r in rec])
    betas = np.array([r[2] for r in rec])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    assert betas.min() >= 0.02 and betas.max() <= 0.3
    assert [r[0] for r in rec[:4]] == ["er", "rgg", "er", "rgg"]
    # log-uniform: the median of log n sits near the middle of the range
    mid = 0.5 * (math.log(1000) + math.log(200_000))
    assert abs(np.median(np.log(ns)) - mid) < 0.5


# ------------------------------------------------------------------------------------------
# shift variants of Sec. 5's closing remarks
# ------------------------------------------------------------------------------------------
def test_integer_shifts_with_permutation_tie_break():
    """Integer parts are those of the Exp(beta) shifts (same draws); the fractional parts encode
    the seeded ranking (rank 0 wins every tie: the largest fraction), distinct while n <= 2^20."""
    for n, beta, seed in ((1, 0.1, 1), (997, 0.1, 3), (20000, 0.05, 8)):
        s = inputs.make_shifts_variant(n, beta, seed, inputs.SHIFTS_INT_PERM)
        e = inputs.make_shifts(n, beta, seed)
        assert np.array_equal(s >> 20, e >> 20)
        rank = inputs.perm_rank(n, seed)
        assert np.array_equal(np.sort(rank), np.arange(n))
        frac = s & ((1 << 20) - 1)
        assert np.array_equal(frac, ((n - 1 - rank) << 20) // n)
        assert np.unique(frac).size == n


def test_shifts_from_permutation_positions():
    """The vertex of rank i takes floor(2^20 (H_n - H_i) / beta): checked against exact rational
    harmonic numbers (within one fixed-point unit, nearly always equal); the values decrease with
    the rank, and their mean is 1/beta (the mean of the exponential order statistics)."""
    from fractions import Fraction
    n, beta, seed = 600, 0.25, 4
    s = inputs.make_shifts_variant(n, beta, seed, inputs.SHIFTS_PERM_ORDER)
    rank = inputs.perm_rank(n, seed)
    by_rank = np.empty(n, np.int64)
    by_rank[rank] = s
    h = [Fraction(0)]
    for j in range(1, n + 1):
        h.append(h[-1] + Fraction(1, j))
    exact = np.array([math.floor((h[n] - h[i]) / Fraction(beta) * (1 << 20)) for i in range(n)], np.int64)
    assert np.abs(by_rank - exact).max() <= 1 and np.count_nonzero(by_rank != exact) <= 3
    assert np.all(np.diff(by_rank) < 0)
    big = inputs.make_shifts_variant(200_000, 0.1, 5, inputs.SHIFTS_PERM_ORDER)
    assert abs(big.mean() / inputs.FIX_ONE - 10.0) < 1e-3


def test_permutation_ranking_is_uniform():
    """Over seeds, the rank of a fixed vertex is uniform over the n positions (chi-square)."""
    n, seeds = 8, 4000
    counts = np.zeros(n)
    for seed in range(seeds):
        counts[inputs.perm_rank(n, 100 + seed)[3]] += 1
    stat = scipy.stats.chisquare(counts)
    assert stat.pvalue > 1e-4
