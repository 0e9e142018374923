"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (``oracle/``) computes, for every vertex v, the centre
    argmin_u (2^20 * dist(u,v) - shift_fix[u], u)      (Algorithm 2, Sec. 4; Eq. (1), Sec. 3)
and the cut of Def. 1.1.  These tests check it against
  * brute force: all-pairs unweighted distances from scipy's csgraph plus a lexicographic
    argmin in numpy -- the definition, computed by code the oracle does not use;
  * closed forms for special shift patterns;
  * the structural facts the paper proves: Lemma 4.1 (each vertex's shortest path to its
    centre stays in the piece, so pieces are connected) and the radius bound used in the
    proof of Theorem 1.1 (dist(c(v),v) <= delta_c - delta_v);
  * the statistical claims of Lemma 4.2 (E[max shift] = H_n / beta, all shifts below
    (d+1) ln n / beta w.h.p.) and Corollary 4.5 (an edge is cut with probability at most
    1 - exp(-beta)).
Planted mistakes in the oracle (a dropped tie-break, a sign, an edge length, truncated
shifts) must each fail at least one of these pins.
"""
import math

import numpy as np
import pytest

import inputs
import oracle



from graphs import (S, all_pairs, brute_force, complete, cycle, disjoint_union, multigraph, path,  # noqa: E402
                    random_graph, shift_family, small_cases, star, KINDS)


CASES = small_cases()


# ------------------------------------------------------------------------------------------
# brute force
# ------------------------------------------------------------------------------------------
def test_oracle_matches_brute_force():
    for rp, ci, s, name in CASES:
        c, length, cut = oracle.decompose(rp, ci, s)
        bc, bcut = brute_force(rp, ci, s)
        assert np.array_equal(c, bc), name
        assert cut == bcut, name
        # length[v] = Delta + 2^20 dist(c,v) - shift[c]
        if s.size:
            d = all_pairs(rp, ci)
            expect = s.max() + S * d[c, np.arange(s.size)].astype(np.int64) - s[c]
            assert np.array_equal(length, expect), name


def test_rounds_oracle_matches_brute_force():
    """The bucketed search of Sec. 5 (one integer distance per round) gives the definition's
    centres, lengths and cut on every small case, tie-heavy shifts included."""
    for rp, ci, s, name in CASES:
        c, length, cut = oracle.decompose_rounds(rp, ci, s)
        bc, bcut = brute_force(rp, ci, s)
        assert np.array_equal(c, bc), name
        assert cut == bcut, name
        if s.size:
            d = all_pairs(rp, ci)
            expect = s.max() + S * d[c, np.arange(s.size)].astype(np.int64) - s[c]
            assert np.array_equal(length, expect), name


def test_rounds_oracle_certified_on_larger_graphs():
    """On graphs too large for brute force, the bucketed search passes the certificate and
    agrees with the heap-based search."""
    for rp, ci, s in (inputs.workload("rmat-16")[:3], inputs.workload("grid3d-64")[:3],
                      (*inputs.er(20000, 3.0, 5), inputs.make_shifts(20000, 0.3, 5))):
        c, length, cut = oracle.decompose_rounds(rp, ci, s)
        assert oracle.certify(rp, ci, s, c) == (oracle.OK, -1)
        c2, length2, cut2 = oracle.decompose(rp, ci, s)
        assert np.array_equal(c, c2) and np.array_equal(length, length2) and cut == cut2


def test_centre_of_matches_brute_force():
    for rp, ci, s, name in CASES[::3]:
        n = rp.size - 1
        bc, _ = brute_force(rp, ci, s)
        for v in range(n):
            c, val = oracle.centre_of(rp, ci, s, v)
            assert c == bc[v], (name, v)


def test_hypothesis_random_graphs():
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=150, deadline=None, derandomize=True)
    @hyp.given(st.integers(1, 24).flatmap(lambda n: st.tuples(
        st.just(n),
        st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n),
        st.lists(st.integers(0, 5 * S), min_size=n, max_size=n) |
        st.lists(st.integers(0, 4).map(lambda k: k * S), min_size=n, max_size=n))))
    def run(args):
        n, edges, shifts = args
        src = [e[0] for e in edges]
        dst = [e[1] for e in edges]
        rp, ci = inputs.from_edges(n, src, dst)
        s = np.array(shifts, np.int64)
        c, _, cut = oracle.decompose(rp, ci, s)
        bc, bcut = brute_force(rp, ci, s)
        assert np.array_equal(c, bc) and cut == bcut

    run()


def test_multigraph_self_loops_and_repeated_arcs():
    """Self-loops and repeated edges change no distance, so the centres are those of the simple
    graph (brute force); the cut counts every copy of a cut edge and never a self-loop (Def. 1.1
    counted per stored edge)."""
    rng = np.random.default_rng(21)
    for _ in range(40):
        n = int(rng.integers(2, 30))
        rp, ci = random_graph(rng, n, float(rng.choice([0.1, 0.3])))
        mrp, mci, copies = multigraph(rng, rp, ci)
        s = shift_family(rng, n, str(rng.choice(KINDS)))
        c, _, cut = oracle.decompose(mrp, mci, s)
        bc, _ = brute_force(rp, ci, s)
        assert np.array_equal(c, bc)
        assert cut == sum(k for (u, v), k in copies.items() if bc[u] != bc[v])


# ------------------------------------------------------------------------------------------
# closed forms
# ------------------------------------------------------------------------------------------
def test_no_edges_every_vertex_alone():
    rp, ci = inputs.from_edges(50, [], [])
    s = np.arange(50, dtype=np.int64) * 977
    c, _, cut = oracle.decompose(rp, ci, s)
    assert np.array_equal(c, np.arange(50)) and cut == 0


def test_shifts_below_one_unit_give_singletons():
    # every shift < 2^20: a neighbour's offer 2^20 - s_u > 0 >= -s_v, so each vertex keeps itself
    rng = np.random.default_rng(3)
    for rp, ci in (inputs.grid2d(9, 11), random_graph(rng, 40, 0.2), complete(7)):
        s = rng.integers(0, S, rp.size - 1).astype(np.int64)
        c, _, cut = oracle.decompose(rp, ci, s)
        assert np.array_equal(c, np.arange(rp.size - 1))
        assert cut == ci.size // 2


def test_equal_shifts_give_singletons():
    rp, ci = inputs.grid2d(6, 6)
    c, _, cut = oracle.decompose(rp, ci, np.full(36, 5 * S, np.int64))
    assert np.array_equal(c, np.arange(36)) and cut == ci.size // 2


def test_dominant_shift_takes_connected_graph():
    # delta_z >= 2^20 (ecc(z)+1) + max others: z's value beats every other vertex everywhere
    rp, ci = inputs.grid2d(8, 8)
    rng = np.random.default_rng(5)
    s = rng.integers(0, 3 * S, 64).astype(np.int64)
    z = 27
    s[z] = S * (14 + 1) + s.max()  # eccentricity of any vertex of an 8x8 grid is at most 14
    c, _, cut = oracle.decompose(rp, ci, s)
    assert np.all(c == z) and cut == 0


def test_tie_goes_to_smaller_id():
    # two adjacent vertices with shifts differing by exactly one unit of distance tie
    rp, ci = path(2)
    c, _, _ = oracle.decompose(rp, ci, np.array([S + 5, 5], np.int64))
    assert c.tolist() == [0, 0]  # vertex 1: (2^20 - s0, 0) == (-s1, 1) in key, 0 < 1 wins
    c, _, _ = oracle.decompose(rp, ci, np.array([5, S + 5], np.int64))
    assert c.tolist() == [0, 1]  # vertex 0: own (-s0, 0) ties with (2^20 - s1, 1); 0 < 1 keeps itself


@pytest.mark.parametrize("length,z,D", [(12, 5, 3), (15, 0, 4), (15, 14, 6), (9, 4, 1), (20, 10, 0)])
def test_path_single_bump(length, z, D):
    # path 0-1-..-(L-1); shift D units at z, 0 elsewhere.  v joins z iff
    # 2^20 |v-z| - D 2^20 < 0, or equal and z < v; otherwise v keeps itself.
    rp, ci = path(length)
    s = np.zeros(length, np.int64)
    s[z] = D * S
    c, _, cut = oracle.decompose(rp, ci, s)
    expect = [z if (abs(v - z) < D or (abs(v - z) == D and z < v)) else v for v in range(length)]
    assert c.tolist() == expect
    assert cut == sum(expect[v] != expect[v + 1] for v in range(length - 1))


def test_complete_graph_formula():
    # K_n: every u != v is at distance 1.  Let u*(v) = lex-argmin over u != v of (-s_u, u).
    # Then c(v) = u* when (2^20 - s_u*, u*) < (-s_v, v) lexicographically, else v.
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(2, 12))
        rp, ci = complete(n)
        s = (rng.integers(0, 4, n) * S + rng.integers(0, 2, n) * (trial % 2)).astype(np.int64)
        c, _, _ = oracle.decompose(rp, ci, s)
        for v in range(n):
            others = [(-int(s[u]), u) for u in range(n) if u != v]
            m = min(others)
            ustar = m[1]
            expect = ustar if (S - int(s[ustar]), ustar) < (-int(s[v]), v) else v
            assert c[v] == expect


# ------------------------------------------------------------------------------------------
# structural facts (Lemma 4.1, the radius bound in the proof of Theorem 1.1)
# ------------------------------------------------------------------------------------------
def piece_distances(rp, ci, c):
    """BFS distance from each centre inside its own piece (-1 if unreachable)."""
    n = rp.size - 1
    d = np.full(n, -1, np.int64)
    q = [v for v in range(n) if c[v] == v]
    for v in q:
        d[v] = 0
    head = 0
    while head < len(q):
        u = q[head]
        head += 1
        for w in ci[rp[u]:rp[u + 1]]:
            if d[w] < 0 and c[w] == c[u]:
                d[w] = d[u] + 1
                q.append(w)
    return d


def test_pieces_connected_shortest_paths_inside_and_radius_bound():
    for rp, ci, s, name in CASES:
        n = rp.size - 1
        if n == 0:
            continue
        c, _, _ = oracle.decompose(rp, ci, s)
        assert np.all(c[c] == c), name  # each centre is in its own piece
        dp = piece_distances(rp, ci, c)
        assert np.all(dp >= 0), name  # strong connectivity of each piece
        dg = all_pairs(rp, ci)[c, np.arange(n)]
        assert np.array_equal(dp, dg.astype(np.int64)), name  # Lemma 4.1
        assert np.all(S * dp <= s[c] - s), name  # dist(c,v) - delta_c <= -delta_v


# ------------------------------------------------------------------------------------------
# statistics (Lemma 4.2, Corollary 4.5) on the 64x64 grid at beta = 0.1
# ------------------------------------------------------------------------------------------
def test_statistical_claims_grid64():
    beta, k = 0.1, 200
    rp, ci = inputs.grid2d(64, 64)
    n, m = 4096, ci.size // 2
    maxes, fracs = [], []
    for seed in range(1, k + 1):
        s = inputs.make_shifts(n, beta, seed)
        c, _, cut = oracle.decompose(rp, ci, s)
        dmax = s.max() / S
        maxes.append(dmax)
        fracs.append(cut / m)
        # all shifts below (d+1) ln n / beta with d = 2 (fails with probability <= n^-2)
        assert dmax <= 3 * math.log(n) / beta
        # radius of every piece at most its centre's shift
        dp = piece_distances(rp, ci, c)
        assert np.all(S * dp <= s[c])
    h_n = sum(1.0 / i for i in range(1, n + 1))
    sd = math.sqrt(sum(1.0 / i ** 2 for i in range(1, n + 1))) / beta
    assert abs(np.mean(maxes) - h_n / beta) < 4 * sd / math.sqrt(k)
    se = np.std(fracs, ddof=1) / math.sqrt(k)
    assert np.mean(fracs) <= 1 - math.exp(-beta) + 4 * se


def test_order_statistic_gap_fact():
    # Fact 3.1 at rate beta: the top gap X(n) - X(n-1) is Exp(beta), mean 1/beta
    beta, k = 0.2, 400
    gaps = []
    for seed in range(k):
        s = np.sort(inputs.make_shifts(500, beta, 10_000 + seed))
        gaps.append((s[-1] - s[-2]) / S)
    assert abs(np.mean(gaps) - 1 / beta) < 4 * (1 / beta) / math.sqrt(k)


# ------------------------------------------------------------------------------------------
# the linear-time certificate
# ------------------------------------------------------------------------------------------
def test_certificate_accepts_exact_and_rejects_everything_else():
    rng = np.random.default_rng(21)
    for rp, ci, s, name in CASES:
        n = rp.size - 1
        if n == 0:
            continue
        c, _, _ = oracle.decompose(rp, ci, s)
        assert oracle.certify(rp, ci, s, c)[0] == oracle.OK, name
        # every wrong assignment produced by a planted mistake is rejected
        for mut in oracle.MUTATIONS:
            cm, _, _ = oracle.decompose(rp, ci, s, mutation=mut)
            ok = oracle.certify(rp, ci, s, cm)[0] == oracle.OK
            assert ok == bool(np.array_equal(cm, c)), (name, mut)
        # a single vertex moved to a neighbour's piece is rejected
        src = np.repeat(np.arange(n), np.diff(rp))
        diff = np.nonzero(c[src] != c[ci])[0]
        if diff.size:
            a = diff[rng.integers(0, diff.size)]
            bad = c.copy()
            bad[src[a]] = c[ci[a]]
            assert oracle.certify(rp, ci, s, bad)[0] != oracle.OK, name


def test_certificate_large_rmat():
    rp, ci = inputs.rmat(16, 16, seed=2)
    s = inputs.make_shifts(rp.size - 1, 0.05, 2)
    c, _, cut = oracle.decompose(rp, ci, s)
    assert oracle.certify(rp, ci, s, c)[0] == oracle.OK
    assert oracle.cut(rp, ci, c) == cut
    for v in np.random.default_rng(0).integers(0, rp.size - 1, 20):
        assert oracle.centre_of(rp, ci, s, int(v))[0] == c[v]


# ------------------------------------------------------------------------------------------
# planted mistakes must fail a pin
# ------------------------------------------------------------------------------------------
def pins_fail(mutation):
    failures = []
    for rp, ci, s, name in CASES:
        c, _, cut = oracle.decompose(rp, ci, s, mutation=mutation)
        bc, bcut = brute_force(rp, ci, s)
        if not np.array_equal(c, bc) or cut != bcut:
            failures.append(("brute", name))
            break
    rp, ci = path(2)
    c, _, _ = oracle.decompose(rp, ci, np.array([S + 5, 5], np.int64), mutation=mutation)
    if c.tolist() != [0, 0]:
        failures.append(("tie", ""))
    rp, ci = path(12)
    s = np.zeros(12, np.int64)
    s[5] = 3 * S
    c, _, _ = oracle.decompose(rp, ci, s, mutation=mutation)
    if c.tolist() != [0, 1, 2, 5, 5, 5, 5, 5, 5, 9, 10, 11]:
        failures.append(("bump", ""))
    return failures


def test_pins_pass_on_the_oracle():
    assert pins_fail(oracle.MUT_NONE) == []


@pytest.mark.parametrize("mutation", oracle.MUTATIONS)
def test_planted_mistake_is_caught(mutation):
    assert pins_fail(mutation), f"mutation {mutation} not caught"


def test_bad_arguments_rejected():
    rp, ci = path(3)
    with pytest.raises(oracle.OracleError):
        oracle.decompose(rp, ci, np.array([0, -1, 0], np.int64))
    with pytest.raises(oracle.OracleError):
        oracle.decompose(np.array([0, 1, 1, 5], np.int32), np.array([1, 0, 9, 9, 9], np.int32), np.zeros(3, np.int64))


# ------------------------------------------------------------------------------------------
# the verification bounds of the Las Vegas loop (proof of Theorem 1.1, Sec. 5)
# ------------------------------------------------------------------------------------------
def radius_of(rp, ci, s):
    """Largest distance from a vertex to its centre, from the oracle's lengths."""
    c, length, cut = oracle.decompose(rp, ci, s)
    d = (length - (int(s.max()) - s[c])) >> 20
    return c, int(d.max()), cut


def test_las_vegas_bounds_hold_with_constant_probability():
    """With cut_factor 2 and radius_factor 3, a draw passes both checks with probability at
    least 1/2 (Markov's inequality on E[cut] <= (1 - e^-beta) m, Cor. 4.5; every distance to a
    centre is at most the largest shift, below 3 ln n / beta with probability >= 1 - n^-2,
    Lemma 4.2).  Over 120 seeded draws per graph, far more than half pass."""
    for (rp, ci), beta in ((inputs.grid2d(64, 64), 0.1), (inputs.rmat(12, 16, seed=3), 0.2)):
        n, m = rp.size - 1, ci.size // 2
        ok = 0
        for seed in range(120):
            s = inputs.make_shifts(n, beta, 1000 + seed)
            c, radius, cut = radius_of(rp, ci, s)
            # the radius never exceeds the largest shift (proof of Theorem 1.1)
            assert radius * S <= int(s.max())
            ok += cut <= 2 * beta * m and radius <= 3 * math.log(n) / beta
        assert ok >= 60, ok


# ------------------------------------------------------------------------------------------
# block decomposition by iterated decomposition (Sec. 2, Linial-Saks)
# ------------------------------------------------------------------------------------------
def brute_block_levels(rp, ci, level_shifts):
    """The iteration written with the brute-force decomposition (scipy distances + argmin)."""
    n = rp.size - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    level = np.full(ci.size, -1)
    alive = np.ones(ci.size, bool)
    for L, s in enumerate(level_shifts):
        if not alive.any():
            break
        rp_l, ci_l = inputs.from_edges(n, src[alive], ci[alive])
        c, _ = brute_force(rp_l, ci_l, s)
        inside = alive & (c[src] == c[ci])
        level[inside] = L
        alive &= ~inside
    return level


def test_block_decomposition_matches_brute_force():
    rng = np.random.default_rng(31)
    for _ in range(25):
        n = int(rng.integers(2, 30))
        rp, ci = random_graph(rng, n, float(rng.choice([0.1, 0.3, 0.6])))
        shifts = [shift_family(rng, n, str(rng.choice(KINDS))) for _ in range(12)]
        lv, run, placed = oracle.block_decomposition(rp, ci, shifts)
        assert np.array_equal(lv, brute_block_levels(rp, ci, shifts))
        assert sum(placed) == np.count_nonzero(lv >= 0) // 2


def test_block_decomposition_invariants():
    """Both arcs of an edge share a level; a dominant shift places a connected graph in level 0;
    singleton decompositions (all shifts below one unit) place nothing; with beta = 1/2 the edges
    left shrink geometrically (each level cuts an edge with probability below 1 - e^-1/2 < 0.4,
    Cor. 4.5), so a few dozen levels place all of them."""
    rp, ci = inputs.grid2d(12, 12)
    n = rp.size - 1
    s0 = np.zeros(n, np.int64)
    s0[30] = 100 * S
    lv, run, _ = oracle.block_decomposition(rp, ci, [s0])
    assert run == 1 and np.all(lv == 0)
    lv, run, placed = oracle.block_decomposition(rp, ci, [np.zeros(n, np.int64), s0])
    assert placed[0] == 0 and np.all(lv == 1)
    for (rp, ci) in (inputs.grid2d(40, 40), inputs.rmat(12, 16, seed=6), inputs.er(3000, 6.0, 2)):
        n, m = rp.size - 1, ci.size // 2
        shifts = [inputs.make_shifts(n, 0.5, 500 + L) for L in range(60)]
        lv, run, placed = oracle.block_decomposition(rp, ci, shifts)
        assert np.all(lv >= 0) and run < 60
        src = np.repeat(np.arange(n), np.diff(rp))
        lookup = dict(zip(zip(src.tolist(), ci.tolist()), lv.tolist()))
        assert all(lookup[(v, u)] == l for (u, v), l in lookup.items())
        left = m - np.cumsum(placed)
        assert left[0] <= 0.6 * m and (run < 4 or left[3] <= 0.3 * m)
