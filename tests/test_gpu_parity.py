"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every test calls the C ABI of libldd.so through the Python binding and compares the centre
of every vertex and the cut count with the oracle on the same seeded inputs.  The result is
unique (ties go to the smaller id), so the comparison is exact equality.  Full-size
workloads are compared with stored oracle digests (written by
tests/golden/make_oracle_digests.py, which calls only the oracle), the linear-time
certificate, and per-vertex evaluations of the definition.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import inputs
import oracle
from graphs import S, multigraph, small_cases

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")

# schedules that must all give the same bits: engine (automatic, workgroup, launch, persistent),
# direction policy, grid size, and the label-correcting tail (off, default, or from the first step)
MODES = [
    dict(),
    dict(engine=3),  # one workgroup runs every round
    dict(engine=2),  # one launch per round step over the GPU
    dict(engine=2, direction=1),
    dict(engine=2, direction=2),
    dict(engine=1),
    dict(engine=1, direction=2),
    dict(engine=2, blocks=3),
    dict(engine=2, blocks=7, direction=2),
    dict(engine=2, tail_vertices=-1),
    dict(engine=2, tail_vertices=1),
    dict(engine=4),  # a team of workgroups (one per CU) with a device-memory barrier per round
    dict(engine=4, blocks=7, tail_vertices=1),
    dict(engine=4, blocks=3, tail_vertices=-1),
]


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ldd():
    import torch
    assert torch.cuda.is_available()
    import paper_1307_3692_amd as m
    m.lib()
    return m


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def run(ldd, rp, ci, s, beta=0.1, **opts):
    d_rp, d_ci, d_s = to_dev(rp, ci, s)
    centre, cut, st = ldd.decompose(d_rp, d_ci, d_s, beta, stats=True, **opts)
    return centre.cpu().numpy(), cut, st


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def test_small_graph_families_all_modes(ldd):
    cases = small_cases(seed=1, count=30)
    log(f"{len(cases)} small cases x {len(MODES)} modes")
    for rp, ci, s, name in cases:
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for mode in MODES:
            got, cut, _ = run(ldd, rp, ci, s, **mode)
            assert np.array_equal(got, want_c), (name, mode, np.nonzero(got != want_c)[0][:10])
            assert cut == want_cut, (name, mode)


def test_grid64_beta01_seed1(ldd):
    rp, ci, s, beta = inputs.workload("grid2d-64x64")
    want_c, length, want_cut = oracle.decompose(rp, ci, s)
    for mode in MODES:
        got, cut, st = run(ldd, rp, ci, s, beta, **mode)
        log(f"grid64 {mode}: rounds {st['rounds']} td {st['td_rounds']} bu {st['bu_rounds']} "
            f"tail {st['tail_iters']} cut {cut}")
        assert np.array_equal(got, want_c), mode
        assert cut == want_cut
    assert st["pieces"] == np.count_nonzero(want_c == np.arange(want_c.size))
    assert st["rounds_bound"] == (int(s.max()) >> 20) + 1


def test_deterministic_repeats(ldd):
    rp, ci, s, beta = inputs.workload("rmat-16")
    first = None
    for _ in range(10):
        got, cut, _ = run(ldd, rp, ci, s, beta)
        if first is None:
            first = (got.copy(), cut)
        assert np.array_equal(got, first[0]) and cut == first[1]


def test_tail_stamps_across_calls(ldd):
    """The tail's per-vertex stamps are not cleared between calls (each call tags above every
    earlier tag).  Calls that alternate between graphs of different sizes, with the tail taking
    over from the first step and the engines mixed, keep giving the oracle's bits; the
    persistent engine leaves the stamps in a state the next call must clear."""
    cases = []
    for name in ("rmat-16", "grid2d-64x64", "rmat-18"):
        rp, ci, s, beta = inputs.workload(name)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        cases.append((name, to_dev(rp, ci, s), beta, want_c, want_cut))
    for i in range(12):
        name, d, beta, want_c, want_cut = cases[i % 3]
        mode = dict(tail_vertices=1, engine=1) if i % 4 == 3 else dict(tail_vertices=1 if i % 2 else 8, engine=2)
        centre, cut, st = ldd.decompose(*d, beta, stats=True, **mode)
        got = centre.cpu().numpy()
        log(f"call {i} {name} {mode}: tail sweeps {st['tail_iters']}")
        assert np.array_equal(got, want_c), (i, name, mode, np.count_nonzero(got != want_c))
        assert cut == want_cut


def test_calls_on_alternating_streams(ldd):
    """A call may leave idle round steps queued on its stream when it returns; a next call on
    another stream reuses the same workspace.  Calls alternating between two streams, back to
    back and without synchronising, keep giving the oracle's bits."""
    import torch
    cases = []
    for name in ("rmat-16", "grid2d-64x64", "rmat-18"):
        rp, ci, s, beta = inputs.workload(name)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        cases.append((name, to_dev(rp, ci, s), beta, want_c, want_cut))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i in range(12):
        name, d, beta, want_c, want_cut = cases[i % 3]
        st = streams[i % 2]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            centre, cut = ldd.decompose(*d, beta, stream=st)
            got = centre.cpu().numpy()
        log(f"call {i} {name} on stream {i % 2}")
        assert np.array_equal(got, want_c), (i, name, np.count_nonzero(got != want_c))
        assert cut == want_cut


@pytest.mark.parametrize("name", ["rmat-16", "rmat-18", "grid3d-64", "grid2d-1000"])
def test_medium_workloads_vs_oracle(ldd, name):
    rp, ci, s, beta = inputs.workload(name)
    t = time.time()
    want_c, _, want_cut = oracle.decompose(rp, ci, s)
    log(f"{name}: n={rp.size - 1} nnz={ci.size} oracle {time.time() - t:.2f}s")
    for mode in (dict(), dict(engine=2), dict(engine=2, direction=1), dict(direction=2), dict(engine=1),
                 dict(engine=2, tail_vertices=-1), dict(engine=2, tail_vertices=1), dict(engine=3), dict(engine=4)):
        got, cut, st = run(ldd, rp, ci, s, beta, **mode)
        log(f"  {mode}: rounds {st['rounds']} td {st['td_rounds']} bu {st['bu_rounds']} tail {st['tail_iters']} "
            f"from {st['tail_round']} rounds_ms {st['ms_rounds']:.3f}")
        assert np.array_equal(got, want_c), (mode, np.count_nonzero(got != want_c))
        assert cut == want_cut


def test_automatic_engine_choice(ldd):
    """The automatic engine choice: a sparse graph above 2^15 arcs runs on a team (no frontier
    statistics, one step), a sparse graph with a hub of more than 4096 arcs is refused by the team
    and finishes on the launch engine, and a dense graph (RMAT) or a forced bottom-up policy takes
    the launch engine; every result equals the oracle's.  Run in a process of its own (first
    decompositions of the process) it also checks that the team is sized from the device's
    residency on its first call."""
    from graphs import disjoint_union, path, star
    hub = disjoint_union(star(5001), path(60000))
    cases = [
        ("rgg-50k", inputs.rgg(50000, 6.0, 3), {}, "team"),
        ("star-5000+path-60000", hub, {}, "launch"),
        ("rmat-12", inputs.rmat(12, 16, 0.57, 0.19, 0.19, seed=1, relabel=True), {}, "launch"),
        ("grid2d-300", inputs.grid2d(300, 300), dict(direction=2), "launch"),
        ("grid2d-64", inputs.grid2d(64, 64), {}, "workgroup"),
    ]
    for name, (rp, ci), opts, engine in cases:
        s = inputs.make_shifts(rp.size - 1, 0.05, 7)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        got, cut, st = run(ldd, rp, ci, s, 0.05, **opts)
        log(f"{name} {opts}: steps {st['steps']} blocks {st['blocks']} max_frontier {st['max_frontier']} "
            f"rounds {st['rounds']}")
        assert np.array_equal(got, want_c), (name, np.count_nonzero(got != want_c))
        assert cut == want_cut, name
        if engine == "launch":
            assert st["max_frontier"] > 0, name
        else:
            assert st["max_frontier"] == 0 and st["steps"] == 1, name
            assert (st["blocks"] > 1) == (engine == "team"), name
    # asked for explicitly, a team keeps the hub graph (no degree cap) and still gives the oracle's result
    rp, ci = hub
    s = inputs.make_shifts(rp.size - 1, 0.05, 7)
    want_c, _, want_cut = oracle.decompose(rp, ci, s)
    got, cut, st = run(ldd, rp, ci, s, 0.05, engine=4)
    assert st["max_frontier"] == 0 and st["steps"] == 1 and st["blocks"] > 1
    assert np.array_equal(got, want_c) and cut == want_cut


@pytest.mark.parametrize("kind", ["rgg", "er", "grid"])
def test_team_sizes_and_seeds_vs_oracle(ldd, kind):
    """Teams of 2 to 256 workgroups (their per-round barrier is relaxed: every access another
    member may see in a round is device-scope by itself) on mid-size sparse graphs over several
    graph and shift seeds, with and without the label-correcting tail: every result equals the
    oracle's."""
    for seed in range(3):
        if kind == "rgg":
            rp, ci = inputs.rgg(40000 + 7000 * seed, 6.0, 20 + seed)
        elif kind == "er":
            rp, ci = inputs.er(60000 + 9000 * seed, 5.0, 30 + seed)
        else:
            rp, ci = inputs.grid2d(150 + 31 * seed, 170 + 17 * seed)
        s = inputs.make_shifts(rp.size - 1, 0.03, 40 + seed)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for k, tail in ((2, 0), (5, -1), (37, 1), (128, 0), (256, -1)):
            got, cut, st = run(ldd, rp, ci, s, 0.03, engine=4, blocks=k, tail_vertices=tail)
            assert np.array_equal(got, want_c), (kind, seed, k, tail, np.count_nonzero(got != want_c))
            assert cut == want_cut, (kind, seed, k, tail)
        log(f"{kind} seed {seed}: n={rp.size - 1} rounds {st['rounds']} sweeps {st['tail_iters']}")


def test_pull_rows_finished_by_waves(ldd):
    """An RMAT graph and shifts on which the bottom-up early exit rarely fires (several centres'
    waves meet): most pulled rows run past the per-thread cap and are finished by their wave.
    Every schedule still gives the oracle's bits."""
    rp, ci = inputs.rmat(19, 16, seed=1019)
    s = inputs.make_shifts(rp.size - 1, 0.1, 1044)
    t = time.time()
    want_c, _, want_cut = oracle.decompose(rp, ci, s)
    log(f"rmat-19 beta 0.1: n={rp.size - 1} nnz={ci.size} oracle {time.time() - t:.2f}s")
    for mode in (dict(), dict(direction=2), dict(tail_vertices=1), dict(engine=1)):
        got, cut, st = run(ldd, rp, ci, s, 0.1, **mode)
        log(f"  {mode}: arcs examined / arcs {st['arcs_examined'] / ci.size:.3f}")
        assert np.array_equal(got, want_c), (mode, np.count_nonzero(got != want_c))
        assert cut == want_cut
    assert st["arcs_examined"] > ci.size // 4  # the long-row path was exercised


@pytest.mark.parametrize("kind,n", [("er", 3000), ("rgg", 5000), ("er", 150_000), ("rgg", 200_000)])
def test_batch_graph_kinds_vs_oracle(ldd, kind, n):
    rp, ci = inputs.er(n, 8.0, 77) if kind == "er" else inputs.rgg(n, 6.0, 77)
    for beta in (0.02, 0.3):
        s = inputs.make_shifts(n, beta, 78)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for mode in (dict(), dict(engine=3), dict(engine=4)):
            got, cut, _ = run(ldd, rp, ci, s, beta, **mode)
            assert np.array_equal(got, want_c) and cut == want_cut, mode


def test_tie_heavy_shifts(ldd):
    rng = np.random.default_rng(5)
    rp, ci = inputs.rmat(14, 16, seed=3)
    n = rp.size - 1
    for s in ((rng.integers(0, 6, n) * S).astype(np.int64), np.full(n, 7 * S, np.int64),
              (rng.integers(0, 3, n) * S + rng.integers(0, 2, n)).astype(np.int64)):
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for mode in MODES[:3]:
            got, cut, _ = run(ldd, rp, ci, s, **mode)
            assert np.array_equal(got, want_c) and cut == want_cut


def test_beta_does_not_change_result(ldd):
    rp, ci, s, _ = inputs.workload("grid2d-64x64")
    a, ca, _ = run(ldd, rp, ci, s, 0.1)
    b, cb, _ = run(ldd, rp, ci, s, 0.9)
    assert np.array_equal(a, b) and ca == cb


def full_size(ldd, name, modes):
    with open(GOLDEN) as f:
        gold = json.load(f)[name]
    t = time.time()
    rp, ci, s, beta = inputs.workload(name)
    log(f"{name}: generated n={rp.size - 1} nnz={ci.size} in {time.time() - t:.1f}s")
    assert sha(rp) == gold["sha_row_ptr"] and sha(ci) == gold["sha_col_idx"] and sha(s) == gold["sha_shift"], \
        "input generator output differs from the one the digests were made with"
    for mode in modes:
        got, cut, st = run(ldd, rp, ci, s, beta, **mode)
        log(f"  {mode}: rounds {st['rounds']} td {st['td_rounds']} bu {st['bu_rounds']} tail {st['tail_iters']} "
            f"rounds_ms {st['ms_rounds']:.3f} prep_ms {st['ms_prep']:.3f} cut_ms {st['ms_cut']:.3f}")
        assert sha(got) == gold["sha_centre"], mode
        assert cut == gold["cut"]
    t = time.time()
    code, bad = oracle.certify(rp, ci, s, got)
    log(f"  certificate {code} in {time.time() - t:.1f}s")
    assert code == oracle.OK, bad
    rng = np.random.default_rng(1)
    for v in rng.integers(0, rp.size - 1, 4):
        assert oracle.centre_of(rp, ci, s, int(v))[0] == got[v]


def test_full_size_rmat24(ldd):
    full_size(ldd, "rmat-24", (dict(), dict(direction=1), dict(engine=1), dict(tail_vertices=-1)))


def test_full_size_grid3d_256(ldd):
    full_size(ldd, "grid3d-256", (dict(), dict(engine=1), dict(tail_vertices=-1), dict(engine=4)))


# ------------------------------------------------------------------------------------------
# edge cases and errors
# ------------------------------------------------------------------------------------------
def test_degenerate_graphs(ldd):
    import torch
    # n = 0
    d = torch.zeros(1, dtype=torch.int32, device="cuda")
    c, cut = ldd.decompose(d, torch.zeros(0, dtype=torch.int32, device="cuda"),
                           torch.zeros(0, dtype=torch.int64, device="cuda"), 0.1)
    assert c.numel() == 0 and cut == 0
    # single vertex, no edges, all isolated
    for n in (1, 2, 1000):
        rp, ci = inputs.from_edges(n, [], [])
        s = inputs.make_shifts(n, 0.1, 4)
        got, cut, _ = run(ldd, rp, ci, s)
        assert np.array_equal(got, np.arange(n)) and cut == 0
    # one edge with an exact tie: vertex 1 goes to the smaller id 0
    rp, ci = inputs.from_edges(2, [0], [1])
    got, _, _ = run(ldd, rp, ci, np.array([S + 5, 5], np.int64))
    assert got.tolist() == [0, 0]
    got, _, _ = run(ldd, rp, ci, np.array([5, S + 5], np.int64))
    assert got.tolist() == [0, 1]
    # a star with a hub of high degree (whole-tile and multi-tile rows)
    for leaves in (300, 70_000):
        rp, ci = inputs.from_edges(leaves + 1, np.zeros(leaves, np.int32), np.arange(1, leaves + 1))
        s = inputs.make_shifts(leaves + 1, 0.05, 9)
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for mode in MODES[:3]:
            got, cut, _ = run(ldd, rp, ci, s, **mode)
            assert np.array_equal(got, want_c) and cut == want_cut


def test_self_loops_and_repeated_arcs(ldd):
    """A CSR with self-loops and every edge stored 1-3 times (as the header allows): centres as
    for the simple graph, the cut counting every copy of a cut edge and no self-loop, equal to
    the oracle in every schedule."""
    rng = np.random.default_rng(33)
    cases = []
    for rp, ci, s, name in small_cases(seed=5, count=12)[::4]:
        mrp, mci, _ = multigraph(rng, rp, ci)
        cases.append((mrp, mci, s, "multi-" + name))
    rp, ci = inputs.rmat(14, 16, seed=77)
    mrp, mci, _ = multigraph(rng, rp, ci, max_copies=2, loops=0.05)
    cases.append((mrp, mci, inputs.make_shifts(rp.size - 1, 0.1, 77), "multi-rmat-14"))
    for rp, ci, s, name in cases:
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        for mode in MODES:
            got, cut, _ = run(ldd, rp, ci, s, **mode)
            assert np.array_equal(got, want_c), (name, mode, np.nonzero(got != want_c)[0][:10])
            assert cut == want_cut, (name, mode, cut, want_cut)


def test_errors_are_reported(ldd):
    rp, ci = inputs.grid2d(8, 8)
    s = inputs.make_shifts(64, 0.1, 1)
    bad = s.copy()
    bad[5] = -1
    with pytest.raises(ldd.LddError) as e:
        run(ldd, rp, ci, bad)
    assert e.value.status == ldd.ERR_INVALID_ARG
    # row_ptr not monotone
    rp2 = rp.copy()
    rp2[10] = rp2[11] + 1
    with pytest.raises(ldd.LddError) as e:
        run(ldd, rp2, ci, s)
    assert e.value.status == ldd.ERR_INVALID_ARG
    # column id out of range: caught by the validation pass and by the kernels' own checks
    ci2 = ci.copy()
    ci2[7] = 64
    for validate in (True, False):
        with pytest.raises(ldd.LddError) as e:
            run(ldd, rp, ci2, s, validate=validate)
        assert e.value.status == ldd.ERR_INVALID_ARG
    # a shift range of 2^32 rounds: more than the launch engine takes (ERR_OVERFLOW); the
    # workgroup engine's label-correcting mode for small graphs has no rounds and gives the result
    big = s.copy()
    big[0] = 1 << 52
    with pytest.raises(ldd.LddError) as e:
        run(ldd, rp, ci, big, engine=2)
    assert e.value.status in (ldd.ERR_OVERFLOW,)
    got, cut, _ = run(ldd, rp, ci, big)
    want_c, _, want_cut = oracle.decompose(rp, ci, big)
    assert np.array_equal(got, want_c) and cut == want_cut
    with pytest.raises(ldd.LddError):
        run(ldd, rp, ci, s, beta=0.0)
    # the library still works after errors
    got, cut, _ = run(ldd, rp, ci, s)
    want_c, _, want_cut = oracle.decompose(rp, ci, s)
    assert np.array_equal(got, want_c) and cut == want_cut


def test_batch_entry_matches_single(ldd):
    import torch
    graphs = inputs.batch_graphs(12, seed=3, n_lo=500, n_hi=20_000)
    vo, ao, rps, cis, ss = [0], [0], [], [], []
    for rp, ci, s, beta in graphs:
        vo.append(vo[-1] + rp.size - 1)
        ao.append(ao[-1] + ci.size)
        rps.append(rp)
        cis.append(ci)
        ss.append(s)
    d_rp, d_ci, d_s = to_dev(np.concatenate(rps), np.concatenate(cis), np.concatenate(ss))
    centre, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s)
    centre = centre.cpu().numpy()
    for g, (rp, ci, s, beta) in enumerate(graphs):
        want_c, _, want_cut = oracle.decompose(rp, ci, s)
        assert np.array_equal(centre[vo[g]:vo[g + 1]], want_c), g
        assert cuts[g] == want_cut


def test_many_rounds_fallback_sort(ldd):
    # more than 8192 rounds: the wake-round sort takes its global-atomic path
    rng = np.random.default_rng(12)
    rp, ci = inputs.rgg(20_000, 6.0, 5)
    n = rp.size - 1
    s = rng.integers(0, 3 * S, n).astype(np.int64)
    s[rng.integers(0, n, 50)] = rng.integers(8000 * S, 12000 * S, 50)
    want_c, _, want_cut = oracle.decompose(rp, ci, s)
    for mode in (dict(), dict(tail_vertices=-1), dict(direction=2)):
        got, cut, st = run(ldd, rp, ci, s, **mode)
        assert st["rounds_bound"] > 8192
        assert np.array_equal(got, want_c) and cut == want_cut, mode


def pack(graphs):
    vo, ao, rps, cis, ss = [0], [0], [], [], []
    for rp, ci, s in graphs:
        vo.append(vo[-1] + rp.size - 1)
        ao.append(ao[-1] + ci.size)
        rps.append(rp)
        cis.append(ci)
        ss.append(s)
    return vo, ao, np.concatenate(rps), np.concatenate(cis) if ao[-1] else np.zeros(0, np.int32), np.concatenate(ss)


def test_batch_union_equals_alone_and_oracle(ldd):
    rng = np.random.default_rng(44)
    graphs = [(rp, ci, s) for rp, ci, s, _ in inputs.batch_graphs(40, seed=7, n_lo=200, n_hi=30_000)]
    # degenerate members: an empty graph, an edgeless graph, a single vertex, tie-heavy shifts
    graphs.insert(3, (np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64)))
    rp, ci = inputs.from_edges(50, [], [])
    graphs.insert(7, (rp, ci, inputs.make_shifts(50, 0.1, 3)))
    graphs.insert(11, (np.array([0, 0], np.int32), np.zeros(0, np.int32), np.array([5], np.int64)))
    rp, ci = inputs.grid2d(20, 20)
    graphs.append((rp, ci, (rng.integers(0, 4, 400) * S).astype(np.int64)))
    vo, ao, rp_all, ci_all, s_all = pack(graphs)
    d_rp, d_ci, d_s = to_dev(rp_all, ci_all, s_all)
    want = [oracle.decompose(rp, ci, s) for rp, ci, s in graphs]
    for mode in (dict(), dict(batch_mode=1), dict(batch_mode=3, blocks=5), dict(batch_mode=3, team_arcs=-1),
                 dict(batch_mode=3, team_arcs=64), dict(batch_mode=2),
                 dict(batch_mode=2, direction=2), dict(batch_mode=2, tail_vertices=-1), dict(batch_mode=2, engine=1)):
        centre, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, **mode)
        centre = centre.cpu().numpy()
        for g, (wc, _, wcut) in enumerate(want):
            assert np.array_equal(centre[vo[g]:vo[g + 1]], wc), (mode, g)
            assert cuts[g] == wcut, (mode, g)


def test_batch_teams_equal_oracle(ldd):
    """Graphs split over teams of workgroups (forced by a small team_arcs): many rounds and the
    tail (grid, geometric), few rounds (Erdos-Renyi, RMAT), tie-heavy shifts, teams beside lone
    graphs, teams on a grid of 24 workgroups, and a batch of small graphs where a member's vertex
    slice is empty (200 vertices over 3 members of 128); every graph equals the oracle, with the
    tail on, off, and from the first chance."""
    rng = np.random.default_rng(45)
    big = []
    rp, ci = inputs.grid2d(90, 90)
    big.append((rp, ci, inputs.make_shifts(8100, 0.05, 11)))
    rp, ci = inputs.rgg(20_000, 8.0, 3)
    big.append((rp, ci, inputs.make_shifts(20_000, 0.02, 12)))
    rp, ci = inputs.er(15_000, 10.0, 4)
    big.append((rp, ci, inputs.make_shifts(15_000, 0.1, 13)))
    rp, ci = inputs.rmat(12)
    big.append((rp, ci, inputs.make_shifts(rp.size - 1, 0.2, 14)))
    rp, ci = inputs.grid2d(40, 40)
    big.append((rp, ci, (rng.integers(0, 3, 1600) * S).astype(np.int64)))
    for k in range(6):
        rp, ci = inputs.er(300 + 50 * k, 3.0, 20 + k)
        big.append((rp, ci, inputs.make_shifts(rp.size - 1, 0.1, 30 + k)))
    small = []
    rp, ci = inputs.er(200, 6.0, 5)
    small.append((rp, ci, inputs.make_shifts(200, 0.1, 15)))
    rp, ci = inputs.grid2d(12, 30)
    small.append((rp, ci, inputs.make_shifts(360, 0.1, 16)))
    rp, ci = inputs.from_edges(130, [], [])
    small.append((rp, ci, inputs.make_shifts(130, 0.1, 17)))
    for graphs, modes in ((big, (dict(team_arcs=32), dict(team_arcs=32, tail_vertices=-1),
                                 dict(team_arcs=32, tail_vertices=1), dict(team_arcs=8000),
                                 dict(team_arcs=32, blocks=24))),
                          (small, (dict(team_arcs=32), dict(team_arcs=32, tail_vertices=1)))):
        vo, ao, rp_all, ci_all, s_all = pack(graphs)
        d_rp, d_ci, d_s = to_dev(rp_all, ci_all, s_all)
        want = [oracle.decompose(rp, ci, s) for rp, ci, s in graphs]
        for mode in modes:
            log(f"teams {len(graphs)} graphs {mode}")
            centre, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, batch_mode=3, **mode)
            centre = centre.cpu().numpy()
            for g, (wc, _, wcut) in enumerate(want):
                assert np.array_equal(centre[vo[g]:vo[g + 1]], wc), (mode, g)
                assert cuts[g] == wcut, (mode, g)


def test_batch_team_rejects_bad_column(ldd):
    rp, ci = inputs.rgg(6000, 8.0, 9)
    ci2 = ci.copy()
    ci2[ci.size // 2] = 6000  # out of range, in the middle of the graph (another member's slice)
    graphs = [(rp, ci, inputs.make_shifts(6000, 0.05, 1)), (rp, ci2, inputs.make_shifts(6000, 0.05, 2))]
    vo, ao, rp_all, ci_all, s_all = pack(graphs)
    d_rp, d_ci, d_s = to_dev(rp_all, ci_all, s_all)
    with pytest.raises(ldd.LddError) as e:
        ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, batch_mode=3, team_arcs=256)
    assert e.value.status == ldd.ERR_INVALID_ARG
    vo, ao, rp_all, ci_all, s_all = pack(graphs[:1])
    centre, cuts = ldd.decompose_batch(vo, ao, *to_dev(rp_all, ci_all, s_all), batch_mode=3, team_arcs=256)
    wc, _, wcut = oracle.decompose(rp, ci, graphs[0][2])
    assert np.array_equal(centre.cpu().numpy()[:6000], wc) and cuts[0] == wcut


def test_batch_rejects_bad_local_ids(ldd):
    rp, ci = inputs.grid2d(6, 6)
    ci2 = ci.copy()
    ci2[3] = 36  # local id out of range of its graph (would be valid in the union)
    graphs = [(rp, ci, inputs.make_shifts(36, 0.1, 1)), (rp, ci2, inputs.make_shifts(36, 0.1, 2))]
    vo, ao, rp_all, ci_all, s_all = pack(graphs)
    d_rp, d_ci, d_s = to_dev(rp_all, ci_all, s_all)
    with pytest.raises(ldd.LddError) as e:
        ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s)
    assert e.value.status == ldd.ERR_INVALID_ARG


def test_batch_512_workload_digest(ldd):
    with open(GOLDEN) as f:
        gold = json.load(f)["batch-512"]
    graphs = [(rp, ci, s) for rp, ci, s, _ in inputs.batch_graphs(512, seed=1)]
    vo, ao, rp_all, ci_all, s_all = pack(graphs)
    log(f"batch-512: {vo[-1]} vertices, {ao[-1]} arcs")
    d_rp, d_ci, d_s = to_dev(rp_all, ci_all, s_all)
    for mode in (dict(), dict(batch_mode=2)):  # workgroup engine, disjoint union
        centre, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, **mode)
        assert sha(centre.cpu().numpy()) == gold["sha_centre"], mode
        assert sha(np.array(cuts, np.int64)) == gold["sha_cuts"], mode


def test_tuner_changes_time_only(ldd, tmp_path):
    """ldd_tune searches the engine's knobs by timing; the tuned options give the same bits,
    and a second call is answered from the cache (in the process and in the file)."""
    rp, ci, s, beta = inputs.workload("rmat-16")
    d = to_dev(rp, ci, s)
    cache = str(tmp_path / "tune.txt")
    opts, rep = ldd.tune(*d, cache_path=cache)
    log(f"tuned {opts} {rep}")
    assert rep["runs"] > 0 and rep["from_cache"] == 0 and rep["best_ms"] <= rep["default_ms"]
    c_ref, _, cut_ref = oracle.decompose(rp, ci, s)
    c1, cut1 = ldd.decompose(*d, beta, **opts)
    assert np.array_equal(c1.cpu().numpy(), c_ref) and cut1 == cut_ref
    opts2, rep2 = ldd.tune(*d, cache_path=cache)
    assert rep2["from_cache"] == 1 and opts2 == opts
    with open(cache) as f:
        assert len(f.read().splitlines()) == 1


def test_tuner_on_a_batch(ldd):
    graphs = inputs.batch_graphs(24, seed=5, n_lo=200, n_hi=3000)
    vo, ao = [0], [0]
    for rp, ci, s, _ in graphs:
        vo.append(vo[-1] + rp.size - 1)
        ao.append(ao[-1] + ci.size)
    rp = np.concatenate([g[0] for g in graphs])
    ci = np.concatenate([g[1] for g in graphs])
    s = np.concatenate([g[2] for g in graphs])
    d_rp, d_ci, d_s = to_dev(rp, ci, s)
    opts, rep = ldd.tune(d_rp, d_ci, d_s, vtx_off=vo, arc_off=ao)
    assert rep["runs"] > 0
    centre, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, **opts)
    got = centre.cpu().numpy()
    for g, (grp, gci, gs, _) in enumerate(graphs):
        c_ref, _, cut_ref = oracle.decompose(grp, gci, gs)
        assert np.array_equal(got[vo[g]:vo[g + 1]], c_ref), g
        assert cuts[g] == cut_ref, g
