"""GPU parity of the serving engine (ldd_server_*): every request's result, computed while other
requests join and leave the shared arena, equals the CPU oracle on that request alone, bit for
bit, and equals the single-graph entry point.  Also: queueing when the arena is full, key
rebasing, cancellation, and rejection of bad requests."""
import time

import numpy as np
import pytest

import inputs
import oracle
from graphs import S, small_cases

pytestmark = pytest.mark.gpu


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


def request_mix(seed, count, max_rounds=None):
    """Seeded requests of mixed families and sizes: small exhaustive-style cases, ER and
    random-geometric graphs, grids, RMAT 10-13, each with its own Exp shifts."""
    rng = np.random.default_rng(seed)
    small = small_cases(seed=seed, count=12)
    out = []
    for i in range(count):
        kind = i % 5
        if kind == 0:
            rp, ci, s, name = small[int(rng.integers(len(small)))]
        else:
            n = int(rng.integers(200, 6000))
            gs = int(rng.integers(1, 1 << 30))
            if kind == 1:
                rp, ci = inputs.er(n, float(rng.choice([2.0, 6.0, 12.0])), gs)
            elif kind == 2:
                rp, ci = inputs.rgg(n, 6.0, gs)
            elif kind == 3:
                side = int(np.sqrt(n))
                rp, ci = inputs.grid2d(side, side + 3)
            else:
                rp, ci = inputs.rmat(int(rng.integers(10, 14)), 16, seed=gs)
            beta = float(rng.choice([0.05, 0.1, 0.2, 0.5]))
            s = inputs.make_shifts(rp.size - 1, beta, gs ^ 0x5EED)
            name = f"k{kind}-n{rp.size - 1}-b{beta}"
        if max_rounds is not None and rp.size > 1 and (int(s.max()) >> 20) + 1 > max_rounds:
            s = s % (max_rounds * S // 2)
        out.append((rp, ci, s, name))
    return out


def check(ldd, got, rp, ci, s, name):
    centre_t, cut, info = got
    c_ref, _, cut_ref = oracle.decompose(rp, ci, s)
    c = centre_t.cpu().numpy()
    bad = np.flatnonzero(c != c_ref)
    assert bad.size == 0, f"{name}: {bad.size} centres differ, first at {bad[0]}"
    assert cut == cut_ref, f"{name}: cut {cut} != {cut_ref}"
    assert info["status"] == 0


def test_served_mix_equals_oracle_with_arrivals_in_flight(ldd):
    """Half the requests are submitted, then more arrive while the first are running."""
    reqs = request_mix(seed=3, count=40)
    with ldd.Server(max_vertices=1 << 18, max_arcs=1 << 22, max_slots=16) as srv:
        tensors, tickets = [], []
        for i, (rp, ci, s, name) in enumerate(reqs):
            d = to_dev(rp, ci, s)
            tensors.append(d)
            tickets.append(srv.submit(*d))
            if i == 19:
                first = srv.wait(tickets[0])  # the rest arrive while the mix is in flight
                check(ldd, first, *reqs[0])
        results = {0: first}
        for i in range(1, len(reqs)):
            results[i] = srv.wait(tickets[i])
        for i, (rp, ci, s, name) in enumerate(reqs):
            check(ldd, results[i], rp, ci, s, name)
        info = srv.info()
        log(f"server info {info}")
        assert info["completed"] == sum(1 for rp, _, _, _ in reqs if rp.size > 1)
        assert info["max_active"] > 1


@pytest.mark.parametrize("cfg", [dict(tail_vertices=-1), dict(tail_vertices=1), dict(direction=1),
                                 dict(direction=2), dict(direction=2, tail_vertices=-1), dict(chunk_steps=1),
                                 dict(blocks=5)])
def test_served_schedules_agree_with_oracle(ldd, cfg):
    """Whatever each request's schedule (rounds only, tail from the first step, forced
    directions, chunking, grid size), every served result is the oracle's."""
    reqs = request_mix(seed=21, count=15)
    with ldd.Server(max_vertices=1 << 17, max_arcs=1 << 21, max_slots=6, **cfg) as srv:
        devs = [to_dev(rp, ci, s) for rp, ci, s, _ in reqs]
        tickets = [srv.submit(*d) for d in devs]
        results = [srv.wait(t) for t in tickets]
    for (rp, ci, s, name), res in zip(reqs, results):
        check(ldd, res, rp, ci, s, f"{name} {cfg}")


def test_served_equals_single_graph_path(ldd):
    """The same request, served in a mix, and decomposed alone by ldd_decompose."""
    reqs = request_mix(seed=11, count=10)
    with ldd.Server(max_vertices=1 << 17, max_arcs=1 << 21) as srv:
        devs = [to_dev(rp, ci, s) for rp, ci, s, _ in reqs]
        tickets = [srv.submit(*d) for d in devs]
        served = [srv.wait(t) for t in tickets]
    for (rp, ci, s, name), d, (c_srv, cut_srv, _) in zip(reqs, devs, served):
        c_one, cut_one = ldd.decompose(*d, 0.1)
        assert np.array_equal(c_srv.cpu().numpy(), c_one.cpu().numpy()), name
        assert cut_srv == cut_one, name


def test_small_arena_queues_requests(ldd):
    """Arena for about two requests: the others wait in the queue and still come out right."""
    reqs = []
    for i in range(8):
        rp, ci = inputs.er(1500, 8.0, 100 + i)
        reqs.append((rp, ci, inputs.make_shifts(1500, 0.1, 7 + i), f"er{i}"))
    with ldd.Server(max_vertices=3100, max_arcs=30000, max_slots=8) as srv:
        devs = [to_dev(rp, ci, s) for rp, ci, s, _ in reqs]
        tickets = [srv.submit(*d) for d in devs]
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
    for (rp, ci, s, name), res in zip(reqs, results):
        check(ldd, res, rp, ci, s, name)
    log(f"small arena info {info}")
    assert info["max_active"] <= 2 and info["completed"] == len(reqs)


def test_rebase_keeps_results_exact(ldd):
    """A key range of 64 rounds forces many rebases while requests overlap."""
    reqs = request_mix(seed=5, count=30, max_rounds=31)
    with ldd.Server(max_vertices=1 << 16, max_arcs=1 << 20, max_slots=4, max_rounds=64, chunk_steps=4) as srv:
        assert srv.info()["max_rounds"] == 31
        devs = [to_dev(rp, ci, s) for rp, ci, s, _ in reqs]
        tickets = []
        results = {}
        for i, d in enumerate(devs):
            tickets.append(srv.submit(*d))
            if i % 3 == 2:  # stagger arrivals
                results[i - 2] = srv.wait(tickets[i - 2])
        for i, t in enumerate(tickets):
            if i not in results:
                results[i] = srv.wait(t)
        info = srv.info()
    log(f"rebase info {info}")
    assert info["rebases"] > 0
    for i, (rp, ci, s, name) in enumerate(reqs):
        check(ldd, results[i], rp, ci, s, name)


def test_cancel_queued_request(ldd):
    big = inputs.rmat(14, 16, seed=3)
    small = inputs.grid2d(20, 20)
    with ldd.Server(max_vertices=1 << 16, max_arcs=1 << 20, max_slots=1) as srv:
        d_big = to_dev(*big, inputs.make_shifts(big[0].size - 1, 0.02, 1))
        d_small = [to_dev(*small, inputs.make_shifts(400, 0.2, 10 + i)) for i in range(3)]
        t_big = srv.submit(*d_big)
        t_small = [srv.submit(*d) for d in d_small]
        assert srv.cancel(t_small[2]) is True
        with pytest.raises(ldd.LddError) as e:
            srv.wait(t_small[2])
        assert e.value.status == ldd.ERR_CANCELLED
        srv.wait(t_big)
        for t, d in zip(t_small[:2], d_small[:2]):
            c, cut, _ = srv.wait(t)
            c_ref, _, cut_ref = oracle.decompose(*small, d[2].cpu().numpy())
            assert np.array_equal(c.cpu().numpy(), c_ref) and cut == cut_ref
        with pytest.raises(ldd.LddError):  # a collected ticket is unknown
            srv.cancel(t_big)


def test_bad_requests_fail_alone(ldd):
    """Content errors come back as the request's status; requests beside them are unaffected."""
    import torch
    rp, ci = inputs.grid2d(10, 10)
    s = inputs.make_shifts(100, 0.2, 1)
    bad_ci = ci.copy()
    bad_ci[17] = 100
    bad_rp = rp.copy()
    bad_rp[50] = bad_rp[52]
    neg = s.copy()
    neg[3] = -1
    far = s.copy()
    far[0] = 300 * S
    cases = [((rp, bad_ci, s), ldd.ERR_INVALID_ARG), ((bad_rp, ci, s), ldd.ERR_INVALID_ARG),
             ((rp, ci, neg), ldd.ERR_INVALID_ARG), ((rp, ci, far), ldd.ERR_OVERFLOW)]
    with ldd.Server(max_vertices=1000, max_arcs=10000, max_rounds=256, max_slots=3) as srv:
        assert srv.info()["max_rounds"] == 127
        good = [srv.submit(*to_dev(rp, ci, inputs.make_shifts(100, 0.2, 10 + i))) for i in range(3)]
        bad = [(srv.submit(*to_dev(*arrays)), status) for arrays, status in cases]
        more = [srv.submit(*to_dev(rp, ci, inputs.make_shifts(100, 0.2, 20 + i))) for i in range(3)]
        for t, status in bad:
            with pytest.raises(ldd.LddError) as e:
                srv.wait(t)
            assert e.value.status == status
        for i, t in enumerate(good):
            check(ldd, srv.wait(t), rp, ci, inputs.make_shifts(100, 0.2, 10 + i), f"good {i}")
        for i, t in enumerate(more):
            check(ldd, srv.wait(t), rp, ci, inputs.make_shifts(100, 0.2, 20 + i), f"after {i}")
        brp, bci = inputs.grid2d(40, 40)
        with pytest.raises(ldd.LddError) as e:  # can never fit the arena: refused at submit
            srv.submit(*to_dev(brp, bci, inputs.make_shifts(1600, 0.2, 1)))
        assert e.value.status == ldd.ERR_BUDGET
        # an empty graph completes at once; the server still serves afterwards
        empty = srv.submit(torch.zeros(1, dtype=torch.int32, device="cuda"),
                           torch.zeros(0, dtype=torch.int32, device="cuda"),
                           torch.zeros(0, dtype=torch.int64, device="cuda"))
        c, cut, info = srv.wait(empty)
        assert c.numel() == 0 and cut == 0
        check(ldd, srv.wait(srv.submit(*to_dev(rp, ci, s))), rp, ci, s, "grid after rejects")


def test_poll_until_done(ldd):
    rp, ci = inputs.rmat(12, 16, seed=9)
    s = inputs.make_shifts(rp.size - 1, 0.1, 9)
    with ldd.Server(max_vertices=1 << 14, max_arcs=1 << 18) as srv:
        t = srv.submit(*to_dev(rp, ci, s))
        deadline = time.time() + 60
        got = None
        while got is None and time.time() < deadline:
            got = srv.poll(t)
            time.sleep(0.0005)
        assert got is not None
        check(ldd, got, rp, ci, s, "rmat-12 polled")
        assert got[2]["t_admit"] >= got[2]["t_submit"] and got[2]["t_done"] >= got[2]["t_admit"]


def test_more_requests_than_one_wave_of_slots(ldd):
    """Several hundred requests submitted at once, so that more than one wave's worth of slots
    (64) is on the device together: the per-slot prefix sums of a step are carried from wave to
    wave, and every request still gets exactly its own result."""
    reqs = request_mix(seed=11, count=300)
    with ldd.Server(max_vertices=1 << 22, max_arcs=1 << 24) as srv:
        tensors = [to_dev(rp, ci, s) for rp, ci, s, _ in reqs]
        tickets = [srv.submit(*d) for d in tensors]
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
    log(f"server info {info}")
    for got, (rp, ci, s, name) in zip(results, reqs):
        check(ldd, got, rp, ci, s, name)
    assert info["max_slots"] == 256 and info["max_active"] > 64
