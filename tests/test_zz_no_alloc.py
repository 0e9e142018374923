"""The entry point that allocates nothing (ldd_decompose_static): through the C ABI its result
equals ldd_decompose's, bit for bit, on consecutive calls that reuse the library's fixed scratch
array (the second call smaller than the first, so stale contents of the larger call are left
behind), and it refuses inputs beyond its fixed size before any device work."""
import numpy as np
import pytest

import inputs

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


def dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def both(ldd, rp, ci, s, beta, **opts):
    import torch
    d_rp, d_ci, d_s = dev(rp, ci, s)
    want, want_cut = ldd.decompose(d_rp, d_ci, d_s, beta, **opts)
    got = torch.full_like(want, -7)
    cut = ldd.decompose_static(d_rp, d_ci, d_s, beta, centre=got, **opts)
    torch.cuda.synchronize()
    return got.cpu().numpy(), cut, want.cpu().numpy(), want_cut


def test_static_equals_workspace_path_on_consecutive_calls(ldd):
    cases = [("rmat-20 beta 0.05", *inputs.rmat(20, 16, seed=3), 0.05),
             ("grid2d 64x64 beta 0.1", *inputs.grid2d(64, 64), 0.1),
             ("grid3d 100^3 beta 0.02", *inputs.grid3d(100, 100, 100), 0.02),
             ("er 5000 beta 0.3", *inputs.er(5000, 6.0, 9), 0.3)]
    for k, (name, rp, ci, beta) in enumerate(cases):
        s = inputs.make_shifts(rp.size - 1, beta, 11 + k)
        log(f"case {name}: n={rp.size - 1}")
        got, cut, want, want_cut = both(ldd, rp, ci, s, beta)
        assert np.array_equal(got, want), (name, np.flatnonzero(got != want)[:10])
        assert cut == want_cut, (name, cut, want_cut)
    # schedules: top-down only, bottom-up only, no tail, tail from the start
    rp, ci = inputs.rmat(16, 16, seed=5)
    s = inputs.make_shifts(rp.size - 1, 0.1, 5)
    for opts in (dict(direction=1), dict(direction=2), dict(tail_vertices=-1), dict(tail_vertices=1)):
        got, cut, want, want_cut = both(ldd, rp, ci, s, 0.1, **opts)
        assert np.array_equal(got, want) and cut == want_cut, opts


def test_static_largest_size_then_smaller(ldd):
    import torch
    n_max = ldd.STATIC_MAX_VERTICES
    rp, ci = inputs.rmat(20, 8, seed=8)  # exactly 2^20 vertices
    assert rp.size - 1 == n_max
    s = inputs.make_shifts(n_max, 0.1, 8)
    got, cut, want, want_cut = both(ldd, rp, ci, s, 0.1)
    assert np.array_equal(got, want) and cut == want_cut
    rp2, ci2 = inputs.grid2d(30, 31)
    s2 = inputs.make_shifts(rp2.size - 1, 0.2, 9)
    got, cut, want, want_cut = both(ldd, rp2, ci2, s2, 0.2)
    assert np.array_equal(got, want) and cut == want_cut
    # one vertex more than the array holds: refused before any device work
    rp3, ci3 = inputs.from_edges(n_max + 1, [0], [1])
    d_rp, d_ci, d_s = dev(rp3, ci3, np.zeros(n_max + 1, np.int64))
    with pytest.raises(ldd.LddError) as e:
        ldd.decompose_static(d_rp, d_ci, d_s, 0.1, centre=torch.empty(n_max + 1, dtype=torch.int32, device="cuda"))
    assert e.value.status == ldd.ERR_BUDGET
    # shifts spanning more wake rounds than the array's layout holds: refused (the workspace path runs them)
    rp4, ci4 = inputs.grid2d(20, 20)
    s4 = inputs.make_shifts(400, 0.1, 4)
    s4[7] = (9000 << 20) + 5
    d_rp, d_ci, d_s = dev(rp4, ci4, s4)
    with pytest.raises(ldd.LddError) as e:
        ldd.decompose_static(d_rp, d_ci, d_s, 0.1, centre=torch.empty(400, dtype=torch.int32, device="cuda"))
    assert e.value.status == ldd.ERR_BUDGET
    # and the array still gives exact results afterwards
    got, cut, want, want_cut = both(ldd, rp2, ci2, s2, 0.2)
    assert np.array_equal(got, want) and cut == want_cut
