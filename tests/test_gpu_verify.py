"""GPU: the library's shift sampler and the Las Vegas decomposition (proof of Theorem 1.1,
Sec. 5).  The device sampler equals the host sampler (and so the seeded input generator) bit
for bit; the verified decomposition's accepted draw is exactly the oracle's decomposition of
those shifts, with the cut and the largest distance to a centre it reports equal to the
oracle's, and its accept / reject decision equal to the bounds evaluated on the CPU."""
import math

import numpy as np
import pytest

import inputs
import oracle

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


def test_device_sampler_equals_host_sampler(ldd):
    for n, beta, seed in ((1, 0.1, 3), (4096, 0.1, 1), (1_000_003, 0.02, 9), (1 << 24, 0.05, 1), (70_000, 3.0, 2**64 - 1)):
        log(f"sampler n={n} beta={beta} seed={seed}")
        d = ldd.make_shifts_device(n, beta, seed).cpu().numpy()
        h = ldd.make_shifts(n, beta, seed)
        assert np.array_equal(d, h), (n, beta, seed, np.flatnonzero(d != h)[:5])
    assert np.array_equal(ldd.make_shifts(4096, 0.1, 1), inputs.make_shifts(4096, 0.1, 1))


def radius_of(rp, ci, s):
    c, length, cut = oracle.decompose(rp, ci, s)
    d = (length - (int(s.max()) - s[c])) >> 20
    return c, int(d.max()), cut


def check_draw(ldd, rp, ci, beta, seed, centre, shifts, rep, cut_factor=2.0, radius_factor=3.0):
    n, m = rp.size - 1, ci.size // 2
    s = shifts.cpu().numpy()
    assert np.array_equal(s, ldd.make_shifts(n, beta, rep["seed"]))
    want_c, want_radius, want_cut = radius_of(rp, ci, s)
    assert np.array_equal(centre.cpu().numpy(), want_c)
    assert rep["cut_edges"] == want_cut and rep["max_radius"] == want_radius
    ok = want_cut <= cut_factor * beta * m and want_radius <= radius_factor * math.log(n) / beta
    assert rep["accepted"] == int(ok)
    assert math.isclose(rep["cut_bound"], cut_factor * beta * m)
    assert math.isclose(rep["radius_bound"], radius_factor * math.log(n) / beta)


def test_verified_decomposition_matches_oracle(ldd):
    import torch
    cases = [("grid2d 64x64", *inputs.grid2d(64, 64), 0.1), ("rmat-16", *inputs.rmat(16, 16, seed=1), 0.05),
             ("grid3d 40^3", *inputs.grid3d(40, 40, 40), 0.05), ("er 20000", *inputs.er(20000, 4.0, 3), 0.2)]
    for name, rp, ci, beta in cases:
        d_rp, d_ci = (torch.from_numpy(a).cuda() for a in (rp, ci))
        for seed in (1, 17):
            centre, shifts, rep = ldd.decompose_verified(d_rp, d_ci, beta, seed)
            log(f"{name} seed {seed}: {rep}")
            assert rep["accepted"] == 1 and rep["seed"] == seed + rep["attempts"] - 1
            check_draw(ldd, rp, ci, beta, seed, centre, shifts, rep)


def test_verified_decomposition_retries_and_gives_up(ldd):
    """Bounds no draw can meet: every attempt is made, the status is 'no draw met the bounds',
    and the outputs are the exact decomposition of the last draw."""
    import torch
    rp, ci = inputs.grid2d(50, 50)
    d_rp, d_ci = (torch.from_numpy(a).cuda() for a in (rp, ci))
    centre, shifts, rep = ldd.decompose_verified(d_rp, d_ci, 0.1, 5, cut_factor=1e-9, max_attempts=3)
    assert rep["accepted"] == 0 and rep["attempts"] == 3 and rep["seed"] == 7
    check_draw(ldd, rp, ci, 0.1, 5, centre, shifts, rep, cut_factor=1e-9)
    centre, shifts, rep = ldd.decompose_verified(d_rp, d_ci, 0.1, 5, radius_factor=1e-9, max_attempts=2)
    assert rep["accepted"] == 0 and rep["attempts"] == 2
    check_draw(ldd, rp, ci, 0.1, 5, centre, shifts, rep, radius_factor=1e-9)
    # a bound met only by some draws: the loop stops at the first draw that meets it
    rp, ci = inputs.grid2d(40, 40)
    d_rp, d_ci = (torch.from_numpy(a).cuda() for a in (rp, ci))
    m = ci.size // 2
    cuts = [radius_of(rp, ci, inputs.make_shifts(rp.size - 1, 0.1, 40 + k))[2] for k in range(12)]
    target = (sorted(cuts)[len(cuts) // 3] + 0.5) / (0.1 * m)  # met by about a third of the draws
    first = next(k for k, c in enumerate(cuts) if c <= target * 0.1 * m)
    assert target > 0 and first > 0
    centre, shifts, rep = ldd.decompose_verified(d_rp, d_ci, 0.1, 40, cut_factor=target, radius_factor=100.0,
                                                 max_attempts=12)
    assert rep["accepted"] == 1 and rep["attempts"] == first + 1
    check_draw(ldd, rp, ci, 0.1, 40, centre, shifts, rep, cut_factor=target, radius_factor=100.0)
