"""GPU: the block decomposition by iterated decomposition (Sec. 2, Linial-Saks) equals the
oracle's iteration on the same per-level shifts (the library's sampler at seed, seed + 1, ...,
equal to the input generator's), arc by arc."""
import numpy as np
import pytest

import inputs
import oracle
from graphs import multigraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ldd():
    import torch
    assert torch.cuda.is_available()
    import paper_1307_3692_amd as m
    m.lib()
    return m


def test_block_decomposition_equals_oracle(ldd):
    import torch
    rng = np.random.default_rng(8)
    cases = [("grid 50x50", *inputs.grid2d(50, 50)), ("rmat-14", *inputs.rmat(14, 16, seed=4)),
             ("rgg 20000", *inputs.rgg(20000, 6.0, 9)), ("grid3d 40^3", *inputs.grid3d(40, 40, 40))]
    rp, ci = inputs.grid2d(20, 20)
    mrp, mci, _ = multigraph(rng, rp, ci)
    cases.append(("multigraph grid 20x20", mrp, mci))
    for name, rp, ci in cases:
        n = rp.size - 1
        for beta, seed in ((0.5, 11), (0.2, 12)):
            lv, edges = ldd.block_decompose(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), beta=beta,
                                            seed=seed, max_levels=64)
            shifts = [inputs.make_shifts(n, beta, seed + L) for L in range(len(edges))]
            want, run, placed = oracle.block_decomposition(rp, ci, shifts)
            print(f"{name} beta {beta}: {run} levels, edges per level {placed[:8]}", flush=True)
            assert run == len(edges) and placed == edges, name
            assert np.array_equal(lv.cpu().numpy(), want), name
            assert np.all(want >= 0)
    # too few levels: the arcs left keep -1
    rp, ci = inputs.grid2d(30, 30)
    lv, edges = ldd.block_decompose(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), beta=0.5, seed=3,
                                    max_levels=2)
    shifts = [inputs.make_shifts(900, 0.5, 3 + L) for L in range(2)]
    want, run, placed = oracle.block_decomposition(rp, ci, shifts)
    assert len(edges) == 2 and np.array_equal(lv.cpu().numpy(), want) and np.any(want < 0)
