"""GPU: the shift variants of Sec. 5's closing remarks (integer shifts with a random-ranking
tie-break; shifts assigned from positions in a random ranking) decomposed by the same kernels
give the oracle's result on those shifts, and the largest distance to a centre that the library
reports with its statistics equals the oracle's, in every engine."""
import numpy as np
import pytest

import inputs
import oracle
from graphs import small_cases

pytestmark = pytest.mark.gpu


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


def oracle_radius(rp, ci, s):
    c, length, cut = oracle.decompose(rp, ci, s)
    return c, cut, int(((length - (int(s.max()) - s[c])) >> 20).max()) if s.size else 0


def test_variant_shifts_equal_oracle(ldd):
    graphs = [(rp, ci) for rp, ci, _, _ in small_cases(seed=9, count=8)[::5]]
    graphs += [inputs.grid2d(60, 70), inputs.rmat(14, 16, seed=2), inputs.rgg(30000, 6.0, 4), inputs.grid3d(30, 30, 30)]
    for gi, (rp, ci) in enumerate(graphs):
        n = rp.size - 1
        for kind in (ldd.SHIFTS_INT_PERM, ldd.SHIFTS_PERM_ORDER):
            for beta in (0.05, 0.3):
                s = ldd.make_shifts_variant(n, beta, 40 + gi, kind)
                want_c, want_cut, want_r = oracle_radius(rp, ci, s)
                for engine in (0, 2, 3):
                    centre, cut, st = ldd.decompose(*dev(rp, ci, s), beta, stats=True, engine=engine)
                    assert np.array_equal(centre.cpu().numpy(), want_c), (gi, kind, beta, engine)
                    assert cut == want_cut and st["max_radius"] == want_r, (gi, kind, beta, engine)


def test_stats_radius_equals_oracle(ldd):
    for rp, ci, s, beta in (inputs.workload("grid2d-64x64"), inputs.workload("rmat-16"), inputs.workload("grid3d-64")):
        want_c, want_cut, want_r = oracle_radius(rp, ci, s)
        for mode in (dict(), dict(engine=1), dict(engine=2), dict(engine=3), dict(engine=2, tail_vertices=-1)):
            centre, cut, st = ldd.decompose(*dev(rp, ci, s), beta, stats=True, **mode)
            assert np.array_equal(centre.cpu().numpy(), want_c) and cut == want_cut, mode
            assert st["max_radius"] == want_r, (mode, st["max_radius"], want_r)
