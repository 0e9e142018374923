"""GPU: the paper's only experiment (Figure 1, Sec. 2) -- a 1000 x 1000 grid decomposed at
beta = 0.002, 0.005, 0.01, 0.02, 0.05, 0.1 (shift seed 1).  The figure shows pieces only, so
there are no printed values to match: every decomposition is compared with the oracle's digest
of that beta (centres, cut, pieces), and the trend the figure illustrates holds: a smaller beta
gives fewer, larger pieces and a smaller cut fraction, within the bound of Cor. 4.5."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


@pytest.fixture(scope="module")
def ldd():
    import torch
    assert torch.cuda.is_available()
    import paper_1307_3692_amd as m
    m.lib()
    return m


def test_figure1_sweep_equals_oracle(ldd):
    import torch
    with open(GOLDEN) as f:
        gold = json.load(f)["figure1"]
    rp, ci = inputs.grid2d(1000, 1000)
    assert hashlib.sha256(rp.view(np.uint8)).hexdigest() == gold["sha_row_ptr"]
    m = ci.size // 2
    d_rp, d_ci = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    rows = []
    for g in gold["betas"]:
        beta = g["beta"]
        s = inputs.make_shifts(rp.size - 1, beta, 1)
        assert hashlib.sha256(s.view(np.uint8)).hexdigest() == g["sha_shift"]
        centre, cut = ldd.decompose(d_rp, d_ci, torch.from_numpy(s).cuda(), beta)
        c = centre.cpu().numpy()
        pieces = int(np.count_nonzero(c == np.arange(c.size)))
        print(f"beta {beta}: pieces {pieces}, cut {cut} ({cut / m:.4f} of the edges)", flush=True)
        assert hashlib.sha256(c.view(np.uint8)).hexdigest() == g["sha_centre"], beta
        assert cut == g["cut"] and pieces == g["pieces"], beta
        assert cut / m <= 1 - math.exp(-beta) + 4 * math.sqrt(beta / m)
        rows.append((beta, pieces, cut))
    for (b0, p0, c0), (b1, p1, c1) in zip(rows, rows[1:]):
        assert b0 < b1 and p0 < p1 and c0 < c1
