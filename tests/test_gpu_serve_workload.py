"""GPU parity of the serving engine on the serving workload's own inputs: the 66 request
templates (RMAT scale 12-22, edge factor 16, three betas, two shift seeds each) served as one
mixed stream, every result compared with the oracle's digest of that template (written by
tests/golden/make_oracle_digests.py from the oracle alone).  Also: a stream of large top-down
requests whose arcs together pass 2^32 (admission must keep the on-device total below it), and
a fill of all 256 slots at once."""
import hashlib
import json
import os

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ldd():
    import torch
    assert torch.cuda.is_available()
    import paper_1307_3692_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def templates():
    """The templates on the device, each checked against the digest of its inputs."""
    import torch
    with open(GOLDEN) as f:
        gold = json.load(f)["serve-templates"]["templates"]
    recipe = inputs.serve_recipe()
    assert len(recipe) == len(gold) == 66
    graphs, out = {}, []
    for (scale, beta, gseed, sseed), g in zip(recipe, gold):
        assert (g["scale"], g["beta"], g["graph_seed"], g["shift_seed"]) == (scale, beta, gseed, sseed)
        if scale not in graphs:
            rp, ci = inputs.rmat(scale, 16, seed=gseed)
            graphs[scale] = (torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda())
        s = inputs.make_shifts(g["n"], beta, sseed)
        assert sha(s) == g["sha_shift"], "shift generator changed since the digests were written"
        out.append((graphs[scale][0], graphs[scale][1], torch.from_numpy(s).cuda(), g))
    torch.cuda.synchronize()
    return out


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def check(got, g, what):
    centre, cut, info = got
    assert info["status"] == 0, what
    c = centre.cpu().numpy()
    assert sha(c) == g["sha_centre"], f"{what}: centres differ from the oracle"
    assert cut == g["cut"], f"{what}: cut {cut} != {g['cut']}"


def test_serving_templates_mixed_stream_equal_oracle(ldd, templates):
    """Every template twice, in a seeded random order, through one server (16 GiB arena):
    scales 12-22 run side by side and every result equals the oracle's."""
    order = np.random.default_rng(7).permutation(np.repeat(np.arange(len(templates)), 2))
    log(f"{order.size} requests, scales {sorted({templates[i][3]['scale'] for i in order})}")
    with ldd.Server(hbm_budget_bytes=16 << 30) as srv:
        tickets = [srv.submit(*templates[i][:3]) for i in order]
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
    log(f"server info {info}")
    for i, got in zip(order, results):
        g = templates[i][3]
        check(got, g, f"scale {g['scale']} beta {g['beta']} seed {g['shift_seed']}")
    assert info["max_active"] > 1


def test_large_top_down_requests_past_2_32_arcs(ldd, templates):
    """40 top-down scale-22 requests sharing one device CSR (128M arcs each, 5.1G together):
    admission holds the on-device arcs below 2^32, and every result equals the oracle's."""
    big = [t for t in templates if t[3]["scale"] == 22]
    with ldd.Server(hbm_budget_bytes=24 << 30, direction=ldd.DIR_TOP_DOWN) as srv:
        tickets, which = [], []
        for k in range(40):
            t = big[k % len(big)]
            tickets.append(srv.submit(*t[:3]))
            which.append(t[3])
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
    log(f"server info {info}")
    for k, (got, g) in enumerate(zip(results, which)):
        check(got, g, f"request {k}: scale 22 beta {g['beta']} seed {g['shift_seed']}")
    arcs = big[0][3]["nnz"]
    assert info["max_active"] * arcs < 1 << 32 and info["max_active"] >= (1 << 32) // arcs - 1


def test_all_256_slots_filled(ldd, templates):
    """300 requests made ready at the same moment (their stream is held by a long matrix product
    until all are submitted), so that the engine admits every slot at once; each result equals
    the oracle's."""
    import torch
    small = [t for t in templates if t[3]["scale"] <= 13]
    blocker = torch.cuda.Stream()
    with ldd.Server(hbm_budget_bytes=2 << 30) as srv:
        with torch.cuda.stream(blocker):
            a = torch.full((4096, 4096), 1.0 / 4096, device="cuda")
            for _ in range(40):
                a = a @ a
        tickets, which = [], []
        for k in range(300):
            t = small[k % len(small)]
            tickets.append(srv.submit(*t[:3], stream=blocker))
            which.append(t[3])
        results = [srv.wait(t) for t in tickets]
        info = srv.info()
    log(f"server info {info}")
    for got, g in zip(results, which):
        check(got, g, f"scale {g['scale']} beta {g['beta']} seed {g['shift_seed']}")
    assert info["max_slots"] == 256 and info["max_active"] == 256
