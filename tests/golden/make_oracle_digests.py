"""Write ``oracle_digests.json``: the oracle's results on the named workloads.

Stored values come only from ``oracle/`` run on inputs from ``inputs/``: per workload the
SHA-256 of the input arrays (so that a changed generator is reported as such), the SHA-256
of the oracle's centre array, the cut, and the number of pieces.  GPU tests compare the
device result against these digests where running the oracle on the spot would take
too long.

Usage: python tests/golden/make_oracle_digests.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")
DEFAULT = ["grid2d-64x64", "rmat-16", "rmat-18", "rmat-20", "grid3d-64", "grid3d-128", "grid2d-1000",
           "rmat-24", "grid3d-256", "batch-512", "serve-templates", "figure1"]
# Figure 1 (Sec. 2): a 1000 x 1000 grid decomposed at these beta values, shift seed 1
FIGURE1_BETAS = (0.002, 0.005, 0.01, 0.02, 0.05, 0.1)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def batch_digest(num_graphs=512, seed=1):
    """Oracle on every graph of the batched workload: digests of the concatenated centres
    (local ids) and of the per-graph cut counts."""
    centres, cuts, n, nnz = [], [], 0, 0
    t = time.time()
    for rp, ci, s, _ in inputs.batch_graphs(num_graphs, seed=seed):
        c, _, cut = oracle.decompose(rp, ci, s)
        centres.append(c)
        cuts.append(cut)
        n += rp.size - 1
        nnz += ci.size
    return {"graphs": num_graphs, "n": n, "nnz": nnz, "sha_centre": sha(np.concatenate(centres)),
            "sha_cuts": sha(np.array(cuts, np.int64)), "total_cut": int(sum(cuts)),
            "oracle_seconds": round(time.time() - t, 2)}


def serve_digest():
    """Oracle on each of the 66 serving templates (RMAT 12-22, three betas, two shift seeds):
    per template the digest of the centres, the cut and the piece count."""
    out, t = [], time.time()
    graphs = {}
    for scale, beta, gseed, sseed in inputs.serve_recipe():
        if scale not in graphs:
            graphs = {scale: inputs.rmat(scale, 16, seed=gseed)}
        rp, ci = graphs[scale]
        s = inputs.make_shifts(rp.size - 1, beta, sseed)
        c, _, cut = oracle.decompose(rp, ci, s)
        out.append({"scale": scale, "beta": beta, "graph_seed": gseed, "shift_seed": sseed, "n": int(rp.size - 1),
                    "nnz": int(ci.size), "sha_shift": sha(s), "sha_centre": sha(c), "cut": int(cut),
                    "pieces": int(np.count_nonzero(c == np.arange(c.size)))})
        print("serve", out[-1]["scale"], out[-1]["beta"], out[-1]["cut"], flush=True)
    return {"templates": out, "oracle_seconds": round(time.time() - t, 2)}


def figure1_digest():
    """Oracle on the 1000 x 1000 grid at each beta of Figure 1 (shift seed 1): digest of the
    centres, cut, cut fraction, piece count and largest distance to a centre."""
    rp, ci = inputs.grid2d(1000, 1000)
    m = ci.size // 2
    out = []
    for beta in FIGURE1_BETAS:
        s = inputs.make_shifts(rp.size - 1, beta, 1)
        c, length, cut = oracle.decompose(rp, ci, s)
        radius = int(((length - (int(s.max()) - s[c])) >> 20).max())
        out.append({"beta": beta, "sha_shift": sha(s), "sha_centre": sha(c), "cut": int(cut),
                    "cut_fraction": cut / m, "pieces": int(np.count_nonzero(c == np.arange(c.size))),
                    "max_radius": radius})
        print("figure1", out[-1], flush=True)
    return {"n": int(rp.size - 1), "m": int(m), "sha_row_ptr": sha(rp), "sha_col_idx": sha(ci), "betas": out}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        special = {"batch-512": batch_digest, "serve-templates": serve_digest, "figure1": figure1_digest}
        if name in special:
            data[name] = special[name]()
            print(name, data[name], flush=True)
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            continue
        rp, ci, s, beta = inputs.workload(name)
        t = time.time()
        c, length, cut = oracle.decompose(rp, ci, s)
        dt = time.time() - t
        data[name] = {
            "n": int(rp.size - 1), "nnz": int(ci.size), "beta": beta,
            "sha_row_ptr": sha(rp), "sha_col_idx": sha(ci), "sha_shift": sha(s),
            "sha_centre": sha(c), "cut": int(cut), "pieces": int(np.count_nonzero(c == np.arange(c.size))),
            "max_round": int(length.max() >> 20), "rounds_bound": int(s.max() >> 20) + 1,
            "oracle_seconds": round(dt, 2),
        }
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or DEFAULT)
