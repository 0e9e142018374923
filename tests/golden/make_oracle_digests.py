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
           "rmat-24", "grid3d-256", "batch-512"]


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


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        if name == "batch-512":
            data[name] = batch_digest()
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
