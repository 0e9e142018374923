"""Small graph and shift families shared by the oracle pins and the GPU parity tests, and
an independent brute force of the definition (scipy all-pairs BFS + numpy argmin)."""
import numpy as np
import scipy.sparse
import scipy.sparse.csgraph

import inputs

S = 1 << 20


# ------------------------------------------------------------------------------------------
# independent brute force
# ------------------------------------------------------------------------------------------
def all_pairs(rp, ci):
    n = rp.size - 1
    if n == 0:
        return np.zeros((0, 0))
    a = scipy.sparse.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    return scipy.sparse.csgraph.shortest_path(a, method="D", unweighted=True, directed=False)


def brute_force(rp, ci, s):
    n = rp.size - 1
    if n == 0:
        return np.zeros(0, np.int32), 0
    d = all_pairs(rp, ci)
    big = np.int64(1) << 62
    keys = np.where(np.isinf(d), big, S * np.nan_to_num(d, posinf=0).astype(np.int64) - s[:, None].astype(np.int64))
    # keys[u, v]; argmin over u returns the first (smallest) u among equal minima
    centre = np.argmin(keys, axis=0).astype(np.int32)
    src = np.repeat(np.arange(n), np.diff(rp))
    cut = int(np.count_nonzero(centre[src] != centre[ci]) // 2)
    return centre, cut


# ------------------------------------------------------------------------------------------
# small graph and shift families
# ------------------------------------------------------------------------------------------
def path(n):
    return inputs.from_edges(n, np.arange(n - 1), np.arange(1, n))


def cycle(n):
    return inputs.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)


def star(n):
    return inputs.from_edges(n, np.zeros(n - 1, np.int32), np.arange(1, n))


def complete(n):
    iu = np.triu_indices(n, 1)
    return inputs.from_edges(n, iu[0], iu[1])


def random_graph(rng, n, p):
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < p
    return inputs.from_edges(n, iu[0][keep], iu[1][keep])


def disjoint_union(*gs):
    src, dst, off = [], [], 0
    for rp, ci in gs:
        n = rp.size - 1
        s = np.repeat(np.arange(n), np.diff(rp))
        src.append(s + off)
        dst.append(ci + off)
        off += n
    return inputs.from_edges(off, np.concatenate(src), np.concatenate(dst))


def shift_family(rng, n, kind):
    if kind == "exp":
        beta = rng.choice([0.05, 0.2, 0.5, 1.5])
        return np.floor(rng.exponential(1 / beta, n) * S).astype(np.int64)
    if kind == "integer":  # tie-heavy: whole multiples of the unit distance
        return (rng.integers(0, 4, n) * S).astype(np.int64)
    if kind == "equal":
        return np.full(n, 3 * S + 17, np.int64)
    if kind == "tiny":  # all below one unit of distance
        return rng.integers(0, 3, n).astype(np.int64)
    if kind == "mixed":  # integer parts plus a fraction from a two-element set
        return (rng.integers(0, 3, n) * S + rng.integers(0, 2, n)).astype(np.int64)
    raise ValueError(kind)


KINDS = ("exp", "integer", "equal", "tiny", "mixed")


def small_cases(seed=0, count=60):
    rng = np.random.default_rng(seed)
    fixed = [path(1), path(2), path(7), cycle(9), star(8), complete(6), inputs.grid2d(5, 7),
             disjoint_union(path(4), cycle(5), complete(4)), inputs.from_edges(5, [], []),
             disjoint_union(star(5), inputs.from_edges(3, [], []))]
    graphs = list(fixed)
    for _ in range(count):
        n = int(rng.integers(2, 40))
        graphs.append(random_graph(rng, n, float(rng.choice([0.05, 0.1, 0.3, 0.8]))))
    cases = []
    for i, (rp, ci) in enumerate(graphs):
        for kind in KINDS:
            cases.append((rp, ci, shift_family(rng, rp.size - 1, kind), f"g{i}-{kind}"))
    return cases


def multigraph(rng, rp, ci, max_copies=3, loops=0.2):
    """The simple graph (rp, ci) with every edge repeated 1..max_copies times (both arcs each
    time) and a self-loop arc at about a fraction `loops` of the vertices, as a CSR built without
    deduplication.  Returns (row_ptr, col_idx, copies) where copies[a] is the multiplicity of the
    simple graph's arc a."""
    n = rp.size - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    lo = src < ci
    eu, ev = src[lo], ci[lo]
    k = rng.integers(1, max_copies + 1, eu.size)
    s = np.concatenate([np.repeat(eu, k), np.repeat(ev, k)])
    d = np.concatenate([np.repeat(ev, k), np.repeat(eu, k)])
    lv = np.flatnonzero(rng.random(n) < loops)
    s, d = np.concatenate([s, lv]), np.concatenate([d, lv])
    order = np.argsort(s, kind="stable")
    s, d = s[order], d[order]
    mrp = np.zeros(n + 1, np.int32)
    np.add.at(mrp, s + 1, 1)
    copies = {(int(a), int(b)): int(c) for a, b, c in zip(eu, ev, k)}
    return np.cumsum(mrp).astype(np.int32), d.astype(np.int32), copies
