"""Seeded synthetic inputs: CSR graphs and fixed-point exponential shifts.

The decomposition (Algorithm 1 / Algorithm 2 of the paper) consumes an undirected,
unweighted graph and one shift delta_u ~ Exp(beta) per vertex.  This module produces both,
deterministically from a seed, through the C library ``libldd_inputs.so`` built from
``gen.c``.  It is shared by the CPU oracle and the GPU path and contains none of the
decomposition's arithmetic.

Graphs are returned as ``(row_ptr, col_idx)`` int32 numpy arrays (symmetric, sorted
adjacency, no self-loops or duplicates).  Shifts are int64 numpy arrays in units of 2^-20.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libldd_inputs.so")
_SRC = os.path.join(_HERE, "gen.c")

FIX_SHIFT = 20
FIX_ONE = 1 << FIX_SHIFT

# purpose tags: gen.c's own streams (shifts 1, RMAT 2, relabel 3, ER 4, RGG 5) and the draws
# made from Python
TAG_SHIFT = 1
TAG_PERM = 6
TAG_BATCH = 16
TAG_SERVE = 17


def build() -> str:
    """Compile ``gen.c`` into ``libldd_inputs.so`` (always recompiles)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC, "-o", _SO + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp, i64, u64, f64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.ldd_in_make_shifts.argtypes = [i64, f64, u64, vp]
    lib.ldd_in_make_shifts.restype = i32
    lib.ldd_in_make_shifts_variant.argtypes = [i64, f64, u64, i32, vp]
    lib.ldd_in_make_shifts_variant.restype = i32
    lib.ldd_in_u01.argtypes = [u64, u64, u64]
    lib.ldd_in_u01.restype = f64
    lib.ldd_in_draw.argtypes = [u64, u64, u64]
    lib.ldd_in_draw.restype = u64
    for name, args in (
        ("ldd_in_grid2d", [i64, i64]),
        ("ldd_in_grid3d", [i64, i64, i64]),
        ("ldd_in_rmat", [i32, i64, f64, f64, f64, u64, i32]),
        ("ldd_in_er", [i64, f64, u64]),
        ("ldd_in_rgg", [i64, f64, u64]),
        ("ldd_in_from_edges", [i64, i64, vp, vp]),
    ):
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = vp
    lib.ldd_in_graph_n.argtypes = [vp]
    lib.ldd_in_graph_n.restype = i64
    lib.ldd_in_graph_nnz.argtypes = [vp]
    lib.ldd_in_graph_nnz.restype = i64
    lib.ldd_in_graph_copy.argtypes = [vp, vp, vp]
    lib.ldd_in_graph_copy.restype = None
    lib.ldd_in_graph_free.argtypes = [vp]
    lib.ldd_in_graph_free.restype = None
    _lib = lib
    return lib


def _take(handle) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    if not handle:
        raise ValueError("graph generation failed (bad arguments, size or memory)")
    try:
        n = lib.ldd_in_graph_n(handle)
        nnz = lib.ldd_in_graph_nnz(handle)
        row_ptr = np.empty(n + 1, dtype=np.int32)
        col_idx = np.empty(max(nnz, 0), dtype=np.int32)
        lib.ldd_in_graph_copy(handle, row_ptr.ctypes.data, col_idx.ctypes.data)
    finally:
        lib.ldd_in_graph_free(handle)
    return row_ptr, col_idx


def make_shifts(n: int, beta: float, seed: int) -> np.ndarray:
    """delta_u ~ Exp(beta) for u < n, as int64 floor(delta * 2^20)."""
    out = np.empty(n, dtype=np.int64)
    if _load().ldd_in_make_shifts(n, float(beta), seed & (2**64 - 1), out.ctypes.data) != 0:
        raise ValueError(f"bad shift arguments n={n} beta={beta}")
    return out


SHIFTS_EXP, SHIFTS_INT_PERM, SHIFTS_PERM_ORDER = 0, 1, 2


def make_shifts_variant(n: int, beta: float, seed: int, kind: int) -> np.ndarray:
    """Shift variants of Sec. 5's closing remarks: SHIFTS_EXP (the Exp(beta) shifts),
    SHIFTS_INT_PERM (their integer parts plus a random-ranking tie-break as fractional part),
    SHIFTS_PERM_ORDER (the expected exponential order statistics assigned by a random ranking)."""
    out = np.empty(n, dtype=np.int64)
    rc = _load().ldd_in_make_shifts_variant(n, float(beta), seed & (2**64 - 1), int(kind), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"bad shift variant arguments n={n} beta={beta} kind={kind}")
    return out


def perm_rank(n: int, seed: int) -> np.ndarray:
    """The seeded random ranking of the shift variants (vertices by draw of stream (seed, TAG_PERM),
    ties by id): rank[v]."""
    keys = np.array([_load().ldd_in_draw(seed & (2**64 - 1), TAG_PERM, v) for v in range(n)], dtype=np.uint64)
    order = np.lexsort((np.arange(n), keys))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    return rank


def u01(seed: int, tag: int, i: int) -> float:
    """Uniform [0,1) draw i of stream (seed, tag)."""
    return _load().ldd_in_u01(seed & (2**64 - 1), tag, i)


def grid2d(rows: int, cols: int):
    return _take(_load().ldd_in_grid2d(rows, cols))


def grid3d(x: int, y: int, z: int):
    return _take(_load().ldd_in_grid3d(x, y, z))


def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, relabel: bool = True):
    return _take(_load().ldd_in_rmat(scale, edgefactor, a, b, c, seed & (2**64 - 1), int(relabel)))


def er(n: int, avg_degree: float, seed: int):
    p = 0.0 if n < 2 else min(1.0, avg_degree / (n - 1))
    return _take(_load().ldd_in_er(n, p, seed & (2**64 - 1)))


def rgg(n: int, avg_degree: float, seed: int):
    r = math.sqrt(avg_degree / (math.pi * max(n, 1)))
    return _take(_load().ldd_in_rgg(n, r, seed & (2**64 - 1)))


def from_edges(n: int, src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    return _take(_load().ldd_in_from_edges(n, src.size, src.ctypes.data, dst.ctypes.data))


# ------------------------------------------------------------------------------------------
# Workload recipes (sizes and distributions of the benchmarked configurations)
# ------------------------------------------------------------------------------------------

def batch_recipe(num_graphs: int = 512, seed: int = 1, n_lo: int = 1000, n_hi: int = 200_000,
                 beta_lo: float = 0.02, beta_hi: float = 0.3):
    """Per-graph (kind, n, beta, graph_seed, shift_seed) of the batched workload.

    n is log-uniform in [n_lo, n_hi]; even graphs are Erdos-Renyi with mean degree 8, odd
    graphs are 2D random geometric graphs with radius set for mean degree 6; beta is
    log-uniform in [beta_lo, beta_hi]; every graph has its own graph and shift seed.
    """
    out = []
    for g in range(num_graphs):
        un = u01(seed, TAG_BATCH, 4 * g)
        ub = u01(seed, TAG_BATCH, 4 * g + 1)
        n = int(math.floor(math.exp(math.log(n_lo) + un * (math.log(n_hi) - math.log(n_lo)))))
        beta = math.exp(math.log(beta_lo) + ub * (math.log(beta_hi) - math.log(beta_lo)))
        kind = "er" if g % 2 == 0 else "rgg"
        out.append((kind, n, beta, seed * 1_000_003 + 2 * g, seed * 1_000_003 + 2 * g + 1))
    return out


def batch_graphs(num_graphs: int = 512, seed: int = 1, **kw):
    """Generate the batched workload: list of (row_ptr, col_idx, shifts, beta)."""
    graphs = []
    for kind, n, beta, gseed, sseed in batch_recipe(num_graphs, seed, **kw):
        rp, ci = er(n, 8.0, gseed) if kind == "er" else rgg(n, 6.0, gseed)
        graphs.append((rp, ci, make_shifts(n, beta, sseed), beta))
    return graphs


SERVE_SCALES = tuple(range(12, 23))
SERVE_BETAS = (0.05, 0.1, 0.2)


def serve_recipe():
    """The serving workload's request templates: RMAT scale 12..22 (edge factor 16, graph seed
    1000 + scale), each with beta in {0.05, 0.1, 0.2} and two shift seeds
    1000 + 6 (scale - 12) + 2 j + k (j the beta's index, k = 0, 1): 66 templates, as a list of
    (scale, beta, graph_seed, shift_seed).  A request stream draws templates uniformly, so its
    scale is uniform in 12..22 and its beta uniform in the three values."""
    out = []
    for scale in SERVE_SCALES:
        for j, beta in enumerate(SERVE_BETAS):
            for k in range(2):
                out.append((scale, beta, 1000 + scale, 1000 + 6 * (scale - 12) + 2 * j + k))
    return out


# ------------------------------------------------------------------------------------------
# Named single-graph workloads
# ------------------------------------------------------------------------------------------
# name -> (generator, arguments, beta).  Graph seed and shift seed are both 1 unless given.
WORKLOADS = {
    "grid2d-64x64": ("grid2d", (64, 64), 0.1),
    "rmat-24": ("rmat", (24,), 0.05),
    "grid3d-256": ("grid3d", (256, 256, 256), 0.02),
    # smaller members of the same families (parity and CPU-baseline samples)
    "rmat-16": ("rmat", (16,), 0.05),
    "rmat-18": ("rmat", (18,), 0.05),
    "rmat-20": ("rmat", (20,), 0.05),
    "rmat-21": ("rmat", (21,), 0.05),
    "rmat-22": ("rmat", (22,), 0.05),
    "grid3d-64": ("grid3d", (64, 64, 64), 0.02),
    "grid3d-128": ("grid3d", (128, 128, 128), 0.02),
    "grid2d-1000": ("grid2d", (1000, 1000), 0.01),
}


def workload(name: str, graph_seed: int = 1, shift_seed: int = 1, beta: float | None = None):
    """Return ``(row_ptr, col_idx, shift_fix, beta)`` for a named workload.

    ``rmat-<scale>``: RMAT edge factor 16, (a,b,c) = (0.57, 0.19, 0.19), relabelled;
    ``grid2d-<r>x<c>`` / ``grid3d-<k>``: grids; shifts Exp(beta) from ``shift_seed``.
    """
    if name in WORKLOADS:
        gen, args, b = WORKLOADS[name]
    elif name.startswith("rmat-"):
        gen, args, b = "rmat", (int(name[5:]),), 0.05
    else:
        raise KeyError(name)
    if gen == "rmat":
        rp, ci = rmat(args[0], 16, 0.57, 0.19, 0.19, seed=graph_seed, relabel=True)
    elif gen == "grid2d":
        rp, ci = grid2d(*args)
    elif gen == "grid3d":
        rp, ci = grid3d(*args)
    else:
        raise KeyError(name)
    beta = b if beta is None else beta
    return rp, ci, make_shifts(rp.size - 1, beta, shift_seed), beta
