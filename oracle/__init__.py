"""CPU oracle for the exponential-shift low-diameter decomposition -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library never calls it and shares no code with it.

ctypes wrapper over ``liblddoracle.so`` (``ldd_oracle.c``):

* :func:`decompose` -- every vertex's centre and the cut, by Dijkstra from the super source
  of Sec. 5 over (length, first vertex) pairs in lexicographic order;
* :func:`decompose_rounds` -- the same result by the bucketed search of Sec. 5 (one bucket per
  integer distance, Dial's bucket queue), the single-threaded CPU baseline the benchmark times;
* :func:`centre_of` -- one vertex's centre by the definition of Algorithm 2 (BFS from v,
  lexicographic argmin of the shifted distance, Eq. (1));
* :func:`cut` -- cut edges of an assignment (Def. 1.1);
* :func:`certify` -- linear-time certificate that an assignment is the exact argmin;
* :func:`block_decomposition` -- the Linial-Saks block decomposition of Sec. 2 by iterating
  :func:`decompose` on the edges not placed yet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblddoracle.so")
_SRC = os.path.join(_HERE, "ldd_oracle.c")

FIX_ONE = 1 << 20

OK = 0
BAD_ARG = 1
NO_MEM = 2
BAD_CENTRE = 10
DISCONNECTED = 11
NOT_MINIMAL_SELF = 12
NOT_MINIMAL_EDGE = 13

# planted mistakes (tests of the pins only)
MUT_NONE = 0
MUT_TIE_LARGER_ID = 1
MUT_SHIFT_SIGN = 2
MUT_EDGE_LENGTH = 3
MUT_INTEGER_SHIFTS = 4
MUT_NO_TIEBREAK = 5
MUTATIONS = (MUT_TIE_LARGER_ID, MUT_SHIFT_SIGN, MUT_EDGE_LENGTH, MUT_INTEGER_SHIFTS, MUT_NO_TIEBREAK)


class OracleError(RuntimeError):
    pass


def build() -> str:
    """Compile ``ldd_oracle.c`` into ``liblddoracle.so`` (always recompiles)."""
    cmd = ["gcc", "-O2", "-shared", "-fPIC", "-Wall", _SRC, "-o", _SO + ".tmp"]
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
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.oracle_decompose_mut.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32]
    lib.oracle_decompose_mut.restype = i32
    lib.oracle_decompose_rounds.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.oracle_decompose_rounds.restype = i32
    lib.oracle_centre_of.argtypes = [i64, vp, vp, vp, i64, vp, vp]
    lib.oracle_centre_of.restype = i32
    lib.oracle_cut.argtypes = [i64, vp, vp, vp]
    lib.oracle_cut.restype = i64
    lib.oracle_certify.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.oracle_certify.restype = i32
    _lib = lib
    return lib


def _arrays(row_ptr, col_idx, shift_fix=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    sf = None if shift_fix is None else np.ascontiguousarray(shift_fix, dtype=np.int64)
    n = rp.size - 1
    if n < 0 or (sf is not None and sf.size != n):
        raise ValueError("row_ptr / shift_fix sizes disagree")
    return n, rp, ci, sf


def decompose(row_ptr, col_idx, shift_fix, mutation: int = MUT_NONE):
    """Return ``(centre int32[n], length int64[n], cut)`` where length[v] is
    Delta + min over u of (2^20 dist(u,v) - shift_fix[u])."""
    n, rp, ci, sf = _arrays(row_ptr, col_idx, shift_fix)
    centre = np.empty(n, dtype=np.int32)
    length = np.empty(n, dtype=np.int64)
    cut_v = ctypes.c_int64(0)
    rc = _load().oracle_decompose_mut(n, rp.ctypes.data, ci.ctypes.data, sf.ctypes.data, centre.ctypes.data,
                                      length.ctypes.data, ctypes.addressof(cut_v), mutation)
    if rc != OK:
        raise OracleError(f"oracle_decompose failed with code {rc}")
    return centre, length, int(cut_v.value)


def decompose_rounds(row_ptr, col_idx, shift_fix):
    """As :func:`decompose`, by the bucketed search of Sec. 5 (one integer distance per round)."""
    n, rp, ci, sf = _arrays(row_ptr, col_idx, shift_fix)
    centre = np.empty(n, dtype=np.int32)
    length = np.empty(n, dtype=np.int64)
    cut_v = ctypes.c_int64(0)
    rc = _load().oracle_decompose_rounds(n, rp.ctypes.data, ci.ctypes.data, sf.ctypes.data, centre.ctypes.data,
                                         length.ctypes.data, ctypes.addressof(cut_v))
    if rc != OK:
        raise OracleError(f"oracle_decompose_rounds failed with code {rc}")
    return centre, length, int(cut_v.value)


def centre_of(row_ptr, col_idx, shift_fix, v: int):
    """Return ``(centre, shifted distance)`` of vertex v by the definition."""
    n, rp, ci, sf = _arrays(row_ptr, col_idx, shift_fix)
    c = ctypes.c_int32(0)
    val = ctypes.c_int64(0)
    rc = _load().oracle_centre_of(n, rp.ctypes.data, ci.ctypes.data, sf.ctypes.data, int(v),
                                  ctypes.addressof(c), ctypes.addressof(val))
    if rc != OK:
        raise OracleError(f"oracle_centre_of failed with code {rc}")
    return int(c.value), int(val.value)


def cut(row_ptr, col_idx, centre) -> int:
    n, rp, ci, _ = _arrays(row_ptr, col_idx)
    ce = np.ascontiguousarray(centre, dtype=np.int32)
    if ce.size != n:
        raise ValueError("centre has the wrong length")
    return int(_load().oracle_cut(n, rp.ctypes.data, ci.ctypes.data, ce.ctypes.data))


def certify(row_ptr, col_idx, shift_fix, centre):
    """Return ``(code, vertex)``: code OK means the assignment is the exact argmin."""
    n, rp, ci, sf = _arrays(row_ptr, col_idx, shift_fix)
    ce = np.ascontiguousarray(centre, dtype=np.int32)
    if ce.size != n:
        raise ValueError("centre has the wrong length")
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_certify(n, rp.ctypes.data, ci.ctypes.data, sf.ctypes.data, ce.ctypes.data,
                                ctypes.addressof(bad))
    return int(rc), int(bad.value)


def block_decomposition(row_ptr, col_idx, level_shifts):
    """Block decomposition by iterated decomposition (Sec. 2, Linial-Saks): level L decomposes
    the graph of the arcs not placed yet with ``level_shifts[L]``; arcs whose ends share a centre
    take level L, the others go on.  Returns (arc_level int32[nnz] with -1 for arcs not placed,
    the number of levels run, edges placed per level)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    level = np.full(ci.size, -1, np.int32)
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp))
    ids = np.arange(ci.size)
    placed, run = [], 0
    for L, s in enumerate(level_shifts):
        if ids.size == 0:
            break
        rp_l = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int32)
        c, _, _ = decompose(rp_l, ci[ids], s)
        inside = c[src] == c[ci[ids]]
        level[ids[inside]] = L
        placed.append(int(np.count_nonzero(inside)) // 2)
        ids, src = ids[~inside], src[~inside]
        run = L + 1
    return level, run, placed
