"""Exponential-shift low-diameter decomposition on AMD MI355X: Python binding of libldd.

Every vertex v joins the centre u minimising dist(u,v) - delta_u (Algorithm 2 of Miller,
Peng and Xu; shifts delta_u ~ Exp(beta), Eq. (1)), ties to the smaller id; shifts are given
in fixed point (int64, units of 2^-20) so the result is exact.  All computation runs in the
HIP kernels of ``libldd.so``; this module only marshals torch device tensors and the current
stream into the C ABI declared in ``include/ldd.h``.  There is no CPU fallback: if the
library cannot be loaded the call raises.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SO_PATH = os.path.join(_HERE, "libldd.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("ldd_kernels.hip", "ldd_rounds.hip", "ldd_api.hip",
                                                   "ldd_batch.hip", "ldd_server.hip", "ldd_tune.hip",
                                                   "ldd_static.hip", "ldd_shifts.hip", "ldd_block.hip",
                                                   "ldd_blockdec.hip")]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# status codes (ldd_status)
(OK, ERR_INVALID_ARG, ERR_OOM, ERR_OVERFLOW, ERR_HIP, ERR_BUDGET, ERR_CANCELLED, ERR_INTERNAL, ERR_PENDING,
 ERR_RETRIES) = range(10)
DIR_AUTO, DIR_TOP_DOWN, DIR_BOTTOM_UP = 0, 1, 2
ENGINE_AUTO, ENGINE_PERSISTENT, ENGINE_LAUNCH, ENGINE_WORKGROUP, ENGINE_TEAM = 0, 1, 2, 3, 4

EXPORTED = ("ldd_decompose", "ldd_workspace_bytes", "ldd_decompose_batch", "ldd_status_string", "ldd_last_error",
            "ldd_release_workspace", "ldd_server_create", "ldd_server_submit", "ldd_server_poll", "ldd_server_wait",
            "ldd_server_cancel", "ldd_server_query", "ldd_server_destroy", "ldd_tune",
            "ldd_decompose_static", "ldd_make_shifts", "ldd_make_shifts_device", "ldd_decompose_verified",
            "ldd_make_shifts_variant", "ldd_block_decompose")


class LddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ldd status {status}: {msg}")
        self.status = status


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("engine", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("td_to_bu", ctypes.c_int32), ("bu_to_td", ctypes.c_int32),
                ("tail_vertices", ctypes.c_int32), ("batch_mode", ctypes.c_int32), ("team_arcs", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("rounds_bound", ctypes.c_int32), ("td_rounds", ctypes.c_int32),
                ("bu_rounds", ctypes.c_int32), ("tail_iters", ctypes.c_int32), ("tail_round", ctypes.c_int32),
                ("blocks", ctypes.c_int32),
                ("delta", ctypes.c_int64), ("pieces", ctypes.c_int64), ("max_frontier", ctypes.c_int64),
                ("arcs_examined", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("ms_prep", ctypes.c_float), ("ms_rounds", ctypes.c_float), ("ms_finalize", ctypes.c_float),
                ("ms_cut", ctypes.c_float), ("steps", ctypes.c_int32), ("max_radius", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VerifyOptions(ctypes.Structure):
    _fields_ = [("cut_factor", ctypes.c_double), ("radius_factor", ctypes.c_double), ("max_attempts", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class VerifyReport(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_int32), ("accepted", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("cut_edges", ctypes.c_int64), ("max_radius", ctypes.c_int64), ("cut_bound", ctypes.c_double),
                ("radius_bound", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneReport(ctypes.Structure):
    _fields_ = [("default_ms", ctypes.c_float), ("best_ms", ctypes.c_float), ("runs", ctypes.c_int32),
                ("from_cache", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_vertices", ctypes.c_int64), ("max_arcs", ctypes.c_int64),
                ("max_slots", ctypes.c_int32), ("chunk_steps", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("max_rounds", ctypes.c_int32), ("tail_vertices", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("shift_fix", ctypes.c_void_p), ("centre", ctypes.c_void_p),
                ("hip_stream", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("rounds", ctypes.c_int32), ("cut_edges", ctypes.c_int64),
                ("first_round", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("latency_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerInfo(ctypes.Structure):
    _fields_ = [("arena_vertices", ctypes.c_int64), ("arena_arcs", ctypes.c_int64), ("max_rounds", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("max_active", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("rebases", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build() -> str:
    """Compile the HIP sources into ``libldd.so`` for gfx950 (always recompiles)."""
    tmp = SO_PATH + ".tmp"
    subprocess.run(["hipcc", *HIPCC_FLAGS, *SOURCES, "-o", tmp], check=True)
    os.replace(tmp, SO_PATH)
    return SO_PATH


_lib = None


def lib():
    """The loaded ``libldd.so`` (built first if it does not exist yet)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        build()
    L = ctypes.CDLL(SO_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.ldd_decompose.argtypes = [ctypes.POINTER(Csr), vp, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(Options), ctypes.POINTER(Stats), vp]
    L.ldd_decompose.restype = i32
    L.ldd_decompose_static.argtypes = [ctypes.POINTER(Csr), vp, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(Options), vp]
    L.ldd_decompose_static.restype = i32
    L.ldd_make_shifts.argtypes = [i32, ctypes.c_double, ctypes.c_uint64, vp]
    L.ldd_make_shifts.restype = i32
    L.ldd_block_decompose.argtypes = [ctypes.POINTER(Csr), ctypes.c_double, ctypes.c_uint64, i32, vp,
                                      ctypes.POINTER(ctypes.c_int32), vp, ctypes.POINTER(Options), vp]
    L.ldd_block_decompose.restype = i32
    L.ldd_make_shifts_variant.argtypes = [i32, ctypes.c_double, ctypes.c_uint64, i32, vp]
    L.ldd_make_shifts_variant.restype = i32
    L.ldd_make_shifts_device.argtypes = [i32, ctypes.c_double, ctypes.c_uint64, vp, vp]
    L.ldd_make_shifts_device.restype = i32
    L.ldd_decompose_verified.argtypes = [ctypes.POINTER(Csr), ctypes.c_double, ctypes.c_uint64, vp, vp,
                                         ctypes.POINTER(VerifyOptions), ctypes.POINTER(Options),
                                         ctypes.POINTER(VerifyReport), vp]
    L.ldd_decompose_verified.restype = i32
    L.ldd_decompose_batch.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Options), vp]
    L.ldd_decompose_batch.restype = i32
    L.ldd_workspace_bytes.argtypes = [i32, i64]
    L.ldd_workspace_bytes.restype = ctypes.c_size_t
    L.ldd_status_string.argtypes = [i32]
    L.ldd_status_string.restype = ctypes.c_char_p
    L.ldd_last_error.argtypes = []
    L.ldd_last_error.restype = ctypes.c_char_p
    L.ldd_release_workspace.argtypes = []
    L.ldd_release_workspace.restype = None
    L.ldd_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.ldd_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.ldd_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.ldd_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.ldd_server_cancel.argtypes = [vp, ctypes.c_uint64]
    L.ldd_server_query.argtypes = [vp, ctypes.POINTER(ServerInfo)]
    L.ldd_server_destroy.argtypes = [vp]
    for f in ("create", "submit", "poll", "wait", "cancel", "query", "destroy"):
        getattr(L, "ldd_server_" + f).restype = i32
    L.ldd_tune.argtypes = [i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Options), ctypes.c_char_p,
                           ctypes.POINTER(Options), ctypes.POINTER(TuneReport), vp]
    L.ldd_tune.restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        L = lib()
        raise LddError(status, f"{L.ldd_status_string(status).decode()}: {L.ldd_last_error().decode()}")


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _device_tensor(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t


BATCH_AUTO, BATCH_SEQUENTIAL, BATCH_UNION, BATCH_WORKGROUP = 0, 1, 2, 3


def make_options(direction=DIR_AUTO, engine=ENGINE_AUTO, validate=False, blocks=0, td_to_bu=0, bu_to_td=0,
                 tail_vertices=0, batch_mode=BATCH_AUTO, team_arcs=0) -> Options:
    o = Options()
    o.direction, o.engine, o.validate, o.blocks = direction, engine, int(validate), blocks
    o.td_to_bu, o.bu_to_td, o.tail_vertices, o.batch_mode = td_to_bu, bu_to_td, tail_vertices, batch_mode
    o.team_arcs = team_arcs
    return o


def decompose(row_ptr, col_idx, shift_fix, beta: float, *, centre=None, stream=None, stats: bool = False, **opts):
    """Decompose one graph held in device memory.

    row_ptr int32[n+1], col_idx int32[nnz], shift_fix int64[n] (torch tensors on the GPU).
    Returns ``(centre int32[n] tensor, cut_edges)`` or, with ``stats=True``,
    ``(centre, cut_edges, stats dict)``.
    """
    import torch
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    _device_tensor(shift_fix, torch.int64, "shift_fix")
    n = row_ptr.numel() - 1
    if n < 0 or shift_fix.numel() != n:
        raise ValueError("row_ptr and shift_fix sizes disagree")
    if centre is None:
        centre = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    else:
        _device_tensor(centre, torch.int32, "centre")
        if centre.numel() != n:
            raise ValueError("centre has the wrong size")
    g = Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    cut = ctypes.c_int64(0)
    st = Stats()
    o = make_options(**opts)
    # statistics only when asked for: they add a pass over the labels (the largest distance to a
    # centre) and a synchronisation
    _check(lib().ldd_decompose(ctypes.byref(g), shift_fix.data_ptr(), float(beta), centre.data_ptr(),
                               ctypes.byref(cut), ctypes.byref(o), ctypes.byref(st) if stats else None,
                               _stream_handle(stream)))
    if stats:
        return centre, int(cut.value), st.as_dict()
    return centre, int(cut.value)


def make_shifts(n: int, beta: float, seed: int):
    """Host shifts of the library's sampler (``ldd_make_shifts``): numpy int64[n]."""
    import numpy as np
    out = np.empty(n, dtype=np.int64)
    _check(lib().ldd_make_shifts(int(n), float(beta), seed & (2**64 - 1), out.ctypes.data if n else None))
    return out


SHIFTS_EXP, SHIFTS_INT_PERM, SHIFTS_PERM_ORDER = 0, 1, 2


def make_shifts_variant(n: int, beta: float, seed: int, kind: int):
    """Host shifts of a variant of Sec. 5's closing remarks (``ldd_make_shifts_variant``)."""
    import numpy as np
    out = np.empty(n, dtype=np.int64)
    _check(lib().ldd_make_shifts_variant(int(n), float(beta), seed & (2**64 - 1), int(kind),
                                         out.ctypes.data if n else None))
    return out


def make_shifts_device(n: int, beta: float, seed: int, *, out=None, stream=None):
    """Device shifts of the library's sampler (``ldd_make_shifts_device``): torch int64[n] on
    the current GPU, enqueued on the stream (default: torch's current stream)."""
    import torch
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device="cuda")
    else:
        _device_tensor(out, torch.int64, "out")
        if out.numel() != n:
            raise ValueError("out has the wrong size")
    _check(lib().ldd_make_shifts_device(int(n), float(beta), seed & (2**64 - 1), out.data_ptr() if n else None,
                                        _stream_handle(stream)))
    return out


def decompose_verified(row_ptr, col_idx, beta: float, seed: int, *, cut_factor: float = 0.0,
                       radius_factor: float = 0.0, max_attempts: int = 0, stream=None, **opts):
    """Las Vegas decomposition (``ldd_decompose_verified``): shifts drawn on the device from
    seed, seed + 1, ... until the cut and every distance to a centre meet their bounds.
    Returns ``(centre, shift_fix, report dict)``; ``report["accepted"]`` is 0 when every draw
    failed (status LDD_ERR_RETRIES), in which case the outputs hold the last draw."""
    import torch
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr is empty")
    centre = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    shifts = torch.empty(n, dtype=torch.int64, device=row_ptr.device)
    g = Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    v = VerifyOptions()
    v.cut_factor, v.radius_factor, v.max_attempts = cut_factor, radius_factor, max_attempts
    o = make_options(**opts)
    rep = VerifyReport()
    status = lib().ldd_decompose_verified(ctypes.byref(g), float(beta), seed & (2**64 - 1), shifts.data_ptr(),
                                          centre.data_ptr(), ctypes.byref(v), ctypes.byref(o), ctypes.byref(rep),
                                          _stream_handle(stream))
    if status != ERR_RETRIES:
        _check(status)
    return centre, shifts, rep.as_dict()


def block_decompose(row_ptr, col_idx, *, beta: float = 0.5, seed: int = 1, max_levels: int = 64, stream=None,
                    **opts):
    """Linial-Saks block decomposition by iterated decomposition (``ldd_block_decompose``).
    Returns ``(arc_level int32[nnz] tensor, level_edges list)``; arcs left after max_levels
    levels keep level -1 (status LDD_ERR_RETRIES is returned as that, not raised)."""
    import numpy as np
    import torch
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    n = row_ptr.numel() - 1
    arc_level = torch.empty(col_idx.numel(), dtype=torch.int32, device=row_ptr.device)
    g = Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    levels = ctypes.c_int32(0)
    edges = np.zeros(max_levels, np.int64)
    o = make_options(**opts)
    status = lib().ldd_block_decompose(ctypes.byref(g), float(beta), seed & (2**64 - 1), int(max_levels),
                                       arc_level.data_ptr() if col_idx.numel() else None, ctypes.byref(levels),
                                       edges.ctypes.data, ctypes.byref(o), _stream_handle(stream))
    if status != ERR_RETRIES:
        _check(status)
    return arc_level, [int(x) for x in edges[:levels.value]]


STATIC_MAX_VERTICES = 1 << 20  # LDD_STATIC_MAX_VERTICES


def decompose_static(row_ptr, col_idx, shift_fix, beta: float, *, centre, stream=None, **opts):
    """As :func:`decompose`, through ``ldd_decompose_static``: the library allocates nothing
    (its scratch is a fixed device array of the library, n <= STATIC_MAX_VERTICES).  The caller
    provides the output tensor ``centre``.  Returns the cut."""
    import torch
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    _device_tensor(shift_fix, torch.int64, "shift_fix")
    _device_tensor(centre, torch.int32, "centre")
    n = row_ptr.numel() - 1
    if n < 0 or shift_fix.numel() != n or centre.numel() != n:
        raise ValueError("row_ptr, shift_fix and centre sizes disagree")
    g = Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)
    cut = ctypes.c_int64(0)
    o = make_options(**opts)
    _check(lib().ldd_decompose_static(ctypes.byref(g), shift_fix.data_ptr(), float(beta), centre.data_ptr(),
                                      ctypes.byref(cut), ctypes.byref(o), _stream_handle(stream)))
    return int(cut.value)


def decompose_batch(vtx_off, arc_off, row_ptr, col_idx, shift_fix, *, centre=None, stream=None, **opts):
    """Decompose many graphs packed in one offset CSR (see ``ldd_decompose_batch``).

    vtx_off / arc_off: host int64 sequences of length G+1; row_ptr int32[vtx_off[G] + G],
    col_idx int32[arc_off[G]] (local ids), shift_fix int64[vtx_off[G]] on the GPU.
    Returns ``(centre tensor with local ids, list of per-graph cut counts)``.
    """
    import numpy as np
    import torch
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    ao = np.ascontiguousarray(arc_off, dtype=np.int64)
    G = vo.size - 1
    if G < 0 or ao.size != vo.size:
        raise ValueError("vtx_off and arc_off must both have G+1 entries")
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    _device_tensor(shift_fix, torch.int64, "shift_fix")
    nv = int(vo[-1]) if G >= 0 else 0
    if row_ptr.numel() != nv + G or shift_fix.numel() != nv or col_idx.numel() != int(ao[-1]):
        raise ValueError("packed array sizes disagree with the offsets")
    if centre is None:
        centre = torch.empty(nv, dtype=torch.int32, device=row_ptr.device)
    cuts = np.zeros(max(G, 1), dtype=np.int64)
    o = make_options(**opts)
    _check(lib().ldd_decompose_batch(G, vo.ctypes.data, ao.ctypes.data, row_ptr.data_ptr(),
                                     col_idx.data_ptr() if col_idx.numel() else None, shift_fix.data_ptr(),
                                     centre.data_ptr(), cuts.ctypes.data, ctypes.byref(o), _stream_handle(stream)))
    return centre, [int(x) for x in cuts[:G]]


def tune(row_ptr, col_idx, shift_fix, *, vtx_off=None, arc_off=None, centre=None, cache_path=None, stream=None,
         **opts):
    """Tune the engine and its knobs (``ldd_tune``) for one graph (no offsets) or a packed batch.

    Returns ``(options dict for decompose / decompose_batch, report dict)``.
    """
    import numpy as np
    import torch
    _device_tensor(row_ptr, torch.int32, "row_ptr")
    _device_tensor(col_idx, torch.int32, "col_idx")
    _device_tensor(shift_fix, torch.int64, "shift_fix")
    if vtx_off is None:
        n = row_ptr.numel() - 1
        vo = np.array([0, n], dtype=np.int64)
        ao = np.array([0, col_idx.numel()], dtype=np.int64)
    else:
        vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
        ao = np.ascontiguousarray(arc_off, dtype=np.int64)
    G = vo.size - 1
    if centre is None:
        centre = torch.empty(int(vo[-1]), dtype=torch.int32, device=row_ptr.device)
    base = make_options(**opts)
    best = Options()
    rep = TuneReport()
    _check(lib().ldd_tune(G, vo.ctypes.data, ao.ctypes.data, row_ptr.data_ptr(),
                          col_idx.data_ptr() if col_idx.numel() else None, shift_fix.data_ptr(), centre.data_ptr(),
                          ctypes.byref(base), cache_path.encode() if cache_path else None, ctypes.byref(best),
                          ctypes.byref(rep), _stream_handle(stream)))
    tuned = dict(opts, blocks=best.blocks, td_to_bu=best.td_to_bu, bu_to_td=best.bu_to_td,
                 tail_vertices=best.tail_vertices, team_arcs=best.team_arcs)
    if G == 1:
        tuned["engine"] = best.engine
    else:
        tuned["batch_mode"] = best.batch_mode
    return tuned, rep.as_dict()


def workspace_bytes(n: int, nnz: int) -> int:
    return int(lib().ldd_workspace_bytes(n, nnz))


class Server:
    """Continuous-batching decomposition server (``ldd_server_*``): requests are queued, admitted
    into one device-resident arena as room frees up, and advance together one round per step.

    ``submit`` takes device tensors (kept referenced until the result is collected) and returns a
    ticket; ``wait`` / ``poll`` give ``(centre tensor, cut_edges, info dict)``.
    """

    def __init__(self, hbm_budget_bytes: int = 1 << 30, max_vertices: int = 0, max_arcs: int = 0,
                 max_slots: int = 0, chunk_steps: int = 0, blocks: int = 0, direction: int = DIR_AUTO,
                 max_rounds: int = 0, tail_vertices: int = 0):
        cfg = ServerConfig()
        cfg.hbm_budget_bytes, cfg.max_vertices, cfg.max_arcs = hbm_budget_bytes, max_vertices, max_arcs
        cfg.max_slots, cfg.chunk_steps, cfg.blocks = max_slots, chunk_steps, blocks
        cfg.direction, cfg.max_rounds, cfg.tail_vertices = direction, max_rounds, tail_vertices
        h = ctypes.c_void_p()
        _check(lib().ldd_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._live = {}  # ticket -> (tensors kept alive, centre)

    def submit(self, row_ptr, col_idx, shift_fix, *, centre=None, stream=None) -> int:
        import torch
        _device_tensor(row_ptr, torch.int32, "row_ptr")
        _device_tensor(col_idx, torch.int32, "col_idx")
        _device_tensor(shift_fix, torch.int64, "shift_fix")
        n = row_ptr.numel() - 1
        if n < 0 or shift_fix.numel() != n:
            raise ValueError("row_ptr and shift_fix sizes disagree")
        if centre is None:
            centre = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
        else:
            _device_tensor(centre, torch.int32, "centre")
            if centre.numel() != n:
                raise ValueError("centre has the wrong size")
        q = Request(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None,
                    shift_fix.data_ptr(), centre.data_ptr(), _stream_handle(stream).value)
        t = ctypes.c_uint64(0)
        _check(lib().ldd_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._live[t.value] = ((row_ptr, col_idx, shift_fix), centre)
        return t.value

    def _collect(self, ticket, status, res):
        if status == ERR_PENDING:
            return None
        _, centre = self._live.pop(ticket, (None, None))
        _check(status)
        return centre, int(res.cut_edges), res.as_dict()

    def poll(self, ticket: int):
        """``None`` while the request runs, else ``(centre, cut_edges, info)``."""
        res = Result()
        return self._collect(ticket, lib().ldd_server_poll(self._h, ticket, ctypes.byref(res)), res)

    def wait(self, ticket: int):
        res = Result()
        return self._collect(ticket, lib().ldd_server_wait(self._h, ticket, ctypes.byref(res)), res)

    def cancel(self, ticket: int) -> bool:
        """True if the request was still queued (collect it: its status is cancelled)."""
        s = lib().ldd_server_cancel(self._h, ticket)
        if s == ERR_PENDING:
            return False
        _check(s)
        return True

    def info(self) -> dict:
        out = ServerInfo()
        _check(lib().ldd_server_query(self._h, ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if self._h:
            h, self._h = self._h, None
            status = lib().ldd_server_destroy(h)  # runs what is queued: inputs must outlive it
            self._live.clear()
            _check(status)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
