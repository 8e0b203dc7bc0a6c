"""Thin ctypes binding of ``include/gp.h`` (libgp.so).

Every function here only marshals arguments: torch CUDA tensors (or numpy arrays for
host-side geometry) become raw pointers, torch streams become ``hipStream_t``.  All the
work happens in the HIP library.  There is no fallback: if ``libgp.so`` is missing the
import of this module fails.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_float, c_int32, c_int64, c_uint64
from ctypes import c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgp.so")

GP_OK = 0
GP_E_INVALID_ARG = -1
GP_E_BAD_GEOMETRY = -2
GP_E_OOM = -3
GP_E_HIP = -4
GP_E_CAPACITY = -5
GP_E_BUSY = -6
GP_E_CLOSED = -7
GP_E_TIMEOUT = -8
GP_E_NOT_FOUND = -9

GP_PIP = 1
GP_P2P = 2
GP_FP64 = 0
GP_MIXED = 1

PRECISIONS = {"fp64": GP_FP64, "mixed": GP_MIXED}
GP_NOALLOC_SCRATCH_BYTES = 64 << 20  # the workspace gp_query_noalloc holds per GPU
KINDS = {"pip": GP_PIP, "p2p": GP_P2P}


class gp_geometry(Structure):
    _fields_ = [("n_features", c_int64), ("feature_ring_off", c_void_p), ("n_rings", c_int64),
                ("ring_vert_off", c_void_p), ("n_vertices", c_int64), ("x", c_void_p),
                ("y", c_void_p), ("on_device", c_int32)]


class gp_grid_params(Structure):
    _fields_ = [("cell_size", c_double), ("radius_D", c_double), ("x0", c_double),
                ("y0", c_double), ("nx", c_int64), ("ny", c_int64),
                ("pip_cell_classes", c_int32), ("p2p_segment_filter", c_int32),
                ("prestage", c_int32)]


class gp_tuning(Structure):
    _fields_ = [("points_per_lane", c_int32), ("edge_chunk", c_int32), ("wg_per_cu", c_int32),
                ("persistent", c_int32), ("waves_per_item", c_int32), ("vp_points", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gp_stats(Structure):
    _fields_ = [("n_points", c_int64), ("n_paired", c_int64), ("n_items", c_int64),
                ("tests", c_uint64), ("n_rechecked", c_int64), ("ms_pairing", c_float),
                ("ms_refine", c_float), ("ms_recheck", c_float), ("ms_total", c_float),
                ("tests_avoided", c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gp_grid_info(Structure):
    _fields_ = [("kind", c_int32), ("x0", c_double), ("y0", c_double), ("cell_size", c_double),
                ("radius_D", c_double), ("nx", c_int64), ("ny", c_int64), ("n_features", c_int64),
                ("n_edges", c_int64), ("n_pairs", c_int64), ("n_pairs_inside", c_int64),
                ("n_pairs_outside", c_int64), ("n_pairs_boundary", c_int64),
                ("device_bytes", c_int64), ("n_segment_pairs", c_int64)]


class gp_serve_opts(Structure):
    _fields_ = [("n_slots", c_int32), ("slot_points", c_int64), ("mem_budget", c_int64),
                ("precision", c_int32), ("inputs_on_device", c_int32), ("use_graphs", c_int32),
                ("max_queue", c_int32)]


class gp_serve_stats(Structure):
    _fields_ = [("completed", c_int64), ("failed", c_int64), ("pending", c_int64),
                ("in_flight", c_int64), ("p50_us", c_double), ("p99_us", c_double),
                ("mean_us", c_double), ("max_us", c_double), ("points_per_s", c_double),
                ("tests_per_s", c_double), ("points", c_int64), ("tests", c_int64),
                ("graph_replays", c_int64), ("chunks_in_flight", c_int64),
                ("max_in_flight", c_int64), ("max_chunks_in_flight", c_int64),
                ("deferred_for_memory", c_int64), ("bytes_in_use", c_int64),
                ("peak_bytes_in_use", c_int64), ("arena_bytes", c_int64),
                ("latency_samples", c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = c_void_p
_SIGS = {
    "gp_last_error": ([], c_char_p),
    "gp_build_grid": ([c_int32, POINTER(gp_geometry), POINTER(gp_grid_params), _P, POINTER(_P)],
                      c_int32),
    "gp_grid_free": ([_P], None),
    "gp_grid_get_info": ([_P, POINTER(gp_grid_info)], c_int32),
    "gp_grid_candidates": ([_P, _P, _P], c_int32),
    "gp_workspace_bytes": ([_P, c_int64, c_int32, POINTER(ctypes.c_size_t)], c_int32),
    "gp_pair_points": ([_P, c_int64, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], c_int32),
    "gp_pip": ([_P, c_int64, _P, _P, _P, c_int32, _P, ctypes.c_size_t, _P, POINTER(gp_stats)],
               c_int32),
    "gp_p2p": ([_P, c_int64, _P, _P, _P, _P, c_int32, _P, ctypes.c_size_t, _P,
                POINTER(gp_stats)], c_int32),
    "gp_query_noalloc": ([_P, c_int32, c_int64, _P, _P, _P, _P, c_int32, _P], c_int32),
    "gp_set_tuning": ([_P, c_int32, POINTER(gp_tuning)], c_int32),
    "gp_get_tuning": ([_P, c_int32, POINTER(gp_tuning)], c_int32),
    "gp_autotune": ([_P, c_int32, c_int64, _P, _P, _P, ctypes.c_size_t, _P, POINTER(gp_tuning),
                     POINTER(c_float)], c_int32),
    "gp_probe_rate": ([c_int32, c_int32, POINTER(c_double), POINTER(c_float)], c_int32),
    "gp_tuning_cache_save": ([c_char_p], c_int32),
    "gp_tuning_cache_load": ([c_char_p], c_int32),
    "gp_tuning_cache_clear": ([], c_int32),
    "gp_tuning_cache_size": ([POINTER(c_int64)], c_int32),
    "gp_sweep_cell_size": ([c_int32, _P, _P, _P, c_int32, c_int64, _P, _P, c_int32, _P,
                            POINTER(c_double), _P, _P, _P, _P], c_int32),
    "gp_serve_create": ([_P, _P, POINTER(gp_serve_opts), POINTER(_P)], c_int32),
    "gp_serve_submit": ([_P, c_int32, c_int64, _P, _P, _P, _P, POINTER(c_uint64)], c_int32),
    "gp_serve_poll": ([_P, c_uint64, POINTER(c_int32)], c_int32),
    "gp_serve_wait": ([_P, c_uint64, c_int64], c_int32),
    "gp_serve_stats_get": ([_P, POINTER(gp_serve_stats)], c_int32),
    "gp_serve_stats_reset": ([_P], c_int32),
    "gp_serve_destroy": ([_P], c_int32),
}
EXPORTED = sorted(_SIGS)


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


class GPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gp status {status}: {msg}")
        self.status = status


def check(rc):
    if rc != GP_OK:
        raise GPError(rc, lib.gp_last_error().decode(errors="replace"))
    return rc


def _ptr(t):
    """Raw pointer of a torch tensor or numpy array (None stays NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --------------------------------------------------------------------------- grids


class Grid:
    """Owner of a ``gp_grid*``; freed with ``gp_grid_free`` when collected."""

    def __init__(self, handle, kind, keep=()):
        self.handle = handle
        self.kind = kind
        self._keep = keep
        self._lib = lib  # module globals are cleared at interpreter shutdown

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and getattr(self, "_lib", None) is not None:
            self._lib.gp_grid_free(h)

    def info(self) -> dict:
        inf = gp_grid_info()
        check(lib.gp_grid_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def candidates(self):
        inf = self.info()
        off = np.empty(inf["nx"] * inf["ny"] + 1, dtype=np.int32)
        ids = np.empty(max(inf["n_pairs"], 1), dtype=np.int32)
        check(lib.gp_grid_candidates(self.handle, _ptr(off), _ptr(ids)))
        return off, ids[: inf["n_pairs"]]


def gp_build_grid(kind, geom, params, stream=None) -> Grid:
    """``kind`` is "pip"/"p2p" (or GP_PIP/GP_P2P); ``geom`` has numpy ``ring_vert_off``,
    ``x``, ``y`` and ``feature_ring_off`` (None for polylines); ``params`` has
    ``cell_size, radius_D, x0, y0, nx, ny`` and optionally ``cell_classes`` (PIP: 1
    classifies every cell/polygon pair at build time), ``segment_filter`` (P2P: 1 keeps
    per cell only the segments within D of it, for the mixed form) and ``prestage`` (1
    computes every cell's mixed-form records at build time: P2P segment records, PIP
    per (cell, polygon) edge records)."""
    k = KINDS.get(kind, kind)
    g, keep = _geometry(geom)
    p = _params(params)
    h = c_void_p()
    check(lib.gp_build_grid(k, ctypes.byref(g), ctypes.byref(p), _stream(stream),
                            ctypes.byref(h)))
    return Grid(h, k)


def gp_workspace_bytes(grid: Grid, n: int, prec="fp64") -> int:
    b = ctypes.c_size_t()
    check(lib.gp_workspace_bytes(grid.handle, int(n), PRECISIONS.get(prec, prec), ctypes.byref(b)))
    return b.value


def new_workspace(grid: Grid, n: int, prec="fp64", device="cuda"):
    import torch
    return torch.empty(gp_workspace_bytes(grid, n, prec), dtype=torch.uint8, device=device)


def gp_pair_points(grid, px, py, perm, pt_off, ws, stream=None):
    check(lib.gp_pair_points(grid.handle, px.numel(), _ptr(px), _ptr(py), _ptr(perm),
                             _ptr(pt_off), _ptr(ws), ws.numel(), _stream(stream)))


def gp_pip(grid, px, py, out_id, prec, ws, stream=None, stats: bool = False):
    st = gp_stats() if stats else None
    check(lib.gp_pip(grid.handle, px.numel(), _ptr(px), _ptr(py), _ptr(out_id),
                     PRECISIONS.get(prec, prec), _ptr(ws), ws.numel(), _stream(stream),
                     ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def gp_p2p(grid, px, py, out_id, out_dist, prec, ws, stream=None, stats: bool = False):
    st = gp_stats() if stats else None
    check(lib.gp_p2p(grid.handle, px.numel(), _ptr(px), _ptr(py), _ptr(out_id), _ptr(out_dist),
                     PRECISIONS.get(prec, prec), _ptr(ws), ws.numel(), _stream(stream),
                     ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def gp_set_tuning(grid, prec, points_per_lane=0, edge_chunk=0, wg_per_cu=0, persistent=1,
                  waves_per_item=0, vp_points=0):
    t = gp_tuning(points_per_lane, edge_chunk, wg_per_cu, persistent, waves_per_item, vp_points)
    check(lib.gp_set_tuning(grid.handle, PRECISIONS.get(prec, prec), ctypes.byref(t)))


def gp_reset_tuning(grid, prec):
    """Restore the library's default kernel configuration (gp_set_tuning with NULL)."""
    check(lib.gp_set_tuning(grid.handle, PRECISIONS.get(prec, prec), None))


def gp_get_tuning(grid, prec) -> dict:
    t = gp_tuning()
    check(lib.gp_get_tuning(grid.handle, PRECISIONS.get(prec, prec), ctypes.byref(t)))
    return t.as_dict()


def gp_autotune(grid, prec, px, py, ws, stream=None):
    t = gp_tuning()
    ms = c_float()
    check(lib.gp_autotune(grid.handle, PRECISIONS.get(prec, prec), px.numel(), _ptr(px), _ptr(py),
                          _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(t),
                          ctypes.byref(ms)))
    return t.as_dict(), ms.value


def gp_tuning_cache_save(path):
    check(lib.gp_tuning_cache_save(os.fsencode(path)))


def gp_tuning_cache_load(path):
    check(lib.gp_tuning_cache_load(os.fsencode(path)))


def gp_tuning_cache_clear():
    check(lib.gp_tuning_cache_clear())


def gp_tuning_cache_size() -> int:
    n = c_int64()
    check(lib.gp_tuning_cache_size(ctypes.byref(n)))
    return n.value


# --------------------------------------------------------------------------- convenience


def run(grid: Grid, px, py, prec="fp64", ws=None, stream=None, stats=False):
    """Allocate outputs (and a workspace if none is given) and run PIP or P2P.  The
    allocations are made on the stream the query runs on, so the caching allocator does
    not hand the workspace out again while the query still uses it."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(px.device)
    elif isinstance(stream, int):
        stream = torch.cuda.ExternalStream(stream, device=px.device)
    n = px.numel()
    with torch.cuda.stream(stream):
        if ws is None:
            ws = new_workspace(grid, n, prec, px.device)
        out_id = torch.empty(n, dtype=torch.int32, device=px.device)
        if grid.kind == GP_PIP:
            st = gp_pip(grid, px, py, out_id, prec, ws, stream, stats)
            return (out_id, st) if stats else out_id
        out_d = torch.empty(n, dtype=torch.float64, device=px.device)
        st = gp_p2p(grid, px, py, out_id, out_d, prec, ws, stream, stats)
        return (out_id, out_d, st) if stats else (out_id, out_d)


def _geometry(geom):
    """numpy geometry -> (gp_geometry, arrays it points into)."""
    rvo = np.ascontiguousarray(geom.ring_vert_off, dtype=np.int64)
    fro = (None if geom.feature_ring_off is None
           else np.ascontiguousarray(geom.feature_ring_off, dtype=np.int64))
    x = np.ascontiguousarray(geom.x, dtype=np.float64)
    y = np.ascontiguousarray(geom.y, dtype=np.float64)
    nf = len(rvo) - 1 if fro is None else len(fro) - 1
    g = gp_geometry(nf, _ptr(fro), len(rvo) - 1, _ptr(rvo), len(x), _ptr(x), _ptr(y), 0)
    return g, (rvo, fro, x, y)


def _params(params):
    return gp_grid_params(float(params.cell_size), float(getattr(params, "radius_D", 0.0)),
                          float(params.x0), float(params.y0), int(params.nx), int(params.ny),
                          int(getattr(params, "cell_classes", 0)),
                          int(getattr(params, "segment_filter", 0)),
                          int(getattr(params, "prestage", 0)))


def gp_sweep_cell_size(kind, geom, params, cell_sizes, px, py, prec="mixed", stream=None):
    """Times the query on device points ``px, py`` for each cell size; returns
    ``(best, rows)`` with one dict per size (ms, pairs, tests, grid bytes)."""
    k = KINDS.get(kind, kind)
    g, keep = _geometry(geom)
    p = _params(params)
    cs = np.ascontiguousarray(cell_sizes, dtype=np.float64)
    m = len(cs)
    ms = np.zeros(m, dtype=np.float32)
    pairs = np.zeros(m, dtype=np.int64)
    tests = np.zeros(m, dtype=np.uint64)
    gbytes = np.zeros(m, dtype=np.int64)
    best = c_double()
    check(lib.gp_sweep_cell_size(k, ctypes.byref(g), ctypes.byref(p), _ptr(cs), m, px.numel(),
                                 _ptr(px), _ptr(py), PRECISIONS.get(prec, prec), _stream(stream),
                                 ctypes.byref(best), _ptr(ms), _ptr(pairs), _ptr(tests),
                                 _ptr(gbytes)))
    rows = [{"cell_size": float(cs[i]), "ms": float(ms[i]), "pairs": int(pairs[i]),
             "tests": int(tests[i]), "grid_bytes": int(gbytes[i])} for i in range(m)]
    return best.value, rows


def gp_probe_rate(which: int, iters: int):
    """(rate, ms) of a measurement probe: 0 FP32 FMA FLOP/s, 1 FP64 FMA FLOP/s,
    2 LDS broadcast reads/s, 3 mixed P2P tests/s on register data."""
    r = c_double()
    ms = c_float()
    check(lib.gp_probe_rate(int(which), int(iters), ctypes.byref(r), ctypes.byref(ms)))
    return r.value, ms.value


# --------------------------------------------------------------------------- serving


class Server:
    """``gp_serve_*`` wrapper.  Inputs/outputs must stay alive until their ticket is done."""

    def __init__(self, pip_grid=None, p2p_grid=None, n_slots=4, slot_points=1 << 20,
                 mem_budget=8 << 30, precision="mixed", inputs_on_device=True, use_graphs=True,
                 max_queue=0):
        o = gp_serve_opts(n_slots, slot_points, mem_budget, PRECISIONS.get(precision, precision),
                          int(inputs_on_device), int(use_graphs), max_queue)
        h = c_void_p()
        check(lib.gp_serve_create(pip_grid.handle if pip_grid else None,
                                  p2p_grid.handle if p2p_grid else None, ctypes.byref(o),
                                  ctypes.byref(h)))
        self.handle = h
        self._grids = (pip_grid, p2p_grid)
        self._live = {}

    def gp_serve_submit(self, kind, px, py, out_id, out_dist=None) -> int:
        t = c_uint64()
        check(lib.gp_serve_submit(self.handle, KINDS.get(kind, kind), px.numel() if hasattr(px, "numel") else len(px),
                                  _ptr(px), _ptr(py), _ptr(out_id), _ptr(out_dist),
                                  ctypes.byref(t)))
        self._live[t.value] = (px, py, out_id, out_dist)
        return t.value

    submit = gp_serve_submit

    def gp_serve_poll(self, ticket) -> bool:
        """True once done; that releases the ticket (as gp_serve_wait does)."""
        d = c_int32()
        check(lib.gp_serve_poll(self.handle, ticket, ctypes.byref(d)))
        if d.value:
            self._live.pop(ticket, None)
        return bool(d.value)

    poll = gp_serve_poll

    def gp_serve_wait(self, ticket, timeout_us=-1):
        rc = lib.gp_serve_wait(self.handle, ticket, int(timeout_us))
        if rc != GP_E_TIMEOUT:  # complete (or unknown): the ticket is released
            self._live.pop(ticket, None)
        return check(rc)

    wait = gp_serve_wait

    def gp_serve_stats(self) -> dict:
        s = gp_serve_stats()
        check(lib.gp_serve_stats_get(self.handle, ctypes.byref(s)))
        return s.as_dict()

    stats = gp_serve_stats

    def gp_serve_stats_reset(self):
        check(lib.gp_serve_stats_reset(self.handle))

    reset_stats = gp_serve_stats_reset

    def gp_serve_destroy(self):
        h, self.handle = self.handle, None
        if h:
            check(lib.gp_serve_destroy(h))
        self._live.clear()

    close = gp_serve_destroy

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and lib is not None:
            lib.gp_serve_destroy(h)
