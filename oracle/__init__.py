"""CPU oracle for the grid-filtered PIP / P2P join -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, loads or calls
it, and it never calls the GPU library: the two share no code.

The arithmetic lives in ``gp_oracle.c`` (plain scalar FP64, built with
``-O2 -ffp-contract=off``); this module only marshals numpy arrays into it.  The
definitions it follows are given at the top of ``gp_oracle.c`` with the paper's
sections (Sec. III.A filter, Sec. III.B P2P, Sec. III.C PIP).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc.  ``extra`` adds flags (used by mutation tests)."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


def _bind(lib):
    lib.or_mbb.argtypes = [ctypes.c_int, _I64, _P, _P, _P, _P, _D, _D, _P]
    lib.or_extent.argtypes = [_I64, _P, _D, _P, _P, _P, _P]
    lib.or_point_cells.argtypes = [_I64, _P, _P, _D, _D, _D, _I64, _I64, _P]
    lib.or_candidates.argtypes = [_I64, _P, _D, _D, _D, _I64, _I64, _P, _P]
    lib.or_candidates.restype = _I64
    lib.or_sort_points.argtypes = [_I64, _P, _I64, _P, _P]
    lib.or_test_count.argtypes = [_I64, _P, _P, _P, _P]
    lib.or_test_count.restype = ctypes.c_uint64
    lib.or_pip.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _P, _D, _D, _D, _I64, _I64, _P, _P,
                           _P, ctypes.c_int]
    lib.or_pip_count.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _P, _P, ctypes.c_int]
    lib.or_p2p.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _D, _D, _D, _D, _I64, _I64, _P, _P,
                           _P, _P, ctypes.c_int]
    lib.or_polygon_inside.argtypes = [_D, _D, _I64, _P, _P, _P, _P]
    lib.or_polygon_inside.restype = ctypes.c_int
    lib.or_segment_d2.argtypes = [_D, _D, _D, _D, _D, _D]
    lib.or_segment_d2.restype = _D
    lib.or_max_threads.restype = ctypes.c_int
    return lib


def load(path: str = _LIB):
    """Load (building first if needed) the oracle library."""
    global _lib
    if path != _LIB:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def max_threads(lib=None) -> int:
    return (lib or load()).or_max_threads()


def nedges_of(geom) -> np.ndarray:
    """Edges per feature: all ring vertices of a polygon (rings are closed), m-1 for a
    polyline of m vertices."""
    rvo = _i64(geom.ring_vert_off)
    per_ring = np.diff(rvo)
    if geom.feature_ring_off is None:
        return np.maximum(per_ring - 1, 0)
    fro = _i64(geom.feature_ring_off)
    csum = np.concatenate([[0], np.cumsum(per_ring)])
    return csum[fro[1:]] - csum[fro[:-1]]


@dataclasses.dataclass
class OracleGrid:
    kind: str
    x0: float
    y0: float
    cs: float
    nx: int
    ny: int
    D: float
    mbb: np.ndarray
    cand_off: np.ndarray
    cand_id: np.ndarray
    nedges: np.ndarray

    @property
    def ncells(self):
        return self.nx * self.ny


def build_grid(geom, params, lib=None) -> OracleGrid:
    """Sec. III.A filter: feature MBBs (expanded by D for P2P), the extent, and the
    cell -> candidate lists sorted by feature id."""
    lib = lib or load()
    kind = 1 if geom.feature_ring_off is not None else 2
    nf = geom.n_features
    fro = _i64(geom.feature_ring_off) if kind == 1 else None
    rvo, x, y = _i64(geom.ring_vert_off), _f64(geom.x), _f64(geom.y)
    D = float(params.radius_D) if kind == 2 else 0.0
    cs = float(params.cell_size)
    mbb = np.empty(4 * max(nf, 1), dtype=np.float64)
    lib.or_mbb(kind, nf, _ptr(fro), _ptr(rvo), _ptr(x), _ptr(y), D, cs, _ptr(mbb))
    if params.nx == 0 or params.ny == 0:
        x0 = ctypes.c_double()
        y0 = ctypes.c_double()
        nx = ctypes.c_int64()
        ny = ctypes.c_int64()
        lib.or_extent(nf, _ptr(mbb), cs, ctypes.byref(x0), ctypes.byref(y0), ctypes.byref(nx),
                      ctypes.byref(ny))
        x0, y0, nx, ny = x0.value, y0.value, nx.value, ny.value
    else:
        x0, y0, nx, ny = float(params.x0), float(params.y0), int(params.nx), int(params.ny)
    cand_off = np.zeros(nx * ny + 1, dtype=np.int64)
    npairs = lib.or_candidates(nf, _ptr(mbb), x0, y0, cs, nx, ny, _ptr(cand_off), None)
    cand_id = np.empty(max(npairs, 1), dtype=np.int32)
    lib.or_candidates(nf, _ptr(mbb), x0, y0, cs, nx, ny, _ptr(cand_off), _ptr(cand_id))
    return OracleGrid("pip" if kind == 1 else "p2p", x0, y0, cs, nx, ny, D, mbb[:4 * nf],
                      cand_off, cand_id[:npairs], nedges_of(geom))


def point_cells(grid: OracleGrid, px, py, lib=None) -> np.ndarray:
    lib = lib or load()
    px, py = _f64(px), _f64(py)
    out = np.empty(len(px), dtype=np.int64)
    lib.or_point_cells(len(px), _ptr(px), _ptr(py), grid.x0, grid.y0, grid.cs, grid.nx, grid.ny,
                       _ptr(out))
    return out


def sort_points(grid: OracleGrid, cells, lib=None):
    """Stable grouping by cell.  Returns (pt_off[ncells+1], perm[n])."""
    lib = lib or load()
    cells = _i64(cells)
    pt_off = np.empty(grid.ncells + 1, dtype=np.int64)
    perm = np.empty(len(cells), dtype=np.int64)
    lib.or_sort_points(len(cells), _ptr(cells), grid.ncells, _ptr(pt_off), _ptr(perm))
    return pt_off, perm


def test_count(grid: OracleGrid, px, py, lib=None) -> int:
    lib = lib or load()
    pt_off, _ = sort_points(grid, point_cells(grid, px, py, lib), lib)
    ne = _i64(grid.nedges)
    return int(lib.or_test_count(grid.ncells, _ptr(pt_off), _ptr(grid.cand_off),
                                 _ptr(grid.cand_id), _ptr(ne)))


def pip(geom, px, py, grid: OracleGrid | None = None, threads: int = 0, lib=None) -> np.ndarray:
    """Smallest polygon id containing each point (even-odd rule), else -1."""
    lib = lib or load()
    px, py = _f64(px), _f64(py)
    fro, rvo = _i64(geom.feature_ring_off), _i64(geom.ring_vert_off)
    x, y = _f64(geom.x), _f64(geom.y)
    out = np.empty(len(px), dtype=np.int32)
    if grid is None:
        lib.or_pip(len(px), _ptr(px), _ptr(py), geom.n_features, _ptr(fro), _ptr(rvo), _ptr(x),
                   _ptr(y), 0.0, 0.0, 1.0, 0, 0, None, None, _ptr(out), threads)
    else:
        lib.or_pip(len(px), _ptr(px), _ptr(py), geom.n_features, _ptr(fro), _ptr(rvo), _ptr(x),
                   _ptr(y), grid.x0, grid.y0, grid.cs, grid.nx, grid.ny, _ptr(grid.cand_off),
                   _ptr(grid.cand_id), _ptr(out), threads)
    return out


def pip_count(geom, px, py, threads: int = 0, lib=None) -> np.ndarray:
    """Number of polygons (over all of them) whose even-odd test holds for each point."""
    lib = lib or load()
    px, py = _f64(px), _f64(py)
    fro, rvo = _i64(geom.feature_ring_off), _i64(geom.ring_vert_off)
    x, y = _f64(geom.x), _f64(geom.y)
    out = np.empty(len(px), dtype=np.int32)
    lib.or_pip_count(len(px), _ptr(px), _ptr(py), geom.n_features, _ptr(fro), _ptr(rvo), _ptr(x),
                     _ptr(y), _ptr(out), threads)
    return out


def p2p(geom, px, py, D, grid: OracleGrid | None = None, threads: int = 0, lib=None):
    """Nearest polyline within D (ties: smallest id) and its distance; (-1, inf) if none."""
    lib = lib or load()
    px, py = _f64(px), _f64(py)
    rvo, x, y = _i64(geom.ring_vert_off), _f64(geom.x), _f64(geom.y)
    oid = np.empty(len(px), dtype=np.int32)
    od = np.empty(len(px), dtype=np.float64)
    if grid is None:
        lib.or_p2p(len(px), _ptr(px), _ptr(py), geom.n_features, _ptr(rvo), _ptr(x), _ptr(y),
                   float(D), 0.0, 0.0, 1.0, 0, 0, None, None, _ptr(oid), _ptr(od), threads)
    else:
        lib.or_p2p(len(px), _ptr(px), _ptr(py), geom.n_features, _ptr(rvo), _ptr(x), _ptr(y),
                   float(D), grid.x0, grid.y0, grid.cs, grid.nx, grid.ny, _ptr(grid.cand_off),
                   _ptr(grid.cand_id), _ptr(oid), _ptr(od), threads)
    return oid, od


def polygon_inside(geom, f, px, py, lib=None) -> bool:
    lib = lib or load()
    fro, rvo = _i64(geom.feature_ring_off), _i64(geom.ring_vert_off)
    x, y = _f64(geom.x), _f64(geom.y)
    return bool(lib.or_polygon_inside(float(px), float(py), int(f), _ptr(fro), _ptr(rvo), _ptr(x),
                                      _ptr(y)))


def segment_d2(px, py, ax, ay, bx, by, lib=None) -> float:
    lib = lib or load()
    return lib.or_segment_d2(float(px), float(py), float(ax), float(ay), float(bx), float(by))


def run(workload, threads: int = 0, lib=None):
    """Grid-filtered oracle result for a synthetic workload: (grid, ids[, dist])."""
    g = build_grid(workload.geom, workload.params, lib)
    if workload.kind == "pip":
        return g, pip(workload.geom, workload.px, workload.py, g, threads, lib)
    ids, d = p2p(workload.geom, workload.px, workload.py, workload.params.radius_D, g, threads, lib)
    return g, ids, d
