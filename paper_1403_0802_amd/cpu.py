"""Thin ctypes binding of ``include/gp_cpu.h`` (libgp_cpu.so): the host multi-core /
AVX-512 implementation of the two refinements, for the CPU side of the comparison.
Argument marshalling only; numpy arrays in, numpy arrays out."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_double, c_int32, c_int64, c_uint64, c_void_p

import numpy as np

from .gp import GP_P2P, KINDS, GPError, _geometry, _params, _ptr

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgp_cpu.so")
MODES = {"sc": 0, "mc": 1, "sc_simd": 2, "mc_simd": 3}


class gp_cpu_stats(Structure):
    _fields_ = [("tests", c_uint64), ("threads", c_int32), ("simd", c_int32),
                ("ms_filter", c_double), ("ms_refine", c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.gp_cpu_join.argtypes = [c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_int32, c_int32, POINTER(gp_cpu_stats)]
    lib.gp_cpu_join.restype = c_int32
    lib.gp_cpu_has_simd.argtypes = []
    lib.gp_cpu_has_simd.restype = c_int32
    return lib


lib = _load()
EXPORTED = ["gp_cpu_has_simd", "gp_cpu_join"]


def gp_cpu_has_simd() -> bool:
    return bool(lib.gp_cpu_has_simd())


def gp_cpu_join(kind, geom, params, px, py, mode="mc_simd", threads=0):
    """Returns ``(ids, dists_or_None, stats_dict)`` for host points ``px, py``."""
    k = KINDS.get(kind, kind)
    g, keep = _geometry(geom)
    p = _params(params)
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    oid = np.empty(len(px), dtype=np.int32)
    od = np.empty(len(px), dtype=np.float64) if k == GP_P2P else None
    st = gp_cpu_stats()
    rc = lib.gp_cpu_join(k, ctypes.byref(g), ctypes.byref(p), len(px), _ptr(px), _ptr(py),
                         _ptr(oid), _ptr(od), MODES.get(mode, mode), int(threads),
                         ctypes.byref(st))
    if rc != 0:
        raise GPError(rc, "gp_cpu_join failed")
    return oid, od, {k2: getattr(st, k2) for k2, _ in st._fields_}
