"""CPU-side checks of the C ABI: the library loads, exports every function the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gp.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(gp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gp_build_grid", "gp_pip", "gp_p2p", "gp_serve_create", "gp_serve_submit",
              "gp_serve_wait", "gp_serve_destroy", "gp_last_error", "gp_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1403_0802_amd import gp
    lib = ctypes.CDLL(gp.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(declared_functions()) == gp.EXPORTED


def test_cpu_library_exports_its_header():
    from paper_1403_0802_amd import cpu
    names = declared_functions(os.path.join(ROOT, "include", "gp_cpu.h"))
    lib = ctypes.CDLL(cpu.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(cpu.EXPORTED)


def test_argument_errors_are_synchronous():
    from paper_1403_0802_amd import gp
    L = gp.lib
    out = ctypes.c_void_p()
    assert L.gp_build_grid(1, None, None, None, ctypes.byref(out)) == gp.GP_E_INVALID_ARG
    geom = gp.gp_geometry()
    params = gp.gp_grid_params(0.0, 0.0, 0.0, 0.0, 0, 0)
    assert L.gp_build_grid(1, ctypes.byref(geom), ctypes.byref(params), None,
                           ctypes.byref(out)) == gp.GP_E_INVALID_ARG
    assert b"cell_size" in L.gp_last_error()
    params.cell_size = 1.0
    assert L.gp_build_grid(7, ctypes.byref(geom), ctypes.byref(params), None,
                           ctypes.byref(out)) == gp.GP_E_INVALID_ARG
    params.radius_D = -1.0
    assert L.gp_build_grid(2, ctypes.byref(geom), ctypes.byref(params), None,
                           ctypes.byref(out)) == gp.GP_E_INVALID_ARG
    geom.n_features = 1 << 31
    params.radius_D = 0.0
    assert L.gp_build_grid(2, ctypes.byref(geom), ctypes.byref(params), None,
                           ctypes.byref(out)) == gp.GP_E_CAPACITY
    b = ctypes.c_size_t()
    assert L.gp_workspace_bytes(None, 10, 0, ctypes.byref(b)) == gp.GP_E_INVALID_ARG
    assert L.gp_pip(None, 10, None, None, None, 0, None, 0, None, None) == gp.GP_E_INVALID_ARG
    assert L.gp_p2p(None, 10, None, None, None, None, 0, None, 0, None, None) == gp.GP_E_INVALID_ARG
    opts = gp.gp_serve_opts(4, 1 << 20, 1 << 30, 1, 1, 1, 0)
    assert L.gp_serve_create(None, None, ctypes.byref(opts), ctypes.byref(out)) == gp.GP_E_INVALID_ARG
    assert L.gp_serve_destroy(None) == gp.GP_E_INVALID_ARG
    assert L.gp_set_tuning(None, 0, None) == gp.GP_E_INVALID_ARG
    assert L.gp_set_tuning(None, 0, ctypes.byref(gp.gp_tuning())) == gp.GP_E_INVALID_ARG


def test_oracle_and_gpu_path_share_no_code():
    """The HIP sources never include or name the oracle, and the oracle never loads the
    HIP library."""
    for sub in ("csrc", "cpu"):
        src = os.path.join(ROOT, "paper_1403_0802_amd", sub)
        for f in os.listdir(src):
            text = open(os.path.join(src, f)).read()
            assert "oracle" not in text.lower(), f
    pkg = os.path.join(ROOT, "paper_1403_0802_amd")
    for f in ("gp.py", "cpu.py", "build.py", "synth.py", "__init__.py"):
        assert "import oracle" not in open(os.path.join(pkg, f)).read()
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "libgp" not in text and "paper_1403_0802_amd.gp" not in text, f
