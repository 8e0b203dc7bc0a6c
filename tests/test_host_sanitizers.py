"""The host C/C++ code (the oracle and the host SIMD library) built with AddressSanitizer
and UndefinedBehaviorSanitizer, then run on pins and on the host library's checks in a
child process that preloads the ASan runtime.  Any out-of-bounds access, use after free
or undefined operation aborts the child (and fails the test).  CPU only."""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle
from paper_1403_0802_amd import build as gpbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle
    from paper_1403_0802_amd import cpu, synth
    from tests import pins
    lib = oracle.load({olib!r})
    for pin in (pins.pin_pip_boxes, pins.pin_pip_hole, pins.pin_pip_convex,
                pins.pin_pip_grid_equals_brute, pins.pin_p2p_single_segment,
                pins.pin_p2p_ties_and_range, pins.pin_p2p_grid_equals_brute,
                pins.pin_grid_definition, pins.pin_pip_count_overlaps, pins.pin_golden):
        pin(lib)
        print("pin ok", pin.__name__, flush=True)
    cpu.lib = cpu.ctypes.CDLL({clib!r})
    cpu.lib.gp_cpu_join.argtypes = cpu._load().gp_cpu_join.argtypes
    cpu.lib.gp_cpu_join.restype = cpu.ctypes.c_int32
    cpu.lib.gp_cpu_has_simd.restype = cpu.ctypes.c_int32
    w1 = synth.config1(n_points=5_003, grid_n=4, seed_salt=2)
    w2 = synth.config2(n_points=5_003, n_lines=400, seed_salt=5)
    for w in (w1, w2):
        want = oracle.run(w, lib=lib)[1:]
        for mode in ("sc", "mc", "sc_simd", "mc_simd"):
            got = cpu.gp_cpu_join(w.kind, w.geom, w.params, w.px, w.py, mode)
            assert np.array_equal(got[0], want[0]), (w.kind, mode)
            if w.kind == "p2p":
                assert np.array_equal(got[1], want[1]), mode
            print("host", w.kind, mode, "ok", flush=True)
    print("ALL OK", flush=True)
""")


def test_oracle_and_host_library_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime for gcc")
    olib = str(tmp_path / "liboracle_san.so")
    oracle.build(out=olib, extra=SAN)
    clib = str(tmp_path / "libgp_cpu_san.so")
    r = subprocess.run(["g++", *gpbuild.CPU_FLAGS, *SAN, gpbuild.CPU_SRC, "-o", clib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = CHILD.format(root=ROOT, olib=olib, clib=clib)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ALL OK" in r.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
