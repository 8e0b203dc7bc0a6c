"""The host multi-core / AVX-512 implementation (libgp_cpu.so) against the oracle: every
mode (single core, multi-core, each with and without SIMD) returns the oracle's ids and
distances bit for bit, including partial SIMD blocks, holes, ties, degenerate segments
and points off the grid."""
import numpy as np
import pytest

import oracle
from paper_1403_0802_amd import synth
from tests import pins

MODES = ["sc", "mc", "sc_simd", "mc_simd"]


@pytest.fixture(scope="module")
def cpu():
    from paper_1403_0802_amd import cpu as cpumod
    return cpumod


@pytest.mark.parametrize("mode", MODES)
def test_pip_c1_all_modes(cpu, mode):
    w = synth.config1(n_points=30_000, grid_n=6, seed_salt=2)
    _, want = oracle.run(w)
    got, _, st = cpu.gp_cpu_join("pip", w.geom, w.params, w.px, w.py, mode)
    assert np.array_equal(got, want), np.sum(got != want)
    assert st["tests"] == oracle.test_count(oracle.build_grid(w.geom, w.params), w.px, w.py)
    assert st["simd"] == (mode.endswith("simd") and cpu.gp_cpu_has_simd())


@pytest.mark.parametrize("mode", MODES)
def test_pip_holes_overlaps_off_grid(cpu, mode):
    rng = np.random.default_rng(21)
    sq = pins.box(0.2, 0.2, 0.8, 0.8)
    hole = pins.box(0.3, 0.3, 0.7, 0.7, ccw=False)
    dup = pins.box(0.1, 0.6, 0.4, 0.9) + [(0.1, 0.6)]
    g = pins.polygons([[sq, hole], [dup], [pins.box(0.25, 0.25, 0.5, 0.5)]])
    params = synth.GridParams(cell_size=1 / 16, nx=14, ny=15)  # part of the square is off-grid
    px, py = rng.uniform(-0.1, 1.1, (2, 20_003))
    px[:5] = [0.2, 0.8, 0.3, np.nan, 0.5]
    py[:5] = [0.5, 0.5, 0.3, 0.5, np.inf]
    want = oracle.pip(g, px, py, oracle.build_grid(g, params))
    got, _, _ = cpu.gp_cpu_join("pip", g, params, px, py, mode)
    assert np.array_equal(got, want), np.sum(got != want)


@pytest.mark.parametrize("mode", MODES)
def test_p2p_all_modes(cpu, mode):
    w = synth.config2(n_points=40_001, n_lines=1_500, seed_salt=5)
    _, want_id, want_d = oracle.run(w)
    gid, gd, _ = cpu.gp_cpu_join("p2p", w.geom, w.params, w.px, w.py, mode)
    assert np.array_equal(gid, want_id)
    assert np.array_equal(gd, want_d)


@pytest.mark.parametrize("mode", MODES)
def test_p2p_ties_degenerate_derived_extent(cpu, mode):
    lines = [[(0.0, 2.0), (10.0, 2.0)], [(0.0, -2.0), (10.0, -2.0)],
             [(3.0, 3.0), (3.0, 3.0), (4.0, 3.5)], [(20.0, 20.0)] * 3]
    g = pins.polylines(lines)
    params = synth.GridParams(cell_size=1.0, radius_D=2.0)  # derived extent
    rng = np.random.default_rng(2)
    px = np.concatenate([[5.0, 5.0, 20.0, 3.0], rng.uniform(-5, 25, 9_999)])
    py = np.concatenate([[0.0, 4.0, 20.0, 1.0], rng.uniform(-5, 25, 9_999)])
    og = oracle.build_grid(g, params)
    want_id, want_d = oracle.p2p(g, px, py, params.radius_D, og)
    gid, gd, _ = cpu.gp_cpu_join("p2p", g, params, px, py, mode)
    assert np.array_equal(gid, want_id) and np.array_equal(gd, want_d)


def test_bad_arguments(cpu):
    w = synth.config1(n_points=10, grid_n=2)
    with pytest.raises(Exception):
        cpu.gp_cpu_join("pip", w.geom, w.params, w.px, w.py, 9)
    bad = synth.GridParams(cell_size=0.0)
    with pytest.raises(Exception):
        cpu.gp_cpu_join("pip", w.geom, bad, w.px, w.py, "sc")
