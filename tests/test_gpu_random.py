"""Randomised workloads through the C ABI against the oracle.

Each seed draws a geometry, a grid and points of its own:

* PIP: overlapping star polygons (some with star holes) at a random scale and a random
  offset of the coordinates from the origin; P2P: random-walk polylines with repeated
  vertices (zero-length segments) and polylines that share endpoints, at a random range D;
* grids from a few cells per feature to many, with an explicit extent (offset origin,
  points also outside it) or a derived one;
* points uniform over and around the extent, clustered, exactly on vertices and edge
  midpoints, level with vertices, and (P2P) near the polylines at about D.

Every case runs in both precision forms, on grids with and without build-time records,
with the default kernel shapes and with every few-point item vertex-parallel, and must
equal the oracle bit for bit (ids; P2P distances too).
"""
import numpy as np
import pytest

import oracle
from paper_1403_0802_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEEDS = range(24)


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_0802_amd import gp as gpmod
    return gpmod


def say(*a):
    print(*a, flush=True)


def random_pip(seed):
    rng = np.random.default_rng(9000 + seed)
    scale = float(10.0 ** rng.uniform(-3, 3))
    off = float(rng.choice([0.0, 1e2, -1e3, 1e4])) * scale
    xs, ys, roff, froff = [], [], [0], [0]
    for _ in range(int(rng.integers(5, 40))):
        cx, cy = off + rng.uniform(0, scale, 2)
        r = rng.uniform(0.02, 0.3) * scale
        m = int(rng.integers(12, 200))
        x, y, _, _ = synth.star_ring(rng, cx, cy, m, 0.6 * r, r)
        xs.append(x), ys.append(y), roff.append(roff[-1] + m)
        for _ in range(int(rng.integers(0, 3))):  # holes strictly inside the outer ring
            hx, hy = rng.uniform(-0.1, 0.1, 2) * r
            mh = int(rng.integers(3, 30))
            x, y, _, _ = synth.star_ring(rng, cx + hx, cy + hy, mh, 0.05 * r, 0.3 * r)
            xs.append(x[::-1]), ys.append(y[::-1]), roff.append(roff[-1] + mh)
        froff.append(len(roff) - 1)
    x, y = np.concatenate(xs), np.concatenate(ys)
    geom = synth.Geometry("pip", np.asarray(roff, np.int64), x, y, np.asarray(froff, np.int64))
    n = 20_000
    px = off + rng.uniform(-0.1, 1.1, n) * scale
    py = off + rng.uniform(-0.1, 1.1, n) * scale
    k = rng.integers(0, len(x), 3000)
    px[:1000], py[:1000] = x[k[:1000]], y[k[:1000]]  # on vertices
    nxt = np.minimum(k[1000:2000] + 1, len(x) - 1)
    px[1000:2000] = 0.5 * (x[k[1000:2000]] + x[nxt])  # edge midpoints (of ring neighbours)
    py[1000:2000] = 0.5 * (y[k[1000:2000]] + y[nxt])
    py[2000:3000] = y[k[2000:3000]]  # level with vertices
    return geom, px, py, scale, off, rng


def random_p2p(seed):
    rng = np.random.default_rng(9500 + seed)
    scale = float(10.0 ** rng.uniform(-2, 4))
    off = float(rng.choice([0.0, 1e2, -1e3])) * scale
    nl = int(rng.integers(20, 400))
    counts = rng.integers(2, 40, nl)
    g = synth.random_walk_polylines(rng, nl, counts, 0.0, scale, 0.001 * scale, 0.05 * scale)
    x, y = g.x + off, g.y + off
    # repeated vertices (zero-length segments) and polylines sharing an endpoint
    dup = rng.choice(len(x) - 1, len(x) // 20, replace=False)
    x[dup + 1], y[dup + 1] = x[dup], y[dup]
    first, last = g.ring_vert_off[1:-1], g.ring_vert_off[1:-1] - 1
    share = rng.random(len(first)) < 0.2
    x[first[share]], y[first[share]] = x[last[share]], y[last[share]]
    geom = synth.Geometry("p2p", g.ring_vert_off, x, y, None)
    D = float(rng.uniform(0.005, 0.05)) * scale
    n = 20_000
    px = off + rng.uniform(-0.1, 1.1, n) * scale
    py = off + rng.uniform(-0.1, 1.1, n) * scale
    k = rng.integers(0, len(x), 6000)
    px[:1000], py[:1000] = x[k[:1000]], y[k[:1000]]  # on vertices
    ang = rng.uniform(0, 2 * np.pi, 5000)
    rad = D * rng.uniform(0.9, 1.1, 5000)  # about D from a vertex
    px[1000:6000] = x[k[1000:]] + rad * np.cos(ang)
    py[1000:6000] = y[k[1000:]] + rad * np.sin(ang)
    return geom, px, py, scale, off, D, rng


def random_params(rng, scale, off, D=0.0):
    if rng.random() < 0.25:  # derived extent
        cs = scale / float(rng.choice([3, 16, 60]))
        return synth.GridParams(cell_size=cs, radius_D=D)
    ng = int(rng.choice([4, 16, 64, 200]))
    cs = scale / ng
    x0 = off - float(rng.uniform(0, 0.05)) * scale
    y0 = off - float(rng.uniform(0, 0.05)) * scale
    n = ng + 1  # points slightly beyond the far side stay outside the extent
    return synth.GridParams(cell_size=cs, radius_D=D, x0=x0, y0=y0, nx=n, ny=n)


def gpu_run(gp, grid, px, py, prec, tuning):
    gp.gp_reset_tuning(grid, prec)
    if tuning:
        gp.gp_set_tuning(grid, prec, **tuning)
    tx = torch.from_numpy(np.ascontiguousarray(px)).cuda()
    ty = torch.from_numpy(np.ascontiguousarray(py)).cuda()
    r = gp.run(grid, tx, ty, prec)
    torch.cuda.synchronize()
    if grid.kind == gp.GP_PIP:
        return r.cpu().numpy()
    return r[0].cpu().numpy(), r[1].cpu().numpy()


@pytest.mark.parametrize("seed", SEEDS)
def test_random_pip_equals_oracle(gp, seed):
    geom, px, py, scale, off, rng = random_pip(seed)
    params = random_params(rng, scale, off)
    og = oracle.build_grid(geom, params)
    want = oracle.pip(geom, px, py, og)
    inside = oracle.point_cells(og, px, py) >= 0
    # the grid only drops candidates that cannot matter: brute force agrees in the extent
    assert np.array_equal(want[inside], oracle.pip(geom, px[inside], py[inside]))
    say(f"pip seed {seed}: scale {scale:.3g}, offset {off:.3g}, cell {params.cell_size:.3g}, "
        f"{geom.n_features} polygons, {int(np.sum(want >= 0))} points inside")
    for pre in (0, 1):
        grid = gp.gp_build_grid("pip", geom, synth.GridParams(**{**params.__dict__,
                                                                 "prestage": pre}))
        for prec in ("fp64", "mixed"):
            for tuning in (None, dict(vp_points=64)):
                got = gpu_run(gp, grid, px, py, prec, tuning)
                assert np.array_equal(got, want), (seed, pre, prec, tuning,
                                                   int(np.sum(got != want)))


@pytest.mark.parametrize("seed", SEEDS)
def test_random_p2p_equals_oracle(gp, seed):
    geom, px, py, scale, off, D, rng = random_p2p(seed)
    params = random_params(rng, scale, off, D)
    og = oracle.build_grid(geom, params)
    want_id, want_d = oracle.p2p(geom, px, py, D, og)
    inside = oracle.point_cells(og, px, py) >= 0
    bid, bd = oracle.p2p(geom, px[inside], py[inside], D)
    assert np.array_equal(want_id[inside], bid) and np.array_equal(want_d[inside], bd)
    say(f"p2p seed {seed}: scale {scale:.3g}, offset {off:.3g}, D {D:.3g}, "
        f"cell {params.cell_size:.3g}, {geom.n_features} polylines, "
        f"{int(np.sum(want_id >= 0))} points in range")
    for pre in (0, 1):
        grid = gp.gp_build_grid("p2p", geom, synth.GridParams(**{**params.__dict__,
                                                                 "prestage": pre}))
        for prec in ("fp64", "mixed"):
            for tuning in (None, dict(vp_points=64)):
                got_id, got_d = gpu_run(gp, grid, px, py, prec, tuning)
                assert np.array_equal(got_id, want_id), (seed, pre, prec, tuning,
                                                         int(np.sum(got_id != want_id)))
                assert np.array_equal(got_d, want_d), (seed, pre, prec, tuning)


def test_signed_zero_coordinates(gp):
    """Points with -0.0 and +0.0 coordinates (equal values) against polygons whose
    vertices and edges lie on the axes, on a grid whose cell centre is the origin (the
    rebased coordinates are then exactly the inputs): the ids must not depend on the
    sign of a zero."""
    rings = [  # (outer ring, holes)
        ([(-2, -2), (2, -2), (2, 2), (-2, 2)], [[(-1, 0), (0, -1), (1, 0), (0, 1)]]),
        ([(0, 0), (3, 0), (3, 3)], []),
        ([(-5, -5), (5, -5), (5, 5), (2, 5), (1, 0), (0.8, 5), (-5, 5)], []),
        ([(1, 0), (3, 0), (3, 1), (1, 1)], []),
        ([(0, -3), (0.5, 0), (0, 3), (-0.5, 0)], []),
    ]
    xs, ys, roff, froff = [], [], [0], [0]
    for outer, holes in rings:
        for ring in [outer] + holes:
            xs += [float(v[0]) for v in ring]
            ys += [float(v[1]) for v in ring]
            roff.append(roff[-1] + len(ring))
        froff.append(len(roff) - 1)
    geom = synth.Geometry("pip", np.asarray(roff, np.int64), np.asarray(xs), np.asarray(ys),
                          np.asarray(froff, np.int64))
    vals = [-0.0, 0.0, -1e-300, 1e-300, 0.5, -0.5, 1.0, -1.0, 0.8, 2.0, -2.0, 3.0]
    px = np.array([a for a in vals for b in vals])
    py = np.array([b for a in vals for b in vals])
    params = synth.GridParams(cell_size=1.0, x0=-6.5, y0=-6.5, nx=13, ny=13)
    want = oracle.pip(geom, px, py, oracle.build_grid(geom, params))
    assert np.array_equal(want, oracle.pip(geom, px, py))
    # the definition itself ignores the sign of a zero (x + 0.0 turns -0.0 into +0.0)
    assert np.array_equal(want, oracle.pip(geom, px + 0.0, py + 0.0))
    for pre in (0, 1):
        grid = gp.gp_build_grid("pip", geom, synth.GridParams(**{**params.__dict__,
                                                                 "prestage": pre}))
        for prec in ("fp64", "mixed"):
            for tuning in (None, dict(vp_points=-1), dict(vp_points=64)):
                got = gpu_run(gp, grid, px, py, prec, tuning)
                assert np.array_equal(got, want), (pre, prec, tuning, int(np.sum(got != want)))


@pytest.mark.parametrize("seed", range(3))
def test_pip_item_sizes(gp, seed):
    """Every count of points per cell from 1 to 300 (so every split of a cell into items:
    full items and remainders of every size, each run with the fewest points per lane that
    hold it), on overlapping star polygons with holes, with points level with and on
    vertices inside each cell: the prestaged mixed form equals the oracle, with and
    without the vertex-parallel path for few-point items, at 1, 2 and 4 points per lane."""
    rng = np.random.default_rng(7100 + seed)
    xs, ys, roff, froff = [], [], [0], [0]
    for _ in range(12):
        cx, cy = rng.uniform(2, 18, 2)
        r = rng.uniform(2, 6)
        m = int(rng.integers(20, 300))
        x, y, _, _ = synth.star_ring(rng, cx, cy, m, 0.5 * r, r)
        xs.append(x), ys.append(y), roff.append(roff[-1] + m)
        if rng.random() < 0.5:
            mh = int(rng.integers(3, 40))
            x, y, _, _ = synth.star_ring(rng, cx, cy, mh, 0.05 * r, 0.4 * r)
            xs.append(x[::-1]), ys.append(y[::-1]), roff.append(roff[-1] + mh)
        froff.append(len(roff) - 1)
    vx, vy = np.concatenate(xs), np.concatenate(ys)
    geom = synth.Geometry("pip", np.asarray(roff, np.int64), vx, vy, np.asarray(froff, np.int64))
    params = synth.GridParams(cell_size=1.0, x0=0.0, y0=0.0, nx=20, ny=20)
    counts = rng.permutation(np.arange(1, 401)) % 300 + 1  # 400 cells, every count 1..300
    pxs, pys = [], []
    for c, k in enumerate(counts):
        i, j = c % 20, c // 20
        px = i + rng.uniform(0, 1, k)
        py = j + rng.uniform(0, 1, k)
        inside = np.nonzero((vx >= i) & (vx < i + 1) & (vy >= j) & (vy < j + 1))[0]
        if len(inside) and k >= 4:
            q = rng.choice(inside, k // 4)
            py[: k // 4] = vy[q]  # level with a vertex of the cell
            px[k // 8: k // 4] = vx[q[k // 8:]]  # on the vertex itself
        pxs.append(px), pys.append(py)
    px, py = np.concatenate(pxs), np.concatenate(pys)
    og = oracle.build_grid(geom, params)
    want = oracle.pip(geom, px, py, og)
    say(f"item sizes seed {seed}: {len(px)} points, {int(np.sum(want >= 0))} inside")
    grid = gp.gp_build_grid("pip", geom, synth.GridParams(**{**params.__dict__, "prestage": 1}))
    for tuning in (dict(vp_points=-1), None, dict(points_per_lane=1, vp_points=-1),
                   dict(points_per_lane=4, vp_points=-1)):
        got = gpu_run(gp, grid, px, py, "mixed", tuning)
        assert np.array_equal(got, want), (seed, tuning, int(np.sum(got != want)))


@pytest.mark.parametrize("seed", range(2))
def test_p2p_item_sizes(gp, seed):
    """P2P with every count of points per cell from 1 to 600 (full 256-point items and
    remainders of every size), points near the polylines, on the vertices and at about D
    from them: ids and distances equal the oracle's in both precision forms, with and
    without build-time records and the vertex-parallel path, at 1, 2 and 4 points per
    lane and with two waves per item."""
    rng = np.random.default_rng(7300 + seed)
    nl = 150
    g = synth.random_walk_polylines(rng, nl, rng.integers(2, 30, nl), 0.0, 24.0, 0.05, 0.6)
    geom = synth.Geometry("p2p", g.ring_vert_off, g.x, g.y, None)
    D = 0.7
    # unit cells over the polylines' boxes grown by D, and one more cell on each side
    x0, y0 = np.floor(g.x.min() - D) - 1.0, np.floor(g.y.min() - D) - 1.0
    nx, ny = int(np.ceil(g.x.max() + D) - x0) + 1, int(np.ceil(g.y.max() + D) - y0) + 1
    assert nx * ny >= 600
    params = synth.GridParams(cell_size=1.0, radius_D=D, x0=x0, y0=y0, nx=nx, ny=ny)
    counts = rng.permutation(np.arange(1, nx * ny + 1)) % 600 + 1  # every count 1..600
    pxs, pys = [], []
    for c, k in enumerate(counts):
        i, j = c % nx, c // nx
        px = x0 + i + rng.uniform(0, 1, k)
        py = y0 + j + rng.uniform(0, 1, k)
        near = np.nonzero((g.x >= px.min()) & (g.x < px.max()) &
                          (g.y >= py.min()) & (g.y < py.max()))[0]
        if len(near) and k >= 4:
            q = rng.choice(near, k // 2)
            ang = rng.uniform(0, 2 * np.pi, k // 2)
            rad = np.where(np.arange(k // 2) % 4 == 0, 0.0, D * rng.uniform(0.98, 1.02, k // 2))
            px[: k // 2] = g.x[q] + rad * np.cos(ang)
            py[: k // 2] = g.y[q] + rad * np.sin(ang)
        pxs.append(px), pys.append(py)
    px, py = np.concatenate(pxs), np.concatenate(pys)
    og = oracle.build_grid(geom, params)
    want_id, want_d = oracle.p2p(geom, px, py, D, og)
    say(f"p2p item sizes seed {seed}: {len(px)} points, {int(np.sum(want_id >= 0))} in range")
    for pre in (0, 1):
        grid = gp.gp_build_grid("p2p", geom, synth.GridParams(**{**params.__dict__,
                                                                 "prestage": pre}))
        for prec, tunings in (("mixed", (None, dict(vp_points=-1), dict(points_per_lane=1),
                                         dict(points_per_lane=2, vp_points=-1),
                                         dict(points_per_lane=4, waves_per_item=2))),
                              ("fp64", (None, dict(points_per_lane=4, vp_points=-1)))):
            for tuning in tunings:
                got_id, got_d = gpu_run(gp, grid, px, py, prec, tuning)
                assert np.array_equal(got_id, want_id), (seed, pre, prec, tuning,
                                                         int(np.sum(got_id != want_id)))
                assert np.array_equal(got_d, want_d), (seed, pre, prec, tuning)
