"""Seeded synthetic workloads that stand in for the paper's datasets.

The paper measures P2P on NYC taxi pickups against the LION street network and PIP
on GBIF occurrence points against WWF ecoregions (Sec. IV.A).  Neither dataset is
available, so these generators produce inputs with the same structure: points
clustered at hot spots against short random-walk polylines (P2P), and scattered plus
clustered points against a watertight tessellation of non-convex polygons with
holes and heavy-tailed vertex counts (PIP).

This module only *draws inputs*.  It holds none of the join's arithmetic (no
crossing test, no distance, no grid hashing), so both the HIP path and the CPU
oracle can consume its output without sharing any of the method's code.

Every workload is seeded with ``numpy.random.Generator(PCG64(14030802 + k))`` for
configuration ``k`` (1..5), so a given call always returns identical arrays.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 14030802


@dataclasses.dataclass
class Geometry:
    """Polygons (multi-ring) or polylines in SoA + CSR form, FP64.

    ``feature_ring_off[f] .. feature_ring_off[f+1]`` are the rings of polygon ``f``
    (ring 0 is the outer ring); it is ``None`` for polylines, where every feature is
    a single vertex chain.  ``ring_vert_off[r] .. ring_vert_off[r+1]`` index ``x``/``y``.
    """

    kind: str  # "pip" or "p2p"
    ring_vert_off: np.ndarray  # int64 [n_rings + 1]
    x: np.ndarray  # float64 [n_vertices]
    y: np.ndarray  # float64 [n_vertices]
    feature_ring_off: Optional[np.ndarray] = None  # int64 [n_features + 1]

    @property
    def n_features(self) -> int:
        if self.feature_ring_off is None:
            return len(self.ring_vert_off) - 1
        return len(self.feature_ring_off) - 1

    @property
    def n_rings(self) -> int:
        return len(self.ring_vert_off) - 1

    @property
    def n_vertices(self) -> int:
        return len(self.x)


@dataclasses.dataclass
class GridParams:
    cell_size: float
    radius_D: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    nx: int = 0  # 0: derive the extent from the (expanded) MBBs
    ny: int = 0
    cell_classes: int = 0  # PIP: 1 asks the GPU grid to classify cell/polygon pairs
    segment_filter: int = 0  # P2P: 1 asks the GPU grid for per-cell segment lists
    prestage: int = 0  # 1 asks the GPU grid for build-time mixed-form records (both kinds)


@dataclasses.dataclass
class Workload:
    name: str
    kind: str
    geom: Geometry
    px: np.ndarray
    py: np.ndarray
    params: GridParams
    info: dict


def _rng(k: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + k + 1000003 * salt))


# --------------------------------------------------------------------------- points


def gaussian_mixture_points(rng, n, centers, sigmas, lo, hi, chunk=8_000_000):
    """``n`` points from an equal-weight isotropic Gaussian mixture, rejection-clipped
    to the half-open box ``[lo, hi)^2``."""
    centers = np.asarray(centers, dtype=np.float64)
    sigmas = np.broadcast_to(np.asarray(sigmas, dtype=np.float64), (len(centers),))
    px = np.empty(n, dtype=np.float64)
    py = np.empty(n, dtype=np.float64)
    filled = 0
    while filled < n:
        m = min(chunk, n - filled)
        comp = rng.integers(0, len(centers), size=m, dtype=np.int32)
        s = sigmas[comp]
        x = centers[comp, 0] + s * rng.standard_normal(m)
        y = centers[comp, 1] + s * rng.standard_normal(m)
        ok = (x >= lo) & (x < hi) & (y >= lo) & (y < hi)
        k = int(ok.sum())
        take = min(k, n - filled)
        px[filled:filled + take] = x[ok][:take]
        py[filled:filled + take] = y[ok][:take]
        filled += take
    return px, py


def uniform_points(rng, n, lo, hi):
    px = rng.uniform(lo, hi, size=n)
    py = rng.uniform(lo, hi, size=n)
    # uniform() can return hi only through rounding; keep the box half-open.
    np.minimum(px, np.nextafter(hi, lo), out=px)
    np.minimum(py, np.nextafter(hi, lo), out=py)
    return px, py


# --------------------------------------------------------------------------- shapes


def star_ring(rng, cx, cy, m, r_lo, r_hi):
    """A simple star-shaped ring: ``m`` vertices at sorted distinct random angles,
    each at its own random radius in ``(r_lo, r_hi)`` from ``(cx, cy)``."""
    while True:
        th = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=m))
        if np.all(np.diff(th) > 0):
            break
    r = rng.uniform(r_lo, r_hi, size=m)
    return cx + r * np.cos(th), cy + r * np.sin(th), th, r


def random_walk_polylines(rng, n_lines, counts, lo, hi, step_lo, step_hi):
    """Polylines that start uniformly in ``[lo, hi]^2`` and take ``counts[i]-1`` steps of
    length ``U[step_lo, step_hi]`` at i.i.d. uniform headings."""
    counts = np.asarray(counts, dtype=np.int64)
    off = np.zeros(n_lines + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    nv = int(off[-1])
    sx = rng.uniform(lo, hi, size=n_lines)
    sy = rng.uniform(lo, hi, size=n_lines)
    step = rng.uniform(step_lo, step_hi, size=nv)
    head = rng.uniform(0.0, 2.0 * math.pi, size=nv)
    dx = step * np.cos(head)
    dy = step * np.sin(head)
    first = off[:-1]
    dx[first] = 0.0
    dy[first] = 0.0
    cx = np.cumsum(dx)
    cy = np.cumsum(dy)
    # restart the running sum at each polyline's first vertex
    base_x = np.repeat(cx[first], counts)
    base_y = np.repeat(cy[first], counts)
    x = np.repeat(sx, counts) + (cx - base_x)
    y = np.repeat(sy, counts) + (cy - base_y)
    return Geometry("p2p", off, x, y, None)


# --------------------------------------------------------------------------- configs


def config1(n_points=50_000, grid_n=8, seed_salt=0):
    """PIP, plain FP64: points uniform in [0,1)^2; one star polygon per cell of a
    ``grid_n`` x ``grid_n`` grid (vertex counts U{16..256}, radius 0.3-0.5 of a cell)."""
    rng = _rng(1, seed_salt)
    xs, ys, roff = [], [], [0]
    w = 1.0 / grid_n
    for r in range(grid_n):
        for c in range(grid_n):
            m = int(rng.integers(16, 257))
            x, y, _, _ = star_ring(rng, (c + 0.5) * w, (r + 0.5) * w, m, 0.3 * w, 0.5 * w)
            xs.append(x)
            ys.append(y)
            roff.append(roff[-1] + m)
    nf = grid_n * grid_n
    geom = Geometry("pip", np.asarray(roff, np.int64), np.concatenate(xs), np.concatenate(ys),
                    np.arange(nf + 1, dtype=np.int64))
    px, py = uniform_points(rng, n_points, 0.0, 1.0)
    params = GridParams(cell_size=1.0 / 64, x0=0.0, y0=0.0, nx=64, ny=64)
    return Workload("c1_pip_stars", "pip", geom, px, py, params,
                    {"n_points": n_points, "n_polygons": nf, "n_vertices": geom.n_vertices})


def _mixture_plane_points(rng, n, n_comp=32, sigma=500.0, side=40_000.0):
    centers = rng.uniform(2000.0, side - 2000.0, size=(n_comp, 2))
    return gaussian_mixture_points(rng, n, centers, sigma, 0.0, side)


def config2(n_points=1_000_000, n_lines=20_000, seed_salt=0):
    """P2P, plain FP64: 32-component Gaussian mixture (sigma 500 m) in a 40 km plane;
    random-walk polylines of U{2..64} vertices with 10-200 m steps; D = 50 m."""
    rng = _rng(2, seed_salt)
    px, py = _mixture_plane_points(rng, n_points)
    counts = rng.integers(2, 65, size=n_lines)
    geom = random_walk_polylines(rng, n_lines, counts, 0.0, 40_000.0, 10.0, 200.0)
    params = GridParams(cell_size=100.0, radius_D=50.0, x0=0.0, y0=0.0, nx=400, ny=400)
    return Workload("c2_p2p_walks", "p2p", geom, px, py, params,
                    {"n_points": n_points, "n_polylines": n_lines, "n_vertices": geom.n_vertices})


def _voronoi_tessellation(rng, n_seeds, median_v, sigma_v, max_v, hole_frac, share=0.5):
    """Watertight tessellation of the unit square: clipped Voronoi cells whose shared
    edges are subdivided once with tapered perpendicular jitter and reused (reversed)
    by both neighbours; ~``hole_frac`` of the cells get 1-3 star holes."""
    from scipy.spatial import Voronoi

    seeds = rng.uniform(0.0, 1.0, size=(n_seeds, 2))
    # mirror the seeds across the four sides so every original cell is bounded and
    # clipped exactly at the unit-square boundary
    mir = [seeds,
           np.c_[-seeds[:, 0], seeds[:, 1]], np.c_[2.0 - seeds[:, 0], seeds[:, 1]],
           np.c_[seeds[:, 0], -seeds[:, 1]], np.c_[seeds[:, 0], 2.0 - seeds[:, 1]]]
    vor = Voronoi(np.concatenate(mir))
    V = vor.vertices.copy()
    for col in (0, 1):
        c = V[:, col]
        c[np.abs(c) < 1e-9] = 0.0
        c[np.abs(c - 1.0) < 1e-9] = 1.0

    rings = []  # per seed: list of Voronoi vertex ids in order
    for i in range(n_seeds):
        reg = vor.regions[vor.point_region[i]]
        assert -1 not in reg and len(reg) >= 3
        rings.append(list(reg))

    # per-polygon vertex targets, log-normal, one forced to the maximum
    targets = np.clip(np.rint(np.exp(math.log(median_v) + sigma_v * rng.standard_normal(n_seeds))),
                      8, max_v).astype(np.int64)
    forced = int(rng.integers(0, n_seeds))
    targets[forced] = max_v

    def interior_angle(ring, k):
        a = V[ring[k - 1]]
        b = V[ring[k]]
        c = V[ring[(k + 1) % len(ring)]]
        u, v = a - b, c - b
        cosang = np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v))
        return math.acos(max(-1.0, min(1.0, cosang)))

    edge_info = {}  # (min,max) vertex ids -> dict(desired=int, theta=float, dseed=float, length)
    for i, ring in enumerate(rings):
        m = len(ring)
        pts = V[ring]
        per = float(np.sum(np.linalg.norm(pts - np.roll(pts, -1, axis=0), axis=1)))
        angs = [interior_angle(ring, k) for k in range(m)]
        for k in range(m):
            u, v = ring[k], ring[(k + 1) % m]
            key = (min(u, v), max(u, v))
            L = float(np.linalg.norm(V[v] - V[u]))
            sh = 1.0 if i == forced else share
            want = max(0, int(round(sh * targets[i] * L / per)) - 1)
            # distance from the seed to the edge's supporting line
            d = V[v] - V[u]
            nrm = np.array([-d[1], d[0]]) / max(L, 1e-300)
            dseed = abs(float(np.dot(seeds[i] - V[u], nrm)))
            th = min(angs[k], angs[(k + 1) % m])
            e = edge_info.setdefault(key, {"want": 0, "theta": math.pi, "dseed": math.inf,
                                           "L": L, "owners": 0})
            e["want"] = max(e["want"], want)
            e["theta"] = min(e["theta"], th)
            e["dseed"] = min(e["dseed"], dseed)
            e["owners"] += 1

    # materialise the subdivided vertices of each edge, oriented from key[0] to key[1]
    edge_pts = {}
    edge_amp = {}
    for key, e in edge_info.items():
        s = e["want"]
        a, b = V[key[0]], V[key[1]]
        if s == 0:
            edge_pts[key] = np.empty((0, 2))
            edge_amp[key] = 0.0
            continue
        t = np.arange(1, s + 1, dtype=np.float64) / (s + 1)
        base = a[None, :] + t[:, None] * (b - a)[None, :]
        if e["owners"] == 2:  # shared edge: jitter; the unit-square sides stay straight
            L = e["L"]
            amp = min(0.05 * L, 0.087 * e["theta"] * L, 0.3 * e["dseed"])
            f1 = int(rng.integers(1, 4))
            ph = rng.uniform(0.0, 2.0 * math.pi)
            prof = 0.7 * np.sin(2.0 * math.pi * f1 * t + ph) + 0.3 * rng.uniform(-1.0, 1.0, size=s)
            off = amp * np.sin(math.pi * t) ** 2 * prof
            d = (b - a) / L
            nrm = np.array([-d[1], d[0]])
            base = base + off[:, None] * nrm[None, :]
            edge_amp[key] = amp
        else:
            edge_amp[key] = 0.0
        edge_pts[key] = base

    xs, ys, roff, froff = [], [], [0], [0]
    n_holes_total = 0
    for i, ring in enumerate(rings):
        m = len(ring)
        parts = []
        dmin = math.inf
        for k in range(m):
            u, v = ring[k], ring[(k + 1) % m]
            key = (min(u, v), max(u, v))
            parts.append(V[u][None, :])
            ep = edge_pts[key]
            parts.append(ep if u == key[0] else ep[::-1])
            # distance from the seed to the edge segment, minus its jitter envelope
            a, b = V[u], V[v]
            ab = b - a
            tt = np.clip(np.dot(seeds[i] - a, ab) / max(np.dot(ab, ab), 1e-300), 0.0, 1.0)
            dmin = min(dmin, float(np.linalg.norm(seeds[i] - (a + tt * ab))) - edge_amp[key])
        outer = np.concatenate(parts)
        xs.append(outer[:, 0])
        ys.append(outer[:, 1])
        roff.append(roff[-1] + len(outer))
        nr = 1
        if rng.uniform() < hole_frac and dmin > 0:
            rho = 0.8 * dmin
            k_h = int(rng.integers(1, 4))
            phi0 = rng.uniform(0.0, 2.0 * math.pi)
            for j in range(k_h):
                if k_h == 1:
                    c = seeds[i]
                    rmax = 0.5 * rho
                else:
                    phi = phi0 + 2.0 * math.pi * j / k_h
                    c = seeds[i] + 0.5 * rho * np.array([math.cos(phi), math.sin(phi)])
                    rmax = 0.4 * rho * math.sin(math.pi / k_h)
                mh = int(rng.integers(8, 65))
                hx, hy, _, _ = star_ring(rng, c[0], c[1], mh, 0.6 * rmax, rmax)
                xs.append(hx)
                ys.append(hy)
                roff.append(roff[-1] + mh)
                nr += 1
                n_holes_total += 1
        froff.append(froff[-1] + nr)
    geom = Geometry("pip", np.asarray(roff, np.int64), np.concatenate(xs), np.concatenate(ys),
                    np.asarray(froff, np.int64))
    return geom, {"n_holes": n_holes_total, "targets_median": float(np.median(targets))}


def config3_geometry(n_polygons=5_000, median_v=200, sigma_v=1.1, max_v=50_000, hole_frac=0.10,
                     seed_salt=0):
    rng = _rng(3, seed_salt)
    geom, info = _voronoi_tessellation(rng, n_polygons, median_v, sigma_v, max_v, hole_frac)
    return geom, info


def config3_points(n_points, seed_salt=0, request=None):
    """70% from a 1,000-component mixture (sigma log-uniform 0.002-0.02), 30% uniform,
    all in [0,1)^2.  ``request`` draws an independent stream for serving requests."""
    rng = _rng(3, 7 + seed_salt) if request is None else _rng(5, 1 + 2 * int(request))
    crng = _rng(3, 5)  # the cluster layout is fixed for the configuration
    centers = crng.uniform(0.0, 1.0, size=(1000, 2))
    sig = np.exp(crng.uniform(math.log(0.002), math.log(0.02), size=1000))
    n_c = int(round(0.7 * n_points))
    cx, cy = gaussian_mixture_points(rng, n_c, centers, sig, 0.0, 1.0)
    ux, uy = uniform_points(rng, n_points - n_c, 0.0, 1.0)
    px = np.concatenate([cx, ux])
    py = np.concatenate([cy, uy])
    perm = rng.permutation(n_points)
    return px[perm], py[perm]


def config3(n_points=50_000_000, n_polygons=5_000, max_v=50_000, grid_n=1024, seed_salt=0):
    """PIP at scale: Voronoi tessellation with jittered shared edges, log-normal vertex
    counts (median 200, max ``max_v``), 10% of polygons with 1-3 holes."""
    geom, ginfo = config3_geometry(n_polygons, max_v=max_v, seed_salt=seed_salt)
    px, py = config3_points(n_points, seed_salt)
    params = GridParams(cell_size=1.0 / grid_n, x0=0.0, y0=0.0, nx=grid_n, ny=grid_n)
    info = {"n_points": n_points, "n_polygons": n_polygons, "n_vertices": geom.n_vertices,
            "n_rings": geom.n_rings, **ginfo}
    return Workload("c3_pip_voronoi", "pip", geom, px, py, params, info)


def config4_geometry(n_lines=200_000, median_v=16, sigma_v=1.0, max_v=512, seed_salt=0):
    rng = _rng(4, seed_salt)
    counts = np.clip(np.rint(np.exp(math.log(median_v) + sigma_v * rng.standard_normal(n_lines))),
                     2, max_v).astype(np.int64)
    return random_walk_polylines(rng, n_lines, counts, 0.0, 40_000.0, 10.0, 200.0)


def config4_points(n_points, seed_salt=0, request=None):
    rng = _rng(4, 7 + seed_salt) if request is None else _rng(5, 2 + 2 * int(request))
    crng = _rng(4, 5)
    centers = crng.uniform(2000.0, 38_000.0, size=(32, 2))
    return gaussian_mixture_points(rng, n_points, centers, 500.0, 0.0, 40_000.0)


def config4(n_points=200_000_000, n_lines=200_000, seed_salt=0):
    """P2P at scale: 32-component mixture points in a 40 km plane; random-walk polylines
    with log-normal vertex counts (median 16, clipped to [2, 512]); D = 100 m."""
    geom = config4_geometry(n_lines, seed_salt=seed_salt)
    px, py = config4_points(n_points, seed_salt)
    params = GridParams(cell_size=100.0, radius_D=100.0, x0=0.0, y0=0.0, nx=400, ny=400)
    return Workload("c4_p2p_walks", "p2p", geom, px, py, params,
                    {"n_points": n_points, "n_polylines": n_lines, "n_vertices": geom.n_vertices})


def serving_stream(n_requests, rate_per_s, min_pts=1_000, max_pts=4_000_000, seed_salt=0):
    """Configuration 5: a Poisson request stream.  Each entry is
    ``(arrival_s, kind, n_points, request_index)``; sizes are log-uniform, kinds 50/50."""
    rng = _rng(5, seed_salt)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    sizes = np.exp(rng.uniform(math.log(min_pts), math.log(max_pts), size=n_requests)).astype(np.int64)
    kinds = np.where(rng.uniform(size=n_requests) < 0.5, "pip", "p2p")
    return [(float(t[i]), str(kinds[i]), int(sizes[i]), i) for i in range(n_requests)]


def request_points(kind, n, request_index):
    if kind == "pip":
        return config3_points(n, request=request_index)
    return config4_points(n, request=request_index)
