"""Reader of the hand-written closed-form fixtures under tests/golden/."""
from __future__ import annotations

import dataclasses
import os

import numpy as np

from paper_1403_0802_amd.synth import Geometry

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@dataclasses.dataclass
class GoldenCase:
    name: str
    kind: str
    geom: Geometry
    radius: float
    px: np.ndarray
    py: np.ndarray
    want_id: np.ndarray
    want_dist: np.ndarray | None


def _xy(tokens):
    return [tuple(float(v) for v in t.split(",")) for t in tokens]


def load(name: str) -> GoldenCase:
    kind, radius = None, 0.0
    rings, pts = [], []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "kind":
            kind = tok[1]
        elif tok[0] == "radius":
            radius = float(tok[1])
        elif tok[0] in ("ring", "line"):
            rings.append((int(tok[1]), _xy(tok[2:])))
        elif tok[0] == "point":
            pts.append(tok[1:])
        else:
            raise ValueError(f"{name}: unknown record {tok[0]!r}")
    fids = [f for f, _ in rings]
    assert fids == sorted(fids) and sorted(set(fids)) == list(range(len(set(fids)))), name
    xs = np.concatenate([np.array([v[0] for v in r]) for _, r in rings])
    ys = np.concatenate([np.array([v[1] for v in r]) for _, r in rings])
    roff = np.cumsum([0] + [len(r) for _, r in rings]).astype(np.int64)
    if kind == "pip":
        fro = np.searchsorted(np.asarray(fids), np.arange(len(set(fids)) + 1)).astype(np.int64)
        geom = Geometry("pip", roff, xs, ys, fro)
    else:
        assert fids == list(range(len(fids))), f"{name}: one chain per polyline"
        geom = Geometry("p2p", roff, xs, ys, None)
    px = np.array([float(p[0]) for p in pts])
    py = np.array([float(p[1]) for p in pts])
    want_id = np.array([int(p[2]) for p in pts], dtype=np.int32)
    want_d = None
    if kind == "p2p":
        want_d = np.array([float(p[3]) for p in pts])
    return GoldenCase(name, kind, geom, radius, px, py, want_id, want_d)


ALL = ["pip_squares_triangle.txt", "p2p_segments.txt"]
