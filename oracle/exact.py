"""Exact rational geometry for pinning the FP64 oracle on tiny inputs -- TEST ONLY.

``fractions.Fraction(float)`` is exact for binary64 values, so everything here is
evaluated without rounding.  The formulations deliberately differ from the oracle's:

* ``inside_exact`` decides each crossing with an exact orientation sign;
* ``winding_number`` is the signed crossing count (a different rule that agrees
  with even-odd parity off the boundary of a simple ring);
* ``segment_d2_exact`` clamps the exact projection parameter to [0, 1] instead of
  branching on the unnormalised dot product.
"""
from __future__ import annotations

from fractions import Fraction as Fr


def _orient(ax, ay, bx, by, px, py):
    """Twice the signed area of (a, b, p): > 0 when p is left of a->b."""
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


def ring_crossings_exact(px, py, ring):
    """Number of ring edges crossed by the +x ray from p (half-open in y)."""
    px, py = Fr(px), Fr(py)
    pts = [(Fr(x), Fr(y)) for x, y in ring]
    n = 0
    m = len(pts)
    for i in range(m):
        (ax, ay), (bx, by) = pts[i], pts[(i + 1) % m]
        if ay == by:
            continue
        if ay < by:
            lo, hi = (ax, ay), (bx, by)
        else:
            lo, hi = (bx, by), (ax, ay)
        if lo[1] <= py < hi[1] and _orient(lo[0], lo[1], hi[0], hi[1], px, py) > 0:
            n += 1
    return n


def inside_exact(px, py, rings):
    return sum(ring_crossings_exact(px, py, r) for r in rings) % 2 == 1


def winding_number(px, py, ring):
    """Signed winding number of a closed ring around p (exact)."""
    px, py = Fr(px), Fr(py)
    pts = [(Fr(x), Fr(y)) for x, y in ring]
    w = 0
    m = len(pts)
    for i in range(m):
        (ax, ay), (bx, by) = pts[i], pts[(i + 1) % m]
        if ay <= py:
            if by > py and _orient(ax, ay, bx, by, px, py) > 0:
                w += 1
        else:
            if by <= py and _orient(ax, ay, bx, by, px, py) < 0:
                w -= 1
    return w


def distance_to_ring_boundary_lb(px, py, ring):
    """Exact squared distance from p to the nearest edge of the ring."""
    m = len(ring)
    return min(segment_d2_exact(px, py, *ring[i], *ring[(i + 1) % m]) for i in range(m))


def segment_d2_exact(px, py, ax, ay, bx, by):
    """Exact squared distance from p to segment [a, b] by clamped projection."""
    px, py, ax, ay, bx, by = map(Fr, (px, py, ax, ay, bx, by))
    dx, dy = bx - ax, by - ay
    L2 = dx * dx + dy * dy
    if L2 == 0:
        t = Fr(0)
    else:
        t = ((px - ax) * dx + (py - ay) * dy) / L2
        t = min(max(t, Fr(0)), Fr(1))
    qx, qy = ax + t * dx - px, ay + t * dy - py
    return qx * qx + qy * qy


def polyline_d2_exact(px, py, xs, ys):
    return min(segment_d2_exact(px, py, xs[i], ys[i], xs[i + 1], ys[i + 1])
               for i in range(len(xs) - 1))
