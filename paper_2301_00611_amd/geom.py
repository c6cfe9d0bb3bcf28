"""Boundary construction helpers: the roles of geom.facetBox and
utils.aabbWalls (utility reference, section 5).

Plain geometry on the host, returning vertex triples and (centre,
half-size) pairs that the caller hands to ``Scene.add_facet`` and
``Scene.add_box`` (or to any other consumer): no library call is made here.
"""
from __future__ import annotations

import numpy as np


def facet_box_triangles(center, half, wall_mask=63):
    """The triangles of geom.facetBox: each kept face of the box with the
    given centre and half-sizes split along a diagonal into two triangles.
    Face order x-, x+, y-, y+, z-, z+ (wall_mask bits 1, 2, 4, 8, 16, 32; the
    tutorials' wallMask=31 leaves the top open)."""
    c = np.asarray(center, dtype=np.float64)
    h = np.asarray(half, dtype=np.float64)
    if c.shape != (3,) or h.shape != (3,) or not np.all(h > 0):
        raise ValueError("facet_box_triangles: centre and positive half-sizes of length 3")
    if not 0 <= int(wall_mask) <= 63:
        raise ValueError("facet_box_triangles: wall_mask is a 6-bit mask")
    tris = []
    for axis in range(3):
        u, v = [a for a in range(3) if a != axis]
        for side, bit in ((-1.0, 1 << (2 * axis)), (1.0, 1 << (2 * axis + 1))):
            if not (wall_mask & bit):
                continue
            corners = []
            for su, sv in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
                p = c.copy()
                p[axis] += side * h[axis]
                p[u] += su * h[u]
                p[v] += sv * h[v]
                corners.append(p)
            tris.append((corners[0], corners[1], corners[2]))
            tris.append((corners[0], corners[2], corners[3]))
    return tris


def aabb_walls(extrema, thickness=None, oversize_factor=1.5):
    """Six boxes wrapping a packing whose bounding box is ``extrema`` =
    (lo, hi), in the order min x, max x, min y, max y, min z, max z (the
    role of utils.aabbWalls).  Each box lies outside the packing with its
    inner face on the packing's bounding plane, is ``thickness`` thick
    (one tenth of the x extent by default) and spans ``oversize_factor``
    times the packing's extent in its own plane, about the packing's centre.
    Returns a list of (centre, half_sizes) pairs."""
    lo = np.asarray(extrema[0], dtype=np.float64)
    hi = np.asarray(extrema[1], dtype=np.float64)
    if lo.shape != (3,) or hi.shape != (3,) or not np.all(hi > lo):
        raise ValueError("aabb_walls: extrema (lo, hi) with hi > lo on every axis")
    size = hi - lo
    t = 0.1 * size[0] if thickness is None else float(thickness)
    if not t > 0 or not oversize_factor > 0:
        raise ValueError("aabb_walls: thickness and oversize_factor must be positive")
    mid = 0.5 * (lo + hi)
    out = []
    for axis in range(3):
        for j, plane in ((0, lo[axis]), (1, hi[axis])):
            c = mid.copy()
            hs = 0.5 * oversize_factor * size
            hs[axis] = 0.5 * t
            c[axis] = plane + (j - 0.5) * t
            out.append((c, hs))
    return out


def packing_extrema(pos, radius):
    """Bounding box of a sphere packing, (lo, hi) over centre -/+ radius."""
    p = np.asarray(pos, dtype=np.float64)
    r = np.asarray(radius, dtype=np.float64)[:, None]
    return (p - r).min(axis=0), (p + r).max(axis=0)
