"""Boundary construction helpers (geom.facetBox and utils.aabbWalls roles)
against their geometric definitions: the triangles tile exactly the kept
faces of the box, and the six wall boxes sit outside the packing with their
inner faces on its bounding planes."""
import numpy as np
import pytest

from paper_2301_00611_amd.geom import aabb_walls, facet_box_triangles, packing_extrema

C = np.array([0.5, -1.0, 2.0])
H = np.array([0.25, 0.5, 1.5])


def _area(t):
    return 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))


@pytest.mark.parametrize("mask,faces", [(63, 6), (31, 5), (0b100001, 2), (0, 0)])
def test_facet_box_tiles_the_kept_faces(mask, faces):
    tris = facet_box_triangles(C, H, wall_mask=mask)
    assert len(tris) == 2 * faces
    kept = [(axis, side) for axis in range(3) for side in (-1, 1) if mask & (1 << (2 * axis + (side > 0)))]
    for f, (axis, side) in enumerate(kept):
        pair = tris[2 * f: 2 * f + 2]
        u, v = [a for a in range(3) if a != axis]
        for t in pair:
            # every vertex on the face plane, inside the face rectangle
            for p in t:
                assert p[axis] == C[axis] + side * H[axis]
                assert abs(p[u] - C[u]) <= H[u] and abs(p[v] - C[v]) <= H[v]
            # the normal is along the face's axis
            nrm = np.cross(t[1] - t[0], t[2] - t[0])
            assert np.allclose(nrm[[u, v]], 0.0) and abs(nrm[axis]) > 0
        # two triangles sharing a diagonal: their areas sum to the face's
        assert sum(_area(t) for t in pair) == pytest.approx(4 * H[u] * H[v], rel=1e-15)
        shared = {tuple(p) for p in pair[0]} & {tuple(p) for p in pair[1]}
        assert len(shared) == 2
        d = np.array(list(shared))
        assert np.allclose(np.abs(d[0] - d[1])[[u, v]], 2 * H[[u, v]])     # the diagonal


def test_open_top_has_no_z_plus_vertex_only_face():
    tris = facet_box_triangles(C, H, wall_mask=31)
    top = C[2] + H[2]
    assert not any(all(p[2] == top for p in t) for t in tris)


def test_aabb_walls_wrap_the_packing():
    rng = np.random.default_rng(3)
    pos = rng.uniform(-1.0, 1.0, (200, 3)) * [1.0, 2.0, 0.5]
    rad = rng.uniform(0.01, 0.05, 200)
    lo, hi = packing_extrema(pos, rad)
    assert np.allclose(lo, (pos - rad[:, None]).min(axis=0)) and np.allclose(hi, (pos + rad[:, None]).max(axis=0))
    size, mid = hi - lo, 0.5 * (lo + hi)
    boxes = aabb_walls((lo, hi))
    assert len(boxes) == 6
    t = 0.1 * size[0]
    for k, (c, h) in enumerate(boxes):
        axis, upper = divmod(k, 2)
        others = [a for a in range(3) if a != axis]
        assert h[axis] == pytest.approx(0.5 * t)
        assert np.allclose(h[others], 0.75 * size[others])        # oversize 1.5 in its plane
        assert np.allclose(c[others], mid[others])
        inner = c[axis] - h[axis] if upper else c[axis] + h[axis]
        assert inner == pytest.approx(hi[axis] if upper else lo[axis], rel=1e-14, abs=1e-15)
        # no sphere centre lies inside a box
        inside = np.all(np.abs(pos - c) < h, axis=1)
        assert not inside.any()
    thick = aabb_walls((lo, hi), thickness=0.02, oversize_factor=1.0)
    for k, (c, h) in enumerate(thick):
        axis = k // 2
        assert h[axis] == pytest.approx(0.01)
        assert np.allclose(np.delete(h, axis), 0.5 * np.delete(size, axis))


def test_helper_errors():
    with pytest.raises(ValueError):
        facet_box_triangles(C, [1.0, 0.0, 1.0])
    with pytest.raises(ValueError):
        facet_box_triangles(C, H, wall_mask=64)
    with pytest.raises(ValueError):
        aabb_walls(([0, 0, 0], [1, 0, 1]))
    with pytest.raises(ValueError):
        aabb_walls(([0, 0, 0], [1, 1, 1]), thickness=-1.0)
