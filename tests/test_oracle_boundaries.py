"""Pins of the oracle's box and facet boundaries (Ig2_Box_Sphere_ScGeom,
Ig2_Facet_Sphere_ScGeom) against closed forms.

Each case places one sphere at rest (no gravity) against one boundary, runs
one step and checks the contact the oracle reports: the normal (from the
boundary towards the sphere), the overlap and the normal force, written out
from the geometry here.  A box is a virtual sphere of the same radius
(normal stiffness k_n = E r for equal materials); a facet's reference radius
is twice the sphere's (k_n = (E 4r)(E 2r)/(E 6r) = 4/3 E r).  A slip in the
closest-point regions (face, edge, corner), in the inside case, in the sign
of the normal or in the reference radius fails one of them.
"""
import math

import numpy as np
import pytest

from oracle import OracleScene

R = 2.0 ** -10
E, NU, RHO = 1e7, 0.3, 1000.0


def _one_contact(add_boundary, center):
    s = OracleScene(dt=1.0)
    m = s.add_material(RHO, E, NU, 0.5)
    add_boundary(s, m)
    s.add_spheres(np.asarray([center], dtype=float), [R], default_mat=m)
    s.set_dt(0.1 * s.pwave_dt())
    s.step(1)
    c = s.get_contacts()
    return s, c


def _check(c, normal, pen, kn):
    assert len(c) == 1
    n = np.asarray(normal, dtype=float)
    n = n / np.linalg.norm(n)
    assert np.allclose(c["normal"][0], n, rtol=0, atol=1e-14)
    assert c["pen"][0] == pytest.approx(pen, rel=1e-11)
    assert c["kn"][0] == pytest.approx(kn, rel=1e-14)
    assert np.allclose(c["fn"][0], kn * pen * n, rtol=1e-11, atol=1e-12 * kn * pen)
    assert c["is_wall"][0] == 1 and c["id1"][0] == 0


BOX_C, BOX_H = np.array([0.0, 0.0, 0.0]), np.array([4 * R, 3 * R, 2 * R])


def _box(s, m):
    s.add_box(BOX_C, BOX_H, m)


def test_box_face(shift):
    """Above the top face, inside its footprint: normal +z, overlap r - gap,
    k_n = E r (virtual sphere of the same radius)."""
    gap = 0.7 * R
    s, c = _one_contact(_box_at(shift), shift + [R, -R, BOX_H[2] + gap])
    _check(c, [0, 0, 1], R - gap, E * R)


def test_box_edge(shift):
    """Beyond the +x / +z edge at 45 degrees: the closest point is on the
    edge, normal (1, 0, 1)/sqrt2."""
    d = 0.6 * R
    a = d / math.sqrt(2.0)
    s, c = _one_contact(_box_at(shift), shift + [BOX_H[0] + a, 0.5 * R, BOX_H[2] + a])
    _check(c, [1, 0, 1], R - d, E * R)


def test_box_corner(shift):
    """Beyond the (+,+,+) corner along the diagonal: normal (1, 1, 1)/sqrt3."""
    d = 0.8 * R
    a = d / math.sqrt(3.0)
    s, c = _one_contact(_box_at(shift), shift + [BOX_H[0] + a, BOX_H[1] + a, BOX_H[2] + a])
    _check(c, [1, 1, 1], R - d, E * R)


@pytest.mark.parametrize("axis,side", [(k, sd) for k in range(3) for sd in (-1, 1)])
def test_box_centre_inside(axis, side, shift):
    """Centre inside the box, 0.3 r from one face (each of the six in turn)
    and deeper from every other one: pushed out through that face, along
    its outward normal, overlap r + 0.3 r."""
    centre = np.zeros(3)
    centre[axis] = side * (BOX_H[axis] - 0.3 * R)
    normal = np.zeros(3)
    normal[axis] = side
    s, c = _one_contact(_box_at(shift), shift + centre)
    _check(c, normal, 1.3 * R, E * R)


def test_box_no_contact_beyond_edge(shift):
    """Within r of both face planes but farther than r from the edge: no
    contact (a box is not two walls)."""
    a = 0.9 * R
    s, c = _one_contact(_box_at(shift), shift + [BOX_H[0] + a, 0.0, BOX_H[2] + a])
    assert len(c) == 0


L = 8 * R
TRI = (np.array([0.0, 0.0, 0.0]), np.array([L, 0.0, 0.0]), np.array([0.0, L, 0.0]))


def _facet(s, m):
    s.add_facet(TRI[0], TRI[1], TRI[2], m)


@pytest.fixture(params=[(0.0, 0.0, 0.0), (24 * R, -16 * R, 12 * R)], ids=["at-origin", "translated"])
def shift(request):
    """Every facet and box configuration also translated as a whole (an
    exact binary offset): the same normals and overlaps, so that nothing
    may depend on a vertex or a corner sitting at the origin."""
    return np.array(request.param)


def _turn(axis, angle):
    u = np.asarray(axis, dtype=float) / np.linalg.norm(axis)
    k = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return np.eye(3) + math.sin(angle) * k + (1.0 - math.cos(angle)) * (k @ k)


PLACEMENTS = {"at-origin": (np.eye(3), np.zeros(3)),
              "translated": (np.eye(3), np.array([24 * R, -16 * R, 12 * R])),
              "turned": (_turn([1.0, -2.0, 0.5], 0.7), np.array([24 * R, -16 * R, 12 * R]))}


@pytest.fixture(params=list(PLACEMENTS))
def place(request):
    """A facet configuration as given, translated, and turned about a skew
    axis then translated: the same overlaps and the normals turned with
    it, so that nothing may depend on the triangle's position or on its
    lying in a coordinate plane."""
    return PLACEMENTS[request.param]


def _facet_at(place):
    Q, t = place
    def add(s, m):
        s.add_facet(Q @ TRI[0] + t, Q @ TRI[1] + t, Q @ TRI[2] + t, m)
    return add


def _placed(place, centre):
    Q, t = place
    return Q @ np.asarray(centre, dtype=float) + t


def _box_at(shift):
    def add(s, m):
        s.add_box(BOX_C + shift, BOX_H, m)
    return add


KN_FACET = (E * 4 * R) * (E * 2 * R) / (E * 6 * R)


def test_facet_face_both_sides(place):
    """Above and below the triangle's interior: normal +z or -z (two-sided),
    overlap r - |height|, k_n from the reference radius 2r."""
    h = 0.4 * R
    s, c = _one_contact(_facet_at(place), _placed(place, [L / 4, L / 4, h]))
    _check(c, place[0] @ np.array([0, 0, 1], dtype=float), R - h, KN_FACET)
    s, c = _one_contact(_facet_at(place), _placed(place, [L / 4, L / 4, -h]))
    _check(c, place[0] @ np.array([0, 0, -1], dtype=float), R - h, KN_FACET)


def test_facet_edge(place):
    """Outside the x = 0 edge, off the plane: the closest point is on the
    edge, normal (-a, 0, b)/|(a, b)|."""
    a, b = 0.3 * R, 0.5 * R
    s, c = _one_contact(_facet_at(place), _placed(place, [-a, L / 3, b]))
    _check(c, place[0] @ np.array([-a, 0, b], dtype=float), R - math.hypot(a, b), KN_FACET)


def test_facet_hypotenuse(place):
    """Outside the slanted edge (L,0,0)-(0,L,0), in the plane: normal along
    (1, 1, 0)/sqrt2."""
    d = 0.5 * R
    p = np.array([L / 2, L / 2, 0.0]) + d / math.sqrt(2.0) * np.array([1.0, 1.0, 0.0])
    s, c = _one_contact(_facet_at(place), _placed(place, p))
    _check(c, place[0] @ np.array([1, 1, 0], dtype=float), R - d, KN_FACET)


def test_facet_vertex(place):
    """Beyond vertex (0,0,0): normal (-a, -a, b)/|.|."""
    a, b = 0.25 * R, 0.35 * R
    s, c = _one_contact(_facet_at(place), _placed(place, [-a, -a, b]))
    _check(c, place[0] @ np.array([-a, -a, b], dtype=float), R - math.sqrt(2 * a * a + b * b), KN_FACET)


def test_facet_centre_on_the_triangle(place):
    """Centre exactly in the triangle: the face normal (v1 - v0) x (v2 - v0)
    = +z, overlap r."""
    s, c = _one_contact(_facet_at(place), _placed(place, [L / 4, L / 4, 0.0]))
    _check(c, place[0] @ np.array([0, 0, 1], dtype=float), R, KN_FACET)


def test_resting_on_a_box_under_gravity():
    """A damped sphere resting on a box top settles at overlap m g / k_n
    with k_n = E r (the static closed form of a wall)."""
    s = OracleScene(dt=1.0, gravity=(0, 0, -9.81), damping=0.3)
    m = s.add_material(RHO, E, NU, 0.5)
    s.add_box(BOX_C, BOX_H, m)
    s.add_spheres(np.asarray([[0.0, 0.0, BOX_H[2] + R]]), [R], default_mat=m)
    s.set_dt(0.2 * s.pwave_dt())
    s.step(20000)
    c = s.get_contacts()
    mass = 4.0 / 3.0 * math.pi * R ** 3 * RHO
    assert c["pen"][0] == pytest.approx(mass * 9.81 / (E * R), rel=1e-6)
