"""Parity of the GPU's box and facet boundaries (C ABI) with the oracle's
(Ig2_Box_Sphere_ScGeom, Ig2_Facet_Sphere_ScGeom readings), and their closed
forms through the GPU path.

Bars as for the rest of the step: pair sets identical, forces within 1e-12
(FP64) from an identical state; a 1,000-step deposition into a facet box
with a box obstacle keeps identical pair sets at every check and its energy
terms within 1 %.
"""
import math

import numpy as np
import pytest

from gpu_helpers import contact_errors, keyset

pytestmark = pytest.mark.gpu

R = 2.0 ** -10
E, NU, RHO = 1e7, 0.3, 1000.0


def _both(build, gravity=(0.0, 0.0, 0.0), damping=0.0, dt_factor=0.2, precision=0):
    """The same boundaries and spheres in the GPU library and the oracle."""
    from oracle import OracleScene
    from paper_2301_00611_amd import dem
    g = dem.Scene(gravity=gravity, damping=damping, precision=precision, track_energy=True)
    mg = g.add_material(RHO, E, NU, 0.5)
    o = OracleScene(dt=1.0, gravity=gravity, damping=damping)
    mo = o.add_material(RHO, E, NU, 0.5)
    build(g, mg, o, mo)
    dt = dt_factor * g.pwave_dt()
    g.set_dt(dt)
    o.set_dt(dt)
    return g, o


def _container(g, mg, o, mo, side):
    """A facet box open at the top (geom.facetBox, wallMask without z+) and a
    box obstacle on its floor."""
    from paper_2301_00611_amd.dem import facet_box_triangles
    c = np.array([0.5 * side, 0.5 * side, 0.5 * side])
    for tri in facet_box_triangles(c, [0.5 * side] * 3, wall_mask=31):
        g.add_facet(*tri, mat=mg)
        o.add_facet(*tri, mat=mo)
    bc, bh = [0.5 * side, 0.5 * side, 0.1 * side], [0.15 * side, 0.1 * side, 0.1 * side]
    g.add_box(bc, bh, mg)
    o.add_box(bc, bh, mo)


def _cloud(side, seed):
    """Lattice nodes of spacing 2r filling the container (the outer ones r
    from its faces), jittered by up to 0.2 r, radii U(0.85, 1.05) r: many
    sphere-sphere and sphere-facet overlaps, none beyond the smaller radius;
    nodes whose centre would be within 0.2 r of the box obstacle are left
    out (a centre inside a box is an overlap beyond the radius)."""
    rng = np.random.default_rng(seed)
    k = int(round(side / (2 * R)))
    g = (np.arange(k) + 0.5) * (side / k)
    nodes = np.array([[x, y, z] for z in g for y in g for x in g])
    pos = nodes + rng.uniform(-0.2, 0.2, nodes.shape) * R
    bc, bh = np.array([0.5 * side, 0.5 * side, 0.1 * side]), np.array([0.15 * side, 0.1 * side, 0.1 * side])
    far = np.any(np.abs(pos - bc) > bh + 0.2 * R, axis=1)
    pos = pos[far]
    rad = rng.uniform(0.85 * R, 1.05 * R, len(pos))
    return pos, rad


@pytest.mark.parametrize("seed", [0, 1])
def test_one_step_against_boundaries(seed):
    """Spheres scattered through a facet box with a box obstacle, many of
    them crossing or touching facets, edges, corners and the box: one step
    from random velocities."""
    side = 24 * R
    pos, rad = _cloud(side, seed)
    n = len(pos)
    vel = np.random.default_rng(seed + 5).normal(0.0, 0.05, (n, 3))

    def build(g, mg, o, mo):
        _container(g, mg, o, mo, side)
        g.add_spheres(pos, rad, vel=vel, default_mat=mg)
        o.add_spheres(pos, rad, vel=vel, default_mat=mo)

    g, o = _both(build)
    g.step(1)
    o.step(1)
    cg, co = g.get_contacts(), o.get_contacts()
    assert keyset(cg) == keyset(co)
    nb = int((co["is_wall"] == 1).sum())
    assert nb > 40, "the cloud should touch the boundaries"
    err = contact_errors(cg, co)
    assert err["f"].max() <= 1e-12
    assert err["normal"].max() <= 1e-13
    sg, so = g.get_state(), o.get_state()
    scale = np.abs(so["pos"]).max()
    assert np.abs(sg["pos"] - so["pos"]).max() <= 1e-14 * scale
    # boundary reactions: minus the sum of the forces on the touching spheres
    assert np.allclose(sg["force"][:11], so["force"][:11], rtol=1e-10, atol=1e-12 * np.abs(so["force"]).max())


def test_deposition_in_a_facet_box():
    """500 spheres thrown into the open facet box onto the box obstacle,
    damping 0.3, 1,000 steps: identical pair sets every 100 steps while the
    runs coincide, energy terms within 1 % over the run."""
    side = 30 * R
    n = 500
    rng = np.random.default_rng(7)
    k = 8
    grid = (np.arange(k) + 0.5) * (side / k)
    nodes = np.array([[x, y, z] for z in grid for y in grid for x in grid])[:n]
    rad = rng.uniform(0.8 * R, 1.2 * R, n)
    pos = nodes + rng.uniform(-0.3, 0.3, (n, 3)) * R
    pos[:, 2] += 0.2 * side
    # 1,000 steps are about 3 ms of physical time: the spheres are thrown
    # down at 4 m/s (about 12 r in that time) with a lateral spread, so that
    # they reach the floor, the obstacle and the side facets
    vel = rng.normal(0.0, 1.0, (n, 3))
    vel[:, 2] -= 4.0

    def build(g, mg, o, mo):
        _container(g, mg, o, mo, side)
        g.add_spheres(pos, rad, vel=vel, default_mat=mg)
        o.add_spheres(pos, rad, vel=vel, default_mat=mo)

    g, o = _both(build, gravity=(0.0, 0.0, -9.81), damping=0.3, dt_factor=0.3)
    sg_, so_ = [], []
    touched = 0
    for step in range(10):
        g.step(100)
        o.step(100)
        cg, co = g.get_contacts(), o.get_contacts()
        assert keyset(cg) == keyset(co), f"pair sets differ after {100 * (step + 1)} steps"
        touched += int((co["is_wall"] == 1).sum())
        if len(co):
            assert contact_errors(cg, co)["f"].max() <= 1e-8
        eg, eo = g.get_energy(), o.get_energy()
        sg_.append([eg[x] for x in ("kinetic", "grav_work", "damp_dissip", "elastic", "plastic_dissip")])
        so_.append([eo[x] for x in ("kinetic", "grav_work", "damp_dissip", "elastic", "plastic_dissip")])
    assert touched > 0
    a, b = np.array(sg_), np.array(so_)
    # each term within 1 % of the largest (the initial kinetic energy)
    assert np.abs(a - b).max() <= 0.01 * np.abs(b).max()
    assert b[-1, 2] > 0.0 and b[-1, 4] > 0.0       # damping and sliding did act


@pytest.mark.parametrize("case", ["box_edge", "box_corner", "box_inside", "facet_vertex", "facet_face_below"])
def test_boundary_closed_forms_on_the_gpu(case):
    """A few of the oracle's closed-form cases through the GPU path: normal,
    overlap and k_n (E r for a box, 4/3 E r for a facet)."""
    half = np.array([4 * R, 3 * R, 2 * R])
    L = 8 * R
    tri = ([0.0, 0.0, 0.0], [L, 0.0, 0.0], [0.0, L, 0.0])
    if case == "box_edge":
        d = 0.6 * R
        a = d / math.sqrt(2.0)
        center, normal, pen, kn = [half[0] + a, 0.5 * R, half[2] + a], [1, 0, 1], R - d, E * R
    elif case == "box_corner":
        d = 0.8 * R
        a = d / math.sqrt(3.0)
        center, normal, pen, kn = [half[0] + a, half[1] + a, half[2] + a], [1, 1, 1], R - d, E * R
    elif case == "box_inside":
        center, normal, pen, kn = [0.0, 0.0, half[2] - 0.3 * R], [0, 0, 1], 1.3 * R, E * R
    elif case == "facet_vertex":
        a, b = 0.25 * R, 0.35 * R
        center, normal, pen = [-a, -a, b], [-a, -a, b], R - math.sqrt(2 * a * a + b * b)
        kn = (E * 4 * R) * (E * 2 * R) / (E * 6 * R)
    else:
        h = 0.4 * R
        center, normal, pen = [L / 4, L / 4, -h], [0, 0, -1], R - h
        kn = (E * 4 * R) * (E * 2 * R) / (E * 6 * R)

    def build(g, mg, o, mo):
        if case.startswith("box"):
            g.add_box([0, 0, 0], half, mg)
            o.add_box([0, 0, 0], half, mo)
        else:
            g.add_facet(*tri, mat=mg)
            o.add_facet(*tri, mat=mo)
        g.add_spheres(np.asarray([center], dtype=float), [R], default_mat=mg)
        o.add_spheres(np.asarray([center], dtype=float), [R], default_mat=mo)

    g, o = _both(build, dt_factor=0.1)
    g.step(1)
    c = g.get_contacts()
    assert len(c) == 1 and c["is_wall"][0] == 1 and c["id1"][0] == 0
    n = np.asarray(normal, dtype=float)
    n /= np.linalg.norm(n)
    assert np.allclose(c["normal"][0], n, rtol=0, atol=1e-13)
    assert c["pen"][0] == pytest.approx(pen, rel=1e-10)
    assert c["kn"][0] == pytest.approx(kn, rel=1e-14)


def test_boundary_call_errors():
    from paper_2301_00611_amd import dem
    g = dem.Scene(gravity=(0, 0, 0))
    m = g.add_material(RHO, E, NU, 0.5)
    with pytest.raises(dem.DemError):
        g.add_box([0, 0, 0], [1.0, 0.0, 1.0], m)
    with pytest.raises(dem.DemError):
        g.add_facet([0, 0, 0], [1, 1, 1], [2, 2, 2], m)
    with pytest.raises(dem.DemError):
        g.add_facet([0, 0, 0], [1, 0, 0], [0, 1, 0], 7)
    p = dem.Scene(periodic=True, hsize=np.eye(3) * 0.1)
    mp = p.add_material(RHO, E, NU, 0.5)
    with pytest.raises(dem.DemError):
        p.add_box([0, 0, 0], [1, 1, 1], mp)
    ids = [g.add_facet(*t, mat=m) for t in dem.facet_box_triangles([0, 0, 0], [1, 1, 1], wall_mask=63)]
    assert len(ids) == 12 and ids == list(range(12))
    st = g.get_state()
    assert np.allclose(st["pos"][0], [-1.0, 1.0 / 3.0, -1.0 / 3.0])


def test_aabb_walls_one_step():
    """A jittered lattice pressed into utils.aabbWalls boxes (their inner
    faces 0.3 r inside the packing's bounding box): one step from random
    velocities, pair sets identical, forces within 1e-12."""
    from paper_2301_00611_amd.geom import aabb_walls, packing_extrema
    rng = np.random.default_rng(11)
    k = 9
    grid = (np.arange(k) + 0.5) * 2.2 * R
    pos = np.array([[x, y, z] for z in grid for y in grid for x in grid])
    pos += rng.uniform(-0.05, 0.05, pos.shape) * R
    rad = rng.uniform(0.95 * R, 1.05 * R, len(pos))
    lo, hi = packing_extrema(pos, rad)
    walls = aabb_walls((lo + 0.3 * R, hi - 0.3 * R))
    vel = rng.normal(0.0, 0.05, pos.shape)

    def build(g, mg, o, mo):
        ids = g.add_aabb_walls((lo + 0.3 * R, hi - 0.3 * R), mg)
        assert ids == list(range(6))
        for c, h in walls:
            o.add_box(c, h, mo)
        g.add_spheres(pos, rad, vel=vel, default_mat=mg)
        o.add_spheres(pos, rad, vel=vel, default_mat=mo)

    g, o = _both(build)
    g.step(1)
    o.step(1)
    cg, co = g.get_contacts(), o.get_contacts()
    assert keyset(cg) == keyset(co)
    assert int((co["is_wall"] == 1).sum()) >= 6 * k * k - 12 * k      # most outer spheres touch a wall
    err = contact_errors(cg, co)
    assert err["f"].max() <= 1e-12
    sg, so = g.get_state(), o.get_state()
    assert np.abs(sg["pos"] - so["pos"]).max() <= 1e-14 * np.abs(so["pos"]).max()


def test_full_size_spot_check_facet_column():
    """The benchmark's 200,000-sphere column in an open facet box,
    compressed so that many pairs overlap and the lowest and outermost
    spheres cross the facets, with random velocities: one step on the GPU
    against the oracle's spot mode on sampled bodies (half of them next to
    a facet), each evaluated against all N and every facet."""
    from oracle import OracleScene
    from paper_2301_00611_amd.scenes import grid_column, random_velocities
    from gpu_helpers import twin
    spec = grid_column(n=200_000, spacing=2.6e-3, seed=0, boundary="facets")
    n, nb = spec.n, spec.n_boundaries
    assert nb == 10 and not spec.walls
    v, w = random_velocities(n, 0.02, 9)
    g, _, dt = twin(spec, vel=v, angvel=w * 0.05, track_energy=False)
    o = OracleScene(dt=dt, gravity=spec.gravity, damping=spec.damping)
    mo = o.add_material(2600.0, spec.material.young, 0.3, 0.5)
    for tri in spec.facets:
        o.add_facet(*tri, mat=mo)
    o.add_spheres(spec.pos, spec.radius, vel=v, angvel=w * 0.05, default_mat=mo)
    rng = np.random.default_rng(5)
    near = np.flatnonzero((spec.pos[:, 0] < spec.radius) | (spec.pos[:, 1] < spec.radius)
                          | (spec.pos[:, 2] < spec.radius))
    ids = nb + np.concatenate([rng.choice(near, size=100, replace=False),
                               rng.choice(n, size=100, replace=False)])
    spot = o.spot_step(ids)
    g.step(1)
    st = g.get_state()
    stats = g.stats()
    assert stats["n_contacts_ss"] > 50_000 and stats["n_contacts_sw"] > 1000
    assert (spot["n_contacts"] > 0).sum() > 100
    # per body: the resultant's error against the sum of its contact
    # forces' magnitudes (plus the overlap's rounding, kn 4 eps (r1 + r2) per contact)
    touched = spot["n_contacts"] > 0
    scale = spot["fmag_sum"] + spot["n_contacts"] * spec.material.young * 1.5e-3 * 4 * np.finfo(float).eps * 3e-3
    ferr = np.linalg.norm(st["force"][ids] - spot["force"], axis=1)
    assert np.all(st["force"][ids][~touched] == 0.0)
    assert (ferr[touched] / scale[touched]).max() <= 1e-12
    assert np.abs(st["pos"][ids] - spot["pos"]).max() <= 1e-15
    assert np.abs(st["vel"][ids] - spot["vel"]).max() <= 1e-12 * np.abs(spot["vel"]).max()


def _thrown_into_facet_box(n, seed, side):
    rng = np.random.default_rng(seed)
    k = int(math.ceil(n ** (1.0 / 3.0)))
    grid = (np.arange(k) + 0.5) * (side / k)
    nodes = np.array([[x, y, z] for z in grid for y in grid for x in grid])[:n]
    rad = rng.uniform(0.8, 1.0, n) * min(R, 0.45 * side / k)
    pos = nodes + rng.uniform(-0.05, 0.05, (n, 3)) * R
    pos[:, 2] += 0.2 * side
    vel = rng.normal(0.0, 1.0, (n, 3))
    vel[:, 2] -= 4.0
    return pos, rad, vel


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_boundaries_match_single_scenes_bitwise(precision):
    """Three scenes of different sizes, each thrown into its own facet box
    with a box obstacle, stepped as one batch equal the same scenes stepped
    alone, bit for bit, after 600 steps (the batched box/facet
    instantiation)."""
    from paper_2301_00611_amd import dem
    sides = [24 * R, 30 * R, 20 * R]
    sizes = [300, 500, 150]
    specs = [_thrown_into_facet_box(n, 20 + i, sd) for i, (n, sd) in enumerate(zip(sizes, sides))]
    probe = dem.Scene(gravity=(0, 0, -9.81))
    pm = probe.add_material(RHO, E, NU, 0.5)
    probe.add_spheres(np.zeros((1, 3)), [R], default_mat=pm)
    dt = 0.3 * probe.pwave_dt()
    params = [dem.make_params(dt=dt, gravity=(0.0, 0.0, -9.81), damping=0.3, precision=precision) for _ in specs]
    batch = dem.Batch(params)
    singles = []
    for i, ((pos, rad, vel), side) in enumerate(zip(specs, sides)):
        for g in (batch.scene(i), dem.Scene(gravity=(0.0, 0.0, -9.81), damping=0.3, precision=precision)):
            m = g.add_material(RHO, E, NU, 0.5)
            g.add_facet_box([0.5 * side] * 3, [0.5 * side] * 3, m, wall_mask=31)
            g.add_box([0.5 * side, 0.5 * side, 0.1 * side], [0.15 * side, 0.1 * side, 0.1 * side], m)
            g.add_spheres(pos, rad, vel=vel, default_mat=m)
        singles.append(g)
        g.set_dt(dt)
    batch.step(600)
    touched = 0
    for i, single in enumerate(singles):
        single.step(600)
        a, b = batch.scene(i).get_state(), single.get_state()
        for key in ("pos", "vel", "angvel"):
            assert np.array_equal(a[key], b[key]), (i, key)
        touched += int((single.get_contacts()["is_wall"] == 1).sum())
    assert touched > 0


def test_boundaries_fp32_mixed_one_step():
    """The one-step cloud of the FP64 test in FP32-mixed mode: identical
    pair sets (the predicate is FP64 in both modes), forces within 1e-5."""
    side = 24 * R
    pos, rad = _cloud(side, 0)
    vel = np.random.default_rng(5).normal(0.0, 0.05, (len(pos), 3))

    def build(g, mg, o, mo):
        _container(g, mg, o, mo, side)
        g.add_spheres(pos, rad, vel=vel, default_mat=mg)
        o.add_spheres(pos, rad, vel=vel, default_mat=mo)

    g, o = _both(build, precision=1)
    g.step(1)
    o.step(1)
    cg, co = g.get_contacts(), o.get_contacts()
    assert keyset(cg) == keyset(co)
    assert int((co["is_wall"] == 1).sum()) > 40
    assert contact_errors(cg, co)["f"].max() <= 1e-5


def _scatter_near(rng, sample, n, existing, r, tries=200):
    """n sphere centres from sample(), each at least 1.3 r from every centre
    already placed (sphere overlaps stay below 0.7 r)."""
    out = []
    for _ in range(n):
        for _ in range(tries):
            p = sample()
            if all(np.linalg.norm(p - q) >= 1.3 * r for q in existing + out):
                out.append(p)
                break
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_triangles_and_boxes_one_step(seed):
    """Arbitrarily oriented triangles and boxes of random shape, each on its
    own cell of a coarse grid, with spheres scattered over their face, edge,
    vertex and (for boxes) inside regions: one step, pair sets identical,
    normals within 1e-13, forces within 1e-12."""
    rng = np.random.default_rng(100 + seed)
    cell = 16 * R
    tris, boxes, centres = [], [], []
    for c in range(27):
        base = (np.array([c % 3, (c // 3) % 3, c // 9], dtype=float) + 0.5) * cell
        if c % 3 == 2:
            half = rng.uniform(1.0, 3.0, 3) * R
            boxes.append((base, half))

            def sample(base=base, half=half):
                u = rng.uniform(-1.0, 1.0, 3) * (half + 0.9 * R)
                return base + u
        else:
            q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            pts = rng.uniform(-3.0, 3.0, (3, 2)) * R
            v = [base + q[:, 0] * p[0] + q[:, 1] * p[1] for p in pts]
            if np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0])) < 2 * R * R:
                continue
            tris.append(tuple(v))
            nrm = q[:, 2]

            def sample(v=v, nrm=nrm):
                a, b = rng.uniform(-0.4, 1.2, 2)
                p = v[0] + a * (v[1] - v[0]) + b * (v[2] - v[0])
                return p + rng.uniform(-0.9, 0.9) * R * nrm
        centres += _scatter_near(rng, sample, 8, centres, R)
    pos = np.array(centres)
    rad = rng.uniform(0.95, 1.0, len(pos)) * R
    vel = rng.normal(0.0, 0.05, pos.shape)

    def build(g, mg, o, mo):
        for c, h in boxes:
            g.add_box(c, h, mg)
            o.add_box(c, h, mo)
        for t in tris:
            g.add_facet(*t, mat=mg)
            o.add_facet(*t, mat=mo)
        g.add_spheres(pos, rad, vel=vel, default_mat=mg)
        o.add_spheres(pos, rad, vel=vel, default_mat=mo)

    g, o = _both(build, gravity=(0.0, 0.0, -9.81), damping=0.1)
    g.step(1)
    o.step(1)
    cg, co = g.get_contacts(), o.get_contacts()
    assert keyset(cg) == keyset(co)
    assert int((co["is_wall"] == 1).sum()) > 60
    err = contact_errors(cg, co)
    assert err["f"].max() <= 1e-12
    # a boundary normal (x - p)/|x - p| from a closest point p computed in a
    # different order carries the rounding of x and p over |x - p|: its
    # error bound grows as the centre nears the triangle or the box
    cs = co[np.lexsort((co["id2"], co["id1"]))]
    nb = len(boxes) + len(tris)
    r2 = rad[cs["id2"] - nb]
    dist = np.where(cs["is_wall"] == 1, r2 - cs["pen"], np.inf)
    bound = 1e-13 + 16 * np.finfo(float).eps * np.abs(pos).max() / np.maximum(dist, 1e-300)
    assert np.all(err["normal"] <= bound)
    sg, so = g.get_state(), o.get_state()
    assert np.abs(sg["pos"] - so["pos"]).max() <= 1e-14 * np.abs(so["pos"]).max()
