"""Shared set-up for the GPU tests: the same seeded inputs handed to the HIP
library (through the C ABI binding) and to the FP64 oracle, plus the
comparison metrics.  Nothing here computes the method itself."""
import numpy as np

EPS = np.finfo(float).eps


def twin(spec, precision=0, track_energy=True, periodic=False, hsize=None, velgrad=None, dt=None,
         vel=None, angvel=None, verlet_dist=-0.5, viscel=None):
    """Build (gpu, oracle, dt) from a scenes.Scene-like spec.  viscel =
    (tc, en, et): a ViscElMat of the spec's density and friction angle in
    place of its FrictMat (dt must then be given)."""
    from oracle import OracleScene
    from paper_2301_00611_amd import dem

    m = spec.material
    g = dem.Scene(gravity=spec.gravity, damping=spec.damping, track_energy=track_energy, precision=precision,
                  periodic=periodic, hsize=hsize, velgrad=velgrad, verlet_dist=verlet_dist)
    if viscel is None:
        mg = g.add_material(m.density, m.young, m.poisson, m.friction)
    else:
        mg = g.add_viscel_material(m.density, *viscel, m.friction)
    for w in spec.walls:
        g.add_wall(w.axis, w.position, w.sense, mg)
    for c, h in getattr(spec, "boxes", []):
        g.add_box(c, h, mg)
    for tri in getattr(spec, "facets", []):
        g.add_facet(*tri, mat=mg)
    g.add_spheres(spec.pos, spec.radius, vel=vel, angvel=angvel, default_mat=mg)
    if dt is None:
        dt = spec.dt_factor * g.pwave_dt()
    g.set_dt(dt)
    o = OracleScene(dt=dt, gravity=spec.gravity, damping=spec.damping, periodic=periodic, hsize=hsize,
                    velgrad=velgrad)
    if viscel is None:
        mo = o.add_material(m.density, m.young, m.poisson, m.friction)
    else:
        mo = o.add_viscel_material(m.density, *viscel, m.friction)
    for w in spec.walls:
        o.add_wall(w.axis, w.position, w.sense, mo)
    for c, h in getattr(spec, "boxes", []):
        o.add_box(c, h, mo)
    for tri in getattr(spec, "facets", []):
        o.add_facet(*tri, mat=mo)
    o.add_spheres(spec.pos, spec.radius, vel=vel, angvel=angvel, default_mat=mo)
    assert spec.dt_factor * o.pwave_dt() == spec.dt_factor * g.pwave_dt()
    return g, o, dt


def keyset(c):
    return set(zip(c["id1"].tolist(), c["id2"].tolist(), map(tuple, c["cell"].tolist())))


def contact_errors(cg, co):
    """Per-contact relative force error, contacts matched by key; the
    denominator adds kn * 4 eps (r1 + r2) for the cancellation in the
    overlap r1 + r2 - l."""
    order_g = np.lexsort((cg["id2"], cg["id1"]))
    order_o = np.lexsort((co["id2"], co["id1"]))
    cg, co = cg[order_g], co[order_o]
    assert np.array_equal(cg["id1"], co["id1"]) and np.array_equal(cg["id2"], co["id2"])
    scale = co["kn"] * 4 * EPS * 2.5e-3
    out = {}
    for key in ("fn", "fs"):
        num = np.linalg.norm(cg[key] - co[key], axis=1)
        out[key] = num / (np.linalg.norm(co[key], axis=1) + scale)
    total_g, total_o = cg["fn"] + cg["fs"], co["fn"] + co["fs"]
    out["f"] = np.linalg.norm(total_g - total_o, axis=1) / (np.linalg.norm(total_o, axis=1) + scale)
    out["normal"] = np.linalg.norm(cg["normal"] - co["normal"], axis=1)
    out["pen"] = np.abs(cg["pen"] - co["pen"]) / (np.abs(co["pen"]) + 4 * EPS * 2.5e-3)
    # contact point, relative to its distance from the origin plus the radius scale
    out["point"] = np.linalg.norm(cg["point"] - co["point"], axis=1) / (np.linalg.norm(co["point"], axis=1) + 1e-3)
    return out


def body_force_errors(sg, so, co):
    """Per-body error of the resultant, relative to the sum of the magnitudes
    of the contact forces acting on that body (the natural scale of a
    near-cancelling sum)."""
    n = sg["force"].shape[0]
    scale = np.zeros(n)
    mag = np.linalg.norm(co["fn"] + co["fs"], axis=1)
    np.add.at(scale, co["id1"], mag)
    np.add.at(scale, co["id2"], mag)
    touched = scale > 0
    ef = np.linalg.norm(sg["force"] - so["force"], axis=1)[touched] / scale[touched]
    return ef, touched


def random_history(pos, radius, walls, rng, fraction=0.8):
    """Synthetic shear history for the currently overlapping pairs: found
    here with a k-d tree (independent of both implementations), with random
    shear forces and slightly tilted previous normals; plus a few records
    for pairs that do not touch (they must be dropped)."""
    from scipy.spatial import cKDTree

    nw = len(walls)
    tree = cKDTree(pos)
    pairs = np.array(sorted(tree.query_pairs(2 * radius.max())), dtype=np.int64).reshape(-1, 2)
    recs = []
    for i, j in pairs:
        d = pos[j] - pos[i]
        dist = np.linalg.norm(d)
        if dist >= radius[i] + radius[j] or rng.random() > fraction:
            continue
        n = d / dist
        t = rng.normal(size=3)
        t -= t.dot(n) * n
        fs = t * rng.uniform(0.0, 2e-3)
        nprev = n + rng.normal(scale=1e-4, size=3)
        nprev /= np.linalg.norm(nprev)
        recs.append((i + nw, j + nw, fs, nprev))
    for k, w in enumerate(walls):
        delta = pos[:, w.axis] - w.position
        touching = np.nonzero(np.abs(delta) < radius)[0]
        for i in touching:
            if rng.random() > fraction:
                continue
            t = rng.normal(size=3)
            t[w.axis] = 0.0
            n = np.zeros(3)
            n[w.axis] = 1.0
            recs.append((k, i + nw, t * 1e-3, n))
    for _ in range(5):  # stale records: not touching, must disappear
        i, j = rng.integers(0, len(pos), size=2)
        if i != j and np.linalg.norm(pos[i] - pos[j]) > radius[i] + radius[j] + 1e-3:
            recs.append((min(i, j) + nw, max(i, j) + nw, np.array([1e-3, 0, 0]), np.array([0, 1.0, 0])))
    if not recs:
        return None
    id1 = np.array([r[0] for r in recs])
    id2 = np.array([r[1] for r in recs])
    fs = np.array([r[2] for r in recs])
    nprev = np.array([r[3] for r in recs])
    return id1, id2, fs, nprev
