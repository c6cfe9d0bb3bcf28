"""Full-size parity at the benchmark sizes.

* The two dense periodic workloads, 2,000,000 lognormal spheres (isotropic
  compression) and 8,000,000 bidisperse spheres (simple shear): a dense
  state built without the GPU (the generators' lattices squeezed so that
  neighbours overlap, random velocities and spins), a synthetic shear
  history on every contact of the sampled bodies (pairs found with a
  periodic k-d tree, independent of both implementations), one step on the
  GPU in FP64 and FP32-mixed against the oracle's spot mode on the sampled
  bodies (each evaluated against all N bodies and their 27 images).  Per
  body the resultant's error is taken against the sum of the magnitudes of
  its contact forces (bars 1e-12 FP64, 1e-5 FP32-mixed); positions,
  velocities and spins after the step too.
* The 512-scene batch: all scenes stepped together, 8 sampled scenes
  against the oracle's own trajectory of each.
"""
import math

import numpy as np
import pytest

from gpu_helpers import EPS, keyset

pytestmark = pytest.mark.gpu


def _periodic_history(pos, radius, box, ids, rng):
    """Synthetic history on every contact of the sampled spheres (0-based
    sphere indices): pairs found by a periodic k-d tree and the exact test
    |d| < r1 + r2 on the nearest image; random shear force normal to the
    pair, previous normal slightly tilted.  Returns (lo, hi, cell, fs,
    nprev) with d = x_hi + box c - x_lo."""
    from scipy.spatial import cKDTree
    tree = cKDTree(pos, boxsize=box)
    seen = set()
    recs = []
    for i, js in zip(ids, tree.query_ball_point(pos[ids], radius[ids] + radius.max())):
        for j in js:
            if j == i:
                continue
            lo, hi = (i, j) if i < j else (j, i)
            d = pos[hi] - pos[lo]
            c = -np.round(d / box).astype(np.int64)
            d = d + box * c
            dist = np.linalg.norm(d)
            if dist >= radius[lo] + radius[hi] or (lo, hi) in seen:
                continue
            seen.add((lo, hi))
            n = d / dist
            t = rng.normal(size=3)
            t -= t.dot(n) * n
            fs = t / np.linalg.norm(t) * rng.uniform(0.0, 1e-4)
            nprev = n + rng.normal(scale=1e-4, size=3)
            nprev /= np.linalg.norm(nprev)
            recs.append((lo, hi, c, fs, nprev))
    lo = np.array([r[0] for r in recs], dtype=np.int64)
    hi = np.array([r[1] for r in recs], dtype=np.int64)
    cell = np.array([r[2] for r in recs], dtype=np.int32).reshape(-1, 3)
    fs = np.array([r[3] for r in recs]).reshape(-1, 3)
    nprev = np.array([r[4] for r in recs]).reshape(-1, 3)
    return lo, hi, cell, fs, nprev


def _periodic_full_size(spec, pos, H, ids, vel_scale, seed):
    """GPU scenes (FP64, FP32-mixed) and the oracle's spot step on `ids`
    from the same dense state (positions pos in the cube H) and history;
    returns the per-precision GPU states and stats after one step, the spot
    result and the step."""
    from oracle import OracleScene
    from paper_2301_00611_amd import dem
    from paper_2301_00611_amd.scenes import random_velocities
    box = float(H[0, 0])
    assert np.allclose(H, np.eye(3) * box) and pos.min() >= 0.0 and pos.max() < box
    n = len(spec.radius)
    v, w = random_velocities(n, vel_scale, seed)
    w = w * 0.1
    rng = np.random.default_rng(seed + 1)
    lo, hi, cell, fs, nprev = _periodic_history(pos, spec.radius, box, ids, rng)
    assert len(lo) > len(ids)
    m = spec.material
    out = {}
    dt = None
    for prec in (0, 1):
        g = dem.Scene(periodic=True, hsize=H, velgrad=spec.velgrad, damping=spec.damping, gravity=spec.gravity,
                      precision=prec)
        mg = g.add_material(m.density, m.young, m.poisson, m.friction)
        g.add_spheres(pos, spec.radius, vel=v, angvel=w, default_mat=mg)
        dt = spec.dt_factor * g.pwave_dt()
        g.set_dt(dt)
        g.set_history(lo, hi, fs, nprev, cell=cell)
        g.step(1)
        out[prec] = (g.get_state(), g.stats())
        g.close()
    o = OracleScene(dt=dt, periodic=True, hsize=H, velgrad=spec.velgrad, damping=spec.damping, gravity=spec.gravity)
    mo = o.add_material(m.density, m.young, m.poisson, m.friction)
    o.add_spheres(pos, spec.radius, vel=v, angvel=w, default_mat=mo)
    assert spec.dt_factor * o.pwave_dt() == dt
    o.set_contacts(lo, hi, fs, nprev, cell=cell)
    spot = o.spot_step(ids)
    o.close()
    return out, spot, dt


def _check_spot(out, spot, ids, spec, dt, kn_max):
    """Per-body resultant against the sum of its contact forces'
    magnitudes; the state after the step within what that force error
    moves it by in one step (dt/m, r dt/I), plus rounding."""
    touched = spot["n_contacts"] > 0
    assert touched.sum() >= len(ids) // 2
    r = spec.radius[ids]
    mass = 4.0 / 3.0 * math.pi * r ** 3 * spec.material.density
    inertia = 0.4 * mass * r * r
    scale = spot["fmag_sum"] + spot["n_contacts"] * kn_max * 4 * EPS * 2 * spec.radius.max()
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        st, _ = out[prec]
        f = st["force"][ids]
        err = np.linalg.norm(f - spot["force"], axis=1)
        assert np.all(f[~touched] == 0.0), prec
        assert (err[touched] / scale[touched]).max() <= tol, (prec, (err[touched] / scale[touched]).max())
        dv = 2 * tol * scale * dt / mass + 8 * EPS * np.linalg.norm(spot["vel"], axis=1)
        dw = 2 * tol * scale * r * dt / inertia + 8 * EPS * np.linalg.norm(spot["angvel"], axis=1)
        dx = dv * dt + 4 * EPS * np.linalg.norm(spot["pos"], axis=1)
        assert np.all(np.linalg.norm(st["vel"][ids] - spot["vel"], axis=1) <= dv), prec
        assert np.all(np.linalg.norm(st["angvel"][ids] - spot["angvel"], axis=1) <= dw), prec
        assert np.all(np.linalg.norm(st["pos"][ids] - spot["pos"], axis=1) <= dx), prec


def test_bidisperse_shear_8m_spot():
    """8,000,000 spheres of radii 0.5 and 2.0 mm (the shear workload's
    generator, lattice squeezed by 0.2 %), simple shear at 1/s: 16 random
    spheres and 8 large ones against the oracle's spot mode."""
    from paper_2301_00611_amd.scenes import periodic_bidisperse_gas
    spec = periodic_bidisperse_gas(n=8_000_000, seed=0)
    n = len(spec.radius)
    rng = np.random.default_rng(31)
    large = np.nonzero(spec.radius > 1e-3)[0]
    ids = np.concatenate([rng.choice(n, size=16, replace=False), rng.choice(large, size=8, replace=False)])
    out, spot, dt = _periodic_full_size(spec, spec.pos * 0.998, spec.hsize * 0.998, ids, 0.01, 32)
    st, stats = out[0]
    assert stats["n_contacts_ss"] > 10_000_000
    _check_spot(out, spot, ids, spec, dt, spec.material.young * 2.0e-3)


def test_bidisperse_shear_8m_spot_after_1000_steps():
    """The benchmark's 8,000,000-sphere packing (prepared as the benchmark
    prepares it: jammed at 1 kPa, settled, tiled 4 x 4 x 4) sheared for 1,000
    steps on the GPU (FP64): from the GPU's own state, sheared cell and
    shear history at that step, one more step of fresh GPU scenes (FP64,
    FP32-mixed) against the oracle's spot mode on 24 sampled spheres (16
    random, 8 large), each evaluated against all bodies and their 27
    images; the history handed over is every contact of a sampled sphere."""
    import bench
    from oracle import OracleScene
    from paper_2301_00611_amd import dem
    spec, st0, H0, _ = bench.prepare_periodic("periodic_shear", 8_000_000)
    n = len(spec.radius)
    m = spec.material

    def scene(prec, pos, vel, angvel, H):
        g = dem.Scene(periodic=True, hsize=H, velgrad=spec.velgrad, damping=spec.damping, gravity=spec.gravity,
                      precision=prec)
        mg = g.add_material(m.density, m.young, m.poisson, m.friction)
        g.add_spheres(pos, spec.radius, vel=vel, angvel=angvel, default_mat=mg)
        g.set_dt(spec.dt_factor * g.pwave_dt())
        return g

    g = scene(0, st0["pos"], st0["vel"], st0["angvel"], H0)
    g.step(1000)
    st = g.get_state()
    H, _ = g.get_cell()
    hist = g.get_history()
    stats = g.stats()
    g.close()
    assert stats["n_contacts_ss"] > 10_000_000 and abs(H[0, 2]) > 0.0  # dense, and the cell has sheared
    rng = np.random.default_rng(33)
    large = np.nonzero(spec.radius > 1e-3)[0]
    ids = np.concatenate([rng.choice(n, size=16, replace=False), rng.choice(large, size=8, replace=False)])
    keep = np.isin(hist["id1"], ids) | np.isin(hist["id2"], ids)
    h = hist[keep]
    assert len(h) > len(ids) and np.abs(h["fs"]).max() > 0.0
    out = {}
    dt = None
    for prec in (0, 1):
        g = scene(prec, st["pos"], st["vel"], st["angvel"], H)
        dt = spec.dt_factor * g.pwave_dt()
        g.set_history(h["id1"], h["id2"], h["fs"], h["nprev"], cell=h["cell"])
        g.step(1)
        out[prec] = (g.get_state(), g.stats())
        g.close()
    o = OracleScene(dt=dt, periodic=True, hsize=H, velgrad=spec.velgrad, damping=spec.damping, gravity=spec.gravity)
    mo = o.add_material(m.density, m.young, m.poisson, m.friction)
    o.add_spheres(st["pos"], spec.radius, vel=st["vel"], angvel=st["angvel"], default_mat=mo)
    o.set_contacts(h["id1"], h["id2"], h["fs"], h["nprev"], cell=h["cell"])
    spot = o.spot_step(ids)
    o.close()
    _check_spot(out, spot, ids, spec, dt, spec.material.young * 2.0e-3)


def test_lognormal_compression_2m_spot():
    """2,000,000 spheres with the compression workload's lognormal radii
    (0.41 to 2.46 mm) on its generator's cubic lattice, with the spacing
    brought down to 3.0 mm and a jitter of +-0.05 mm per axis: pairs with
    r1 + r2 above ~3 mm overlap, and no overlap can exceed the smaller
    radius.  velGrad = -0.01 I; 24 random spheres and 24 of the largest
    against the oracle's spot mode."""
    from paper_2301_00611_amd.scenes import periodic_lognormal_gas
    spec = periodic_lognormal_gas(n=2_000_000, seed=0)
    n = len(spec.radius)
    k = math.ceil(n ** (1 / 3) - 1e-9)
    a = 3.0e-3
    idx = np.arange(n)
    nodes = np.stack([idx % k, (idx // k) % k, idx // (k * k)], axis=1).astype(np.float64) + 0.5
    pos = nodes * a + np.random.default_rng(40).uniform(-5e-5, 5e-5, size=(n, 3))
    H = np.eye(3) * (k * a)
    rng = np.random.default_rng(41)
    big = np.argsort(spec.radius)[-20_000:]
    ids = np.concatenate([rng.choice(n, size=24, replace=False), rng.choice(big, size=24, replace=False)])
    out, spot, dt = _periodic_full_size(spec, pos, H, ids, 0.01, 42)
    st, stats = out[0]
    assert stats["n_contacts_ss"] > 100_000
    _check_spot(out, spot, ids, spec, dt, spec.material.young * 2 * spec.radius.max())


def test_batched_512_scenes_sampled_against_oracle():
    """The 512-scene deposition batch (6.2 M spheres in all), thrown with
    random velocities so that collisions start early, stepped 600 steps as
    one batch; 8 sampled scenes of up to 2,500 spheres against the oracle's
    own 600 steps of each: identical pair sets, positions within 1e-12 m,
    contact forces within 1e-6 (rounding grown over 600 steps)."""
    from oracle import OracleScene
    from paper_2301_00611_amd import dem
    from paper_2301_00611_amd.scenes import batched_deposition, random_velocities
    spec = batched_deposition(n_scenes=512, seed=0)
    dt = 0.5 * spec.dt_radius * math.sqrt(2600.0 / 5e7)
    params = [dem.make_params(dt=dt, gravity=s.gravity, damping=s.damping) for s in spec.scenes]
    batch = dem.Batch(params)
    vels = []
    for i, s in enumerate(spec.scenes):
        view = batch.scene(i)
        m = view.add_material(s.material.density, s.material.young, s.material.poisson, s.material.friction)
        for w in s.walls:
            view.add_wall(w.axis, w.position, w.sense, m)
        v, _ = random_velocities(s.n, 0.3, 5000 + i)
        vels.append(v)
        view.add_spheres(s.pos, s.radius, vel=v, default_mat=m)
    assert sum(s.n for s in spec.scenes) > 5_000_000
    batch.step(600)
    small = [i for i, s in enumerate(spec.scenes) if s.n <= 2500]
    rng = np.random.default_rng(7)
    picked = rng.choice(small, size=8, replace=False)
    compared = 0
    for i in picked:
        s = spec.scenes[i]
        o = OracleScene(dt=dt, gravity=s.gravity, damping=s.damping)
        mo = o.add_material(s.material.density, s.material.young, s.material.poisson, s.material.friction)
        for w in s.walls:
            o.add_wall(w.axis, w.position, w.sense, mo)
        o.add_spheres(s.pos, s.radius, vel=vels[i], default_mat=mo)
        o.step(600)
        view = batch.scene(i)
        cg, co = view.get_contacts(), o.get_contacts()
        assert keyset(cg) == keyset(co), i
        a, b = view.get_state(), o.get_state()
        assert np.abs(a["pos"] - b["pos"]).max() <= 1e-12, i
        if len(co):
            og, oo = np.lexsort((cg["id2"], cg["id1"])), np.lexsort((co["id2"], co["id1"]))
            fg, fo = cg["fn"][og] + cg["fs"][og], co["fn"][oo] + co["fs"][oo]
            err = np.linalg.norm(fg - fo, axis=1) / (np.linalg.norm(fo, axis=1) + co["kn"][oo] * 4 * EPS * 2.4e-3)
            assert err.max() <= 1e-6, i
            compared += len(co)
        o.close()
    assert compared > 0
