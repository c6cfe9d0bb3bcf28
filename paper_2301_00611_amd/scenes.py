"""Seeded synthetic scene generators.

This module only draws numbers: radii, positions, velocities and per-scene
parameters, from numpy's PCG64 (``default_rng(seed)``).  It holds none of the
DEM method's arithmetic (no contact test, no force, no integration, no time
step), so both the GPU path and the FP64 oracle can be fed from it without
sharing any method code.

The workloads follow the shapes of the documentation's tutorials:
gravity deposition into a box (section 3.1.x "Gravity deposition"), and the
benchmark configurations described in the design notes:

* ``cloud_box``  -- C1: 1,000 spheres, r ~ U(0.9, 1.1) mm, random sequential
  placement without overlap in a 30 mm cube closed by 6 walls.
* ``grid_column`` -- C2: 200,000 spheres, r ~ U(0.5, 1.5) mm on a
  33 x 33 column grid of spacing 3.03 mm with per-axis jitter
  U(-j, j), j = (s - 2r)/2, above a floor, inside 4 side walls.
* ``batched_deposition`` -- C4: 512 scenes, sphere count log-uniform in
  [500, 50000], r ~ U(0.8, 1.2) mm, friction ~ U(0.1, 0.7) rad,
  damping ~ U(0.05, 0.4), each a jittered column grid in its own box.
* ``periodic_lognormal_gas`` -- C3's starting cloud: 2,000,000 spheres with
  lognormal radii (median 1 mm, sigma_ln 0.3, truncated at +-3 sigma) on a
  jittered cubic lattice in a periodic cube (periodic simple-shear and
  triaxial tutorials, section 3.1.x), before its isotropic compression.
* ``periodic_bidisperse_gas`` -- C5's starting cloud: 0.5 mm and 2.0 mm
  spheres, equal total volume, large spheres and blocks of small ones at
  randomly permuted nodes of one cubic lattice.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Material:
    density: float
    young: float
    poisson: float
    friction: float


@dataclass
class Wall:
    axis: int
    position: float
    sense: int = 0


@dataclass
class Scene:
    """Plain data: what both implementations receive."""
    pos: np.ndarray                 # (n, 3) float64 [m]
    radius: np.ndarray              # (n,) float64 [m]
    material: Material
    walls: list = field(default_factory=list)
    boxes: list = field(default_factory=list)     # (centre, half-sizes) pairs, added after the walls
    facets: list = field(default_factory=list)    # (v0, v1, v2) triples, added after the boxes
    vel: np.ndarray | None = None   # (n, 3)
    angvel: np.ndarray | None = None
    gravity: tuple = (0.0, 0.0, -9.81)
    damping: float = 0.2
    dt_factor: float = 0.5          # dt = dt_factor * (P-wave step), computed by each side
    steps: int = 1000
    periodic: bool = False
    hsize: np.ndarray | None = None
    velgrad: np.ndarray | None = None
    name: str = ""

    @property
    def n_boundaries(self) -> int:
        """Walls, boxes and facets: the ids before the first sphere."""
        return len(self.walls) + len(self.boxes) + len(self.facets)

    @property
    def n(self) -> int:
        return int(self.radius.size)


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_sequential(n: int, lo: np.ndarray, hi: np.ndarray, rmin: float, rmax: float,
                      seed: int, max_tries: int = 200000) -> tuple[np.ndarray, np.ndarray]:
    """Radii ~ U(rmin, rmax) drawn first, then centres placed one by one
    uniformly in [lo + r, hi - r], rejecting any draw that overlaps an already
    placed sphere.  Placement test is plain geometry on the generator side
    (distance of centres against the sum of radii), done on a coarse hash
    grid so that it stays fast for a few thousand spheres."""
    rng = _rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    radius = rng.uniform(rmin, rmax, size=n)
    pos = np.zeros((n, 3))
    cell = 2.0 * rmax
    grid: dict = {}
    placed = 0
    tries = 0
    while placed < n:
        r = radius[placed]
        p = rng.uniform(lo + r, hi - r)
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_sequential: packing too dense")
        key = tuple(np.floor(p / cell).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((pos[j] - p) ** 2) <= (radius[j] + r) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        pos[placed] = p
        grid.setdefault(key, []).append(placed)
        placed += 1
    return pos, radius


def cloud_box(n: int = 1000, box: float = 0.030, rmin: float = 0.9e-3, rmax: float = 1.1e-3,
              seed: int = 0, steps: int = 1000) -> Scene:
    """C1: random non-overlapping spheres in a cube of 6 two-sided walls."""
    pos, radius = random_sequential(n, np.zeros(3), np.full(3, box), rmin, rmax, seed)
    walls = [Wall(a, p, 0) for a in range(3) for p in (0.0, box)]
    return Scene(pos=pos, radius=radius, material=Material(2600.0, 1e7, 0.3, 0.5), walls=walls,
                 gravity=(0.0, 0.0, -9.81), damping=0.2, dt_factor=0.5, steps=steps,
                 name=f"cloud_box_{n}")


def grid_column(n: int = 200_000, width: float = 0.1, spacing: float = 3.03e-3,
                rmin: float = 0.5e-3, rmax: float = 1.5e-3, seed: int = 0, young: float = 5e7,
                steps: int = 10_000, side_walls: bool = True, boundary: str = "walls") -> Scene:
    """C2: jittered column grid above a floor (z = 0) inside 4 side walls.

    boundary="facets" puts the same column in an open-topped facet box
    (geom.facetBox with wallMask=31, 10 triangles) over [0, width]^2 x
    [0, top + r_max] instead of the 5 planes.

    Node (i, j, k) sits at ((i + 1/2) s, (j + 1/2) s, (k + 1/2) s), filled
    layer by layer (x fastest), and each centre is jittered by U(-j, j) per
    axis with j = (s - 2r)/2, so no two spheres overlap and the lowest layer
    at most touches the floor."""
    rng = _rng(seed)
    cols = int(math.floor(width / spacing))
    per_layer = cols * cols
    radius = rng.uniform(rmin, rmax, size=n)
    idx = np.arange(n)
    ix = idx % cols
    iy = (idx // cols) % cols
    iz = idx // per_layer
    nodes = (np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5) * spacing
    jit = (spacing - 2.0 * radius) / 2.0
    pos = nodes + rng.uniform(-1.0, 1.0, size=(n, 3)) * jit[:, None]
    walls, facets = [Wall(2, 0.0, 1)], []
    if side_walls:
        walls += [Wall(0, 0.0, 0), Wall(0, width, 0), Wall(1, 0.0, 0), Wall(1, width, 0)]
    if boundary == "facets":
        from .geom import facet_box_triangles
        height = float((pos[:, 2] + radius).max()) + rmax
        walls = []
        facets = facet_box_triangles((0.5 * width, 0.5 * width, 0.5 * height), (0.5 * width, 0.5 * width, 0.5 * height),
                                     wall_mask=31)
    elif boundary != "walls":
        raise ValueError("grid_column: boundary is 'walls' or 'facets'")
    return Scene(pos=pos, radius=radius, material=Material(2600.0, young, 0.3, 0.5), walls=walls, facets=facets,
                 gravity=(0.0, 0.0, -9.81), damping=0.2, dt_factor=0.5, steps=steps,
                 name=f"grid_column_{n}" + ("_facets" if facets else ""))


@dataclass
class BatchSpec:
    scenes: list
    dt_radius: float     # the P-wave step of every scene is taken at this radius
    steps: int


def batched_deposition(n_scenes: int = 512, nmin: int = 500, nmax: int = 50_000, seed: int = 0,
                       spacing: float = 2.5e-3, rmin: float = 0.8e-3, rmax: float = 1.2e-3,
                       steps: int = 2000) -> BatchSpec:
    """C4: independent deposition scenes of uneven size.  Master seed draws
    the per-scene parameters; scene s draws its geometry from seed 1000 + s."""
    rng = _rng(seed)
    counts = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_scenes))).astype(int)
    friction = rng.uniform(0.1, 0.7, size=n_scenes)
    damping = rng.uniform(0.05, 0.4, size=n_scenes)
    scenes = []
    for s in range(n_scenes):
        n = int(counts[s])
        k = int(math.ceil(n ** (1.0 / 3.0)))
        g = _rng(1000 + s)
        radius = g.uniform(rmin, rmax, size=n)
        idx = np.arange(n)
        nodes = (np.stack([idx % k, (idx // k) % k, idx // (k * k)], axis=1).astype(np.float64) + 0.5) * spacing
        jit = (spacing - 2.0 * radius) / 2.0
        pos = nodes + g.uniform(-1.0, 1.0, size=(n, 3)) * jit[:, None]
        width = k * spacing
        walls = [Wall(2, 0.0, 1), Wall(0, 0.0, 0), Wall(0, width, 0), Wall(1, 0.0, 0), Wall(1, width, 0)]
        scenes.append(Scene(pos=pos, radius=radius,
                            material=Material(2600.0, 5e7, 0.3, float(friction[s])), walls=walls,
                            gravity=(0.0, 0.0, -9.81), damping=float(damping[s]), steps=steps,
                            name=f"batch_{s}"))
    return BatchSpec(scenes=scenes, dt_radius=rmin, steps=steps)


def truncated_lognormal(rng: np.random.Generator, n: int, median: float, sigma: float, lo: float,
                        hi: float) -> np.ndarray:
    """Lognormal draws (median, sigma of the log) kept inside [lo, hi]:
    out-of-range draws are redrawn."""
    out = np.exp(rng.normal(math.log(median), sigma, size=n))
    bad = (out < lo) | (out > hi)
    while bad.any():
        out[bad] = np.exp(rng.normal(math.log(median), sigma, size=int(bad.sum())))
        bad = (out < lo) | (out > hi)
    return out


def periodic_lognormal_gas(n: int = 2_000_000, seed: int = 0, median: float = 1e-3, sigma: float = 0.3,
                           young: float = 1e8, poisson: float = 0.25, friction: float = 0.3,
                           damping: float = 0.3, strain_rate: float = 0.01, steps: int = 5000) -> Scene:
    """C3's cloud: lognormal radii truncated to median * exp(+-3 sigma); the
    k^3 >= n nodes of a cubic lattice of spacing 2 r_max (1 + 1e-3), filled
    in node order, each centre jittered by U(-j, j) per axis with
    j = (s - 2r)/2, so no two spheres overlap, also across the periodic
    boundaries.  The cube side is k s.  The workload itself is an isotropic
    compression at `strain_rate` (Cell.velGrad = -rate I, homoDeform 2),
    started after a preparation to a dense state."""
    rng = _rng(seed)
    radius = truncated_lognormal(rng, n, median, sigma, median * math.exp(-3 * sigma), median * math.exp(3 * sigma))
    s = 2.0 * radius.max() * (1.0 + 1e-3)
    k = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while k ** 3 < n:
        k += 1
    idx = np.arange(n)
    nodes = (np.stack([idx % k, (idx // k) % k, idx // (k * k)], axis=1).astype(np.float64) + 0.5) * s
    jit = (s - 2.0 * radius) / 2.0
    pos = nodes + rng.uniform(-1.0, 1.0, size=(n, 3)) * jit[:, None]
    sc = Scene(pos=pos, radius=radius, material=Material(2600.0, young, poisson, friction), walls=[],
               gravity=(0.0, 0.0, 0.0), damping=damping, dt_factor=0.5, steps=steps, periodic=True,
               hsize=np.eye(3) * (k * s), velgrad=-strain_rate * np.eye(3), name=f"periodic_lognormal_{n}")
    return sc


def periodic_bidisperse_gas(n: int = 8_000_000, seed: int = 0, r_small: float = 0.5e-3, r_large: float = 2.0e-3,
                            young: float = 1e8, poisson: float = 0.3, friction: float = 0.5,
                            damping: float = 0.1, shear_rate: float = 1.0, steps: int = 2000) -> Scene:
    """C5's cloud: equal total volume of small and large spheres (so
    n_large / n_small = (r_small / r_large)^3, 1/64 for a size ratio of 4).
    A cubic lattice of spacing s = 2 r_large (1 + 1e-3) holds, at randomly
    permuted nodes, either one large sphere or a block of q^3 small spheres
    (q = r_large / r_small) on a sub-lattice of spacing s / q; small centres
    are jittered by U(-j, j), j = (s/q - 2 r_small)/2, large ones sit on
    their node.  No two spheres overlap, also across the periodic
    boundaries.  Ids: large spheres first, then small ones in node order.
    The workload is simple shear v_x = rate z (Cell.velGrad[0][2] = rate)."""
    rng = _rng(seed)
    q = int(round(r_large / r_small))
    ratio = (r_small / r_large) ** 3
    n_large = int(round(n * ratio / (1.0 + ratio)))
    n_small = n - n_large
    n_blocks = -(-n_small // q ** 3)
    m = int(math.ceil((n_large + n_blocks) ** (1.0 / 3.0) - 1e-9))
    while m ** 3 < n_large + n_blocks:
        m += 1
    s = 2.0 * r_large * (1.0 + 1e-3)
    order = rng.permutation(m ** 3)
    nodes_l, nodes_b = order[:n_large], np.sort(order[n_large:n_large + n_blocks])
    grid = lambda i: (np.stack([i % m, (i // m) % m, i // (m * m)], axis=1).astype(np.float64) + 0.5) * s
    pos_l = grid(nodes_l)
    sub = s / q
    o = np.arange(q ** 3)
    offs = (np.stack([o % q, (o // q) % q, o // (q * q)], axis=1).astype(np.float64) + 0.5) * sub - 0.5 * s
    pos_s = (grid(nodes_b)[:, None, :] + offs[None, :, :]).reshape(-1, 3)[:n_small]
    jit = (sub - 2.0 * r_small) / 2.0
    pos_s = pos_s + rng.uniform(-jit, jit, size=(n_small, 3))
    pos = np.concatenate([pos_l, pos_s])
    radius = np.concatenate([np.full(n_large, r_large), np.full(n_small, r_small)])
    L = np.zeros((3, 3))
    L[0, 2] = shear_rate
    return Scene(pos=pos, radius=radius, material=Material(2600.0, young, poisson, friction), walls=[],
                 gravity=(0.0, 0.0, 0.0), damping=damping, dt_factor=0.5, steps=steps, periodic=True,
                 hsize=np.eye(3) * (m * s), velgrad=L, name=f"periodic_bidisperse_{n}")


def random_velocities(n: int, scale: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian translational velocities [m/s] and angular velocities
    [rad/s] (the latter scaled by 1/(1 mm))."""
    rng = _rng(seed)
    v = rng.normal(0.0, scale, size=(n, 3))
    w = rng.normal(0.0, scale / 1e-3, size=(n, 3))
    return v, w


def compressed_cloud(n: int, box: float, rmin: float, rmax: float, squeeze: float, seed: int
                     ) -> tuple[np.ndarray, np.ndarray]:
    """Random sequential cloud in a cube of side box/squeeze, then all
    centres scaled by `squeeze` (< 1): neighbours that were close now
    overlap, which gives states with many contacts for force checks."""
    pos, radius = random_sequential(n, np.zeros(3), np.full(3, box / squeeze), rmin, rmax, seed)
    return pos * squeeze, radius
