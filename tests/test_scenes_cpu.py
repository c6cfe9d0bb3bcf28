"""The seeded input generators (paper_2301_00611_amd/scenes.py) against the
recipes they state: counts, radius ranges and distributions, no two
spheres overlapping at the start (also across periodic boundaries), every
sphere on the right side of its walls, equal volumes of the bidisperse
mix, and the same scene for the same seed.  Small sizes of the same
recipes; an independent k-d tree does the overlap checks."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2301_00611_amd import scenes


def _max_overlap(pos, radius, boxsize=None):
    """Largest r_i + r_j - |x_i - x_j| over all pairs closer than 2 r_max
    (negative when nothing overlaps)."""
    tree = cKDTree(pos, boxsize=boxsize)
    pairs = tree.query_pairs(2.0 * radius.max(), output_type="ndarray")
    if len(pairs) == 0:
        return -np.inf
    d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
    if boxsize is not None:
        d -= boxsize * np.round(d / boxsize)
    return float(np.max(radius[pairs[:, 0]] + radius[pairs[:, 1]] - np.linalg.norm(d, axis=1)))


def test_cloud_box():
    sc = scenes.cloud_box(n=1000, seed=3)
    assert sc.n == 1000 and len(sc.walls) == 6
    assert sc.radius.min() >= 0.9e-3 and sc.radius.max() <= 1.1e-3
    assert _max_overlap(sc.pos, sc.radius) < 0.0
    assert np.all(sc.pos - sc.radius[:, None] >= 0.0) and np.all(sc.pos + sc.radius[:, None] <= 0.030)


def test_grid_column():
    n, width, s = 20_000, 0.1, 3.03e-3
    sc = scenes.grid_column(n=n, seed=4)
    cols = int(math.floor(width / s))
    assert cols == 33 and sc.n == n
    assert sc.radius.min() >= 0.5e-3 and sc.radius.max() <= 1.5e-3
    assert abs(sc.radius.mean() - 1e-3) < 2e-5   # U(0.5, 1.5) mm
    assert _max_overlap(sc.pos, sc.radius) <= 0.0
    assert np.all(sc.pos[:, 2] - sc.radius >= -1e-15)   # the lowest layer at most touches the floor
    assert np.all(sc.pos[:, :2] - sc.radius[:, None] >= -1e-15)
    assert np.all(sc.pos[:, :2] + sc.radius[:, None] <= cols * s + 1e-15)
    assert [(w.axis, w.position, w.sense) for w in sc.walls][0] == (2, 0.0, 1)
    layers = np.unique(np.floor(sc.pos[:, 2] / s))
    assert len(layers) == -(-n // (cols * cols))


def test_batched_deposition():
    b = scenes.batched_deposition(n_scenes=12, nmin=500, nmax=5000, seed=5)
    counts = np.array([sc.n for sc in b.scenes])
    assert len(b.scenes) == 12 and counts.min() >= 500 and counts.max() <= 5000
    for sc in b.scenes:
        assert 0.1 <= sc.material.friction <= 0.7 and 0.05 <= sc.damping <= 0.4
        assert sc.radius.min() >= 0.8e-3 and sc.radius.max() <= 1.2e-3
        assert _max_overlap(sc.pos, sc.radius) <= 0.0
        assert np.all(sc.pos[:, 2] - sc.radius >= -1e-15)
    assert len({sc.material.friction for sc in b.scenes}) == 12


def test_periodic_lognormal_gas():
    n = 20_000
    sc = scenes.periodic_lognormal_gas(n=n, seed=6)
    lo, hi = 1e-3 * math.exp(-0.9), 1e-3 * math.exp(0.9)
    assert sc.n == n and sc.radius.min() >= lo and sc.radius.max() <= hi
    assert abs(np.median(sc.radius) / 1e-3 - 1.0) < 0.01
    assert abs(np.std(np.log(sc.radius)) / 0.3 - 1.0) < 0.03   # the +-3 sigma truncation narrows it ~1.4 %
    side = sc.hsize[0, 0]
    assert np.allclose(sc.hsize, np.eye(3) * side)
    assert np.all(sc.pos >= 0.0) and np.all(sc.pos < side)
    assert _max_overlap(sc.pos, sc.radius, boxsize=side) < 0.0
    assert np.allclose(sc.velgrad, -0.01 * np.eye(3)) and sc.periodic


def test_periodic_bidisperse_gas():
    n = 13_000
    sc = scenes.periodic_bidisperse_gas(n=n, seed=7)
    small, large = sc.radius == 0.5e-3, sc.radius == 2.0e-3
    assert sc.n == n and np.all(small | large)
    vol_s, vol_l = (sc.radius[small] ** 3).sum(), (sc.radius[large] ** 3).sum()
    assert abs(vol_s / vol_l - 1.0) < 0.01          # equal volumes of the two sizes
    assert np.all(np.nonzero(large)[0] < np.nonzero(small)[0].min())   # large spheres first
    side = sc.hsize[0, 0]
    assert np.all(sc.pos >= 0.0) and np.all(sc.pos < side)
    assert _max_overlap(sc.pos, sc.radius, boxsize=side) < 0.0
    assert sc.velgrad[0, 2] == 1.0 and np.count_nonzero(sc.velgrad) == 1


@pytest.mark.parametrize("make", [lambda s: scenes.cloud_box(n=300, seed=s),
                                  lambda s: scenes.grid_column(n=2000, seed=s),
                                  lambda s: scenes.periodic_lognormal_gas(n=2000, seed=s),
                                  lambda s: scenes.periodic_bidisperse_gas(n=6500, seed=s)])
def test_same_seed_same_scene(make):
    a, b, c = make(11), make(11), make(12)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.radius, b.radius)
    assert not np.array_equal(a.pos, c.pos)


def test_random_velocities():
    v, w = scenes.random_velocities(1000, 0.05, 9)
    v2, w2 = scenes.random_velocities(1000, 0.05, 9)
    assert v.shape == (1000, 3) and w.shape == (1000, 3)
    assert np.array_equal(v, v2) and np.array_equal(w, w2)
