"""Preparation of dense periodic packings (the role PeriIsoCompressor and
PeriTriaxController play in the documentation's periodic tutorials).

Two routes, both through the C ABI only (every step runs in the HIP
library):
  * compress_to_pressure: the library's stress-controlled cell
    (dem_set_peri_triax) drives the cell to a target isotropic stress and
    stops there;
  * jam_isotropic: a host-side schedule of compressions, velocity resets
    and relaxations (dem_set_velgrad, dem_step, dem_get_stress,
    dem_set_state), which reaches a static jammed packing;
  * settle_iso: the library's isotropic compressor (dem_set_peri_iso)
    holding a near-jammed packing at a mean stress until its unbalanced
    force is small.
"""
from __future__ import annotations

import time

import numpy as np


def mean_pressure(scene) -> float:
    """p = -trace(sigma)/3 of the Love-Weber stress (compression > 0)."""
    return -float(np.trace(scene.get_stress())) / 3.0


def quench(scene, L) -> None:
    """Remove the velocity fluctuations: every sphere gets the velocity of
    the homogeneous field, v = L x, and no spin (a kinetic-energy reset, as
    used to speed up static packing preparation)."""
    st = scene.get_state()
    scene.set_state(vel=st["pos"] @ np.asarray(L).T, angvel=np.zeros_like(st["pos"]))


def tile_periodic(pos, radius, vel, angvel, hsize, reps=(2, 2, 2)):
    """Replicate a periodic packing reps[0] x reps[1] x reps[2] times: copy
    (i, j, k) is shifted by H (i, j, k); the new cell has columns
    reps[a] * H[:, a].  Contacts across the old boundaries become contacts
    between copies, so the result is the same packing in a bigger cell.
    Copies are ordered with i fastest; within a copy the original order."""
    H = np.asarray(hsize, dtype=np.float64)
    shifts = [H @ np.array([i, j, k], dtype=np.float64)
              for k in range(reps[2]) for j in range(reps[1]) for i in range(reps[0])]
    n = len(radius)
    out_pos = np.concatenate([pos + sh for sh in shifts])
    rep = lambda a: None if a is None else np.tile(np.asarray(a), (len(shifts), 1))
    out_rad = np.tile(np.asarray(radius), len(shifts))
    assert out_pos.shape == (n * len(shifts), 3)
    return out_pos, out_rad, rep(vel), rep(angvel), H * np.asarray(reps, dtype=np.float64)[None, :]


def jam_isotropic(scene, dt: float, solid_volume: float, target_pressure: float, fast_rate: float = 30.0,
                  rate: float = 3.0, loose_fraction: float = 0.58, strain_step: float = 2e-3,
                  max_cycles: int = 60, log=None) -> dict:
    """Isotropic compression of a periodic scene to a jammed packing whose
    static mean pressure is at least the target.

    1. Loose: compress at `fast_rate` [1/s] until the solid fraction reaches
       `loose_fraction`, resetting the fluctuations every 1000 steps.
    2. Cycles: compress by `strain_step` (volumetric strain / 3) at `rate`,
       stop the cell, reset the fluctuations and relax 500 steps four
       times, then relax 1500 steps untouched; the pressure left is the
       static one (a packing below jamming relaxes to zero).  Stop once it
       reaches the target.
    Ends with a zero velocity gradient.  `dt` is the scene's timestep and
    `solid_volume` the spheres' total volume.  Returns a record of the
    run."""
    h0, _ = scene.get_cell()
    vs = float(solid_volume)
    frac = lambda: vs / abs(np.linalg.det(scene.get_cell()[0]))
    t0 = time.perf_counter()
    steps = 0

    def run(r, k):
        nonlocal steps
        L = -r * np.eye(3)
        scene.set_velgrad(L)
        scene.step(k)
        steps += k
        return L

    while frac() < loose_fraction:
        L = run(fast_rate, 1000)
        quench(scene, L)
    p = 0.0
    cycles = 0
    k = max(1, int(round(strain_step / (rate * dt))))
    for cycles in range(1, max_cycles + 1):
        run(rate, k)
        scene.set_velgrad(np.zeros((3, 3)))
        for _ in range(4):
            quench(scene, np.zeros((3, 3)))
            scene.step(500)
        scene.step(1500)
        steps += 3500
        p = mean_pressure(scene)
        if log is not None:
            log(f"jam cycle {cycles}: held p = {p:.4g} Pa, Z = {scene.stats()['coordination']:.3f}, "
                f"solid fraction {frac():.4f}")
        if p >= target_pressure:
            break
    st = scene.stats()
    h, _ = scene.get_cell()
    return {"steps": steps, "cycles": cycles, "pressure": p, "coordination": st["coordination"],
            "solid_fraction": vs / abs(np.linalg.det(h)), "cell": h, "cell0": h0,
            "converged": p >= target_pressure, "seconds": time.perf_counter() - t0}


def compress_to_pressure(scene, target_pressure: float, max_strain_rate: float = 30.0, grow_damping: float = 0.25,
                         glob_update: int = 5, max_unbalanced: float = 0.05, stress_tol: float = 0.05,
                         max_steps: int = 200_000, report_every: int = 2000, reset_fluctuations: bool = False,
                         log=None) -> dict:
    """Isotropic compression of a periodic scene by the stress-controlled
    cell (PeriTriaxController): goal sigma_ii = -target_pressure on every
    axis, reached when each is within stress_tol * target_pressure and the
    unbalanced force is at most max_unbalanced; the cell then stops.  With
    `reset_fluctuations`, the velocity fluctuations are reset (spheres follow the
    cell's homogeneous field) every `report_every` steps, which lets a
    loose packing settle into a static one sooner.  The controller is
    switched off at the end.  Returns a record of the run."""
    p = float(target_pressure)
    scene.set_peri_triax((-p, -p, -p), 7, glob_update=glob_update, max_strain_rate=(max_strain_rate,) * 3,
                         grow_damping=grow_damping, max_unbalanced=max_unbalanced, abs_stress_tol=stress_tol * p,
                         rel_stress_tol=0.0, stop_when_done=1)
    t0 = time.perf_counter()
    it0 = scene.stats()["iter"]
    st = scene.get_peri_triax()
    while scene.stats()["iter"] - it0 < max_steps:
        scene.step(min(report_every, max_steps - (scene.stats()["iter"] - it0)))
        st = scene.get_peri_triax()
        if log is not None:
            log(f"controlled cell: step {scene.stats()['iter'] - it0}, stress {[round(x, 1) for x in st['stress']]}, "
                f"unbalanced {st['unbalanced']:.3g}, strain {[round(x, 4) for x in st['strain']]}, "
                f"Z {scene.stats()['coordination']:.3f}")
        if st["done"]:
            break
        if reset_fluctuations:
            r = st["strain_rate"]
            quench(scene, np.diag(r))
    scene.set_peri_triax(None)
    stats = scene.stats()
    return {"steps": stats["iter"] - it0, "converged": bool(st["done"]), "stress": st["stress"],
            "strain": st["strain"], "unbalanced": st["unbalanced"], "updates": st["updates"],
            "coordination": stats["coordination"], "seconds": time.perf_counter() - t0}



def settle_iso(scene, target_pressure: float, max_unbalanced: float = 0.02, stress_tol: float = 0.02,
               max_steps: int = 100_000, report_every: int = 5000, max_strain_rate: float = 1.0,
               log=None) -> dict:
    """The isotropic compressor (PeriIsoCompressor, keepProportions) driving
    the mean stress of a periodic scene to -target_pressure and holding it
    until the unbalanced force is at most max_unbalanced (the compressor's
    own goal test); the cell then stops.  Meant for a packing that is
    already near jamming (from jam_isotropic): from a gas the stiffness-based
    rate only keeps up the kinetic pressure and the packing densifies
    slowly.  Returns a record of the run."""
    p = float(target_pressure)
    scene.set_peri_iso([-p], global_update=5, max_strain_rate=max_strain_rate, grow_damping=0.25,
                       max_unbalanced=max_unbalanced, abs_stress_tol=stress_tol * p, rel_stress_tol=0.0,
                       stop_when_done=1)
    t0 = time.perf_counter()
    it0 = scene.stats()["iter"]
    st = scene.get_peri_iso()
    while scene.stats()["iter"] - it0 < max_steps:
        scene.step(min(report_every, max_steps - (scene.stats()["iter"] - it0)))
        st = scene.get_peri_iso()
        if log is not None:
            log(f"isotropic compressor: step {scene.stats()['iter'] - it0}, mean stress {st['sigma']:.4g}, "
                f"unbalanced {st['unbalanced']:.3g}, Z {scene.stats()['coordination']:.3f}")
        if st["done"]:
            break
    scene.set_peri_iso(None)
    scene.set_velgrad(np.zeros((3, 3)))
    stats = scene.stats()
    return {"steps": stats["iter"] - it0, "converged": bool(st["done"]), "mean_stress": st["sigma"],
            "unbalanced": st["unbalanced"], "updates": st["updates"], "coordination": stats["coordination"],
            "seconds": time.perf_counter() - t0}
