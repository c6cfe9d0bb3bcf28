#!/usr/bin/env python3
"""Benchmark: one DEM timestep over spheres and walls on one MI355X.

Workload (N=1): 200,000 spheres, radius U(0.5, 1.5) mm, jittered column grid
(spacing 3.03 mm, 33 x 33 columns) falling onto a floor inside four side
walls, E = 5e7 Pa, nu = 0.3, friction 0.5 rad, damping 0.2, gravity -9.81,
dt = 0.5 x P-wave step, FP64.  A "step" is one pass of the whole path:
broad phase when the Verlet budget is spent, contact kernel, ordered force
sum + Newton.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra]

Warm-up runs W steps on a throwaway scene of the same configuration; then a
fresh scene is timed for exactly K steps from its initial state (default
K = 10,000, the configuration's length).  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

# Algorithmic bytes (what the method must move, FP64):
#   integrate kernel, per body: read x, v, w, q, r, m (14 doubles) + material
#   and blocked bytes = 114 B; write x, v, w, q (13 doubles) = 104 B.
#   contact kernel: per body gathered once x, v, w, r = 80 B; per real
#   contact ids 8 + shear force r/w 48 + previous normal r/w 48 = 104 B; per
#   non-real candidate its ids, 8 B.
INTEGRATE_BYTES_PER_BODY = 218
CONTACT_BYTES_PER_BODY = 80
CONTACT_BYTES_PER_REAL = 104
CONTACT_BYTES_PER_CANDIDATE = 8


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "traffic_grid_column_200k.md")
    if not os.path.exists(path):
        return None
    m = re.search(rf"traffic_bytes_per_launch {kernel} (\d+) source_sha256_16 (\w+)", open(path).read())
    if not m:
        return None
    csrc = os.path.join(ROOT, "paper_2301_00611_amd", "csrc")
    src = kernel.replace("k_", "") + ".hip"
    blob = open(os.path.join(csrc, src), "rb").read() + open(os.path.join(csrc, "dem_internal.hpp"), "rb").read()
    if hashlib.sha256(blob).hexdigest()[:16] != m.group(2):
        return None
    return float(m.group(1))


def build_scene(spec, precision=0, timing=False, viscel=None):
    """The GPU scene of a spec; viscel = (tc, en, et, dt): a ViscElMat of the
    spec's density and friction angle in place of its FrictMat, stepped at
    the given dt."""
    from paper_2301_00611_amd import dem
    m = spec.material
    s = dem.Scene(gravity=spec.gravity, damping=spec.damping, precision=precision)
    if viscel is None:
        mat = s.add_material(m.density, m.young, m.poisson, m.friction)
    else:
        mat = s.add_viscel_material(m.density, viscel[0], viscel[1], viscel[2], m.friction)
    for w in spec.walls:
        s.add_wall(w.axis, w.position, w.sense, mat)
    for c, h in spec.boxes:
        s.add_box(c, h, mat)
    for tri in spec.facets:
        s.add_facet(*tri, mat=mat)
    s.add_spheres(spec.pos, spec.radius, default_mat=mat)
    s.set_dt(spec.dt_factor * s.pwave_dt() if viscel is None else viscel[3])
    s.set_timing(timing)
    return s


def autotune_for(spec, precision=0, warmup=100, probe_steps=300, cache=None, viscel=None):
    """Autotuner on a throwaway scene of the workload (its probe steps are
    not timed); returns the chosen setting.  With a cache file that holds
    this workload, the stored setting is used without probing."""
    w = build_scene(spec, precision, viscel=viscel)
    w.step(warmup)
    t = w.autotune(probe_steps=probe_steps, cache_path=cache)
    w.close()
    return {k: v for k, v in t.items() if k != "ms_per_step"}


def timed_run(spec, steps, warmup, precision=0, timing=False, tuning=None, viscel=None):
    """Warm up on a throwaway scene, then time exactly `steps` steps of a
    fresh scene from its initial state.  With timing=True every contact and
    integrate launch is bracketed by HIP events (graph event nodes)."""
    import torch
    if warmup > 0:
        w = build_scene(spec, precision, timing=timing, viscel=viscel)
        w.step(warmup)
        w.close()
    s = build_scene(spec, precision, timing=timing, viscel=viscel)
    if tuning:
        s.set_tuning(**tuning)
    s.step(0)
    st0 = s.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = s.stats()
    kern = {}
    for name in ("contact", "integrate", "rebuild"):
        ms, n = s.get_timing(name)
        kern[name] = {"avg_ms": ms, "launches": n}
    s.close()
    return {
        "seconds": t1 - t0,
        "contact_steps": st1["contact_steps"] - st0["contact_steps"],
        "rebuilds": st1["rebuilds"] - st0["rebuilds"],
        "candidates": st1["n_candidates"],
        "contacts_last": st1["n_contacts_ss"] + st1["n_contacts_sw"],
        "kernels": kern,
    }


def cpu_baseline(spec_full, budget_s=15.0):
    """The FP64 oracle, single thread, on a bounded sample of the same
    workload: the bottom layer of the same column (its first 33 x 33 spheres,
    the layer that meets the floor, with the same 5 walls), stepped from the
    initial state for about `budget_s` seconds."""
    from oracle import OracleScene
    cols = int(math.floor(0.1 / 3.03e-3))
    n_sample = min(cols * cols, spec_full.n)
    pos, rad = spec_full.pos[:n_sample], spec_full.radius[:n_sample]
    m = spec_full.material
    dt = spec_full.dt_factor * spec_full.radius.min() * math.sqrt(m.density / m.young)
    o = OracleScene(dt=dt, gravity=spec_full.gravity, damping=spec_full.damping)
    mo = o.add_material(m.density, m.young, m.poisson, m.friction)
    for w in spec_full.walls:
        o.add_wall(w.axis, w.position, w.sense, mo)
    o.add_spheres(pos, rad, default_mat=mo)
    steps, contacts = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(10)
        steps += 10
        contacts += len(o.get_contacts())  # sampled every 10th step
    t = time.perf_counter() - t0
    per_step = t / steps
    n_full = spec_full.n
    return {
        "value": contacts * 10 / t,
        "unit": "contact-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"bottom layer of the same column ({n_sample} spheres + {len(spec_full.walls)} walls), "
                   f"{steps} steps from the initial state in {t:.1f} s, real contacts counted every 10th step; "
                   f"O(N^2) pairs: {per_step * 1e3:.2f} ms/step, {n_sample * steps / t:.3g} body-steps/s; "
                   f"extrapolated {per_step * (n_full / n_sample) ** 2:.1f} s/step at {n_full} spheres"),
        "body_steps_per_s": n_sample * steps / t,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10_000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32-mixed, batched and CPU legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="column",
                    choices=("column", "periodic_compression", "periodic_shear", "batched", "facet_column",
                             "viscel_column"),
                    help="column: the headline line (default); the others run one extra leg alone")
    ap.add_argument("--prepared-state", default=None,
                    help="periodic_compression: .npz holding the prepared packing (written if missing)")
    ap.add_argument("--tuning-cache", default=None,
                    help="autotuner cache file: reuse a stored setting for this workload, or store the one found")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy three times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    if args.copy_calibration:
        import torch
        n = 256 * 1024 * 1024 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "launches": 3}), flush=True)
        return
    if args.workload in PERIODIC_WORKLOADS:
        out = periodic_leg(args.workload, steps=args.steps, log=log, prepared_state=args.prepared_state)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(batched_leg(steps=args.steps, log=log)), flush=True)
        return
    if args.workload == "facet_column":
        print(json.dumps(facet_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)), flush=True)
        return
    if args.workload == "viscel_column":
        print(json.dumps(viscel_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)), flush=True)
        return

    from paper_2301_00611_amd.scenes import grid_column
    spec = grid_column(n=200_000, seed=0)
    log("autotuning the step kernels' launch shape, graph length and Verlet distance")
    tune = autotune_for(spec, 0, warmup=args.warmup, cache=args.tuning_cache)
    log(f"FP64 leg: {spec.n} spheres, {args.steps} steps, setting {tune}")
    r64 = timed_run(spec, args.steps, args.warmup, precision=0, tuning=tune)
    log(f"FP64 leg done in {r64['seconds']:.2f} s; kernel-timing pass")
    # same workload again with HIP events around every contact / integrate
    # launch: per-kernel durations for the roofline
    rt = timed_run(spec, args.steps, 0, precision=0, timing=True, tuning=tune)
    secs = r64["seconds"]
    value = r64["contact_steps"] / secs
    kern = rt["kernels"]
    # dominant kernel by total device time
    tot = {k: v["avg_ms"] * v["launches"] for k, v in kern.items() if k != "rebuild"}
    dom = max(tot, key=tot.get)
    n = spec.n
    if dom == "integrate":
        alg_bytes = INTEGRATE_BYTES_PER_BODY * n
    else:
        c_real = r64["contact_steps"] / max(args.steps, 1)
        cand = r64["candidates"]
        alg_bytes = (CONTACT_BYTES_PER_BODY * n + CONTACT_BYTES_PER_REAL * c_real
                     + CONTACT_BYTES_PER_CANDIDATE * max(cand - c_real, 0))
    avg_s = kern[dom]["avg_ms"] * 1e-3
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    out = {
        "metric": "contact-steps/s",
        "value": value,
        "unit": "contact-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grid_column deposition: 200,000 spheres r~U(0.5,1.5) mm, 0.1x0.1 m box with floor, "
                               "E=5e7, nu=0.3, phi=0.5, damping 0.2, dt=0.5*P-wave",
                   "n_spheres": n, "n_walls": len(spec.walls), "parallelism": "1 GPU"},
        "body_steps_per_s": n * args.steps / secs,
        "rebuilds": r64["rebuilds"],
        "tuning": tune,
        "kernels_ms": {k: v["avg_ms"] for k, v in kern.items()},
        "timing_pass_ms_per_step": rt["seconds"] / args.steps * 1e3,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic("k_" + dom),
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not args.no_extra:
        log("FP32-mixed leg")
        r32 = timed_run(spec, args.steps, args.warmup, precision=1, tuning=autotune_for(spec, 1, warmup=args.warmup,
                                                                                    cache=args.tuning_cache))
        log("batched leg")
        out["fp32_mixed"] = {"value": r32["contact_steps"] / r32["seconds"], "unit": "contact-steps/s",
                             "ms_per_step": r32["seconds"] / args.steps * 1e3}
        out["batched"] = batched_leg(log=log)
        log("facet-box column leg")
        out["facet_column"] = facet_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)
        log("visco-elastic column leg")
        out["viscel_column"] = viscel_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)
        log("periodic compression leg (FP64 vs FP32-mixed)")
        out["periodic_compression"] = periodic_leg("periodic_compression", log=log)
    if not args.no_cpu and not args.no_extra:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(out), flush=True)


def viscel_column_leg(steps, warmup, log=None, cache=None):
    """The 200,000-sphere column of the headline line with the visco-elastic
    law (ViscElMat, e_n = e_t = 0.5) in place of the linear one, at the same
    dt; t_c = pi sqrt(m_eff / k_n) of the linear law for two 1 mm spheres
    (3.28e-5 s, about 18 steps per collision)."""
    import math
    from paper_2301_00611_amd.scenes import grid_column
    spec = grid_column(n=200_000, seed=0)
    m = spec.material
    mass = 4.0 / 3.0 * math.pi * 1e-3 ** 3 * m.density
    tc = math.pi * math.sqrt(0.5 * mass / (m.young * 1e-3))
    dt = spec.dt_factor * float(spec.radius.min()) * math.sqrt(m.density / m.young)
    ve = (tc, 0.5, 0.5, dt)
    tune = autotune_for(spec, 0, warmup=warmup, cache=cache, viscel=ve)
    if log:
        log(f"visco-elastic column: {spec.n} spheres, tc {tc:.3e} s, dt {dt:.3e} s, {steps} steps, setting {tune}")
    r = timed_run(spec, steps, warmup, precision=0, tuning=tune, viscel=ve)
    rt = timed_run(spec, steps, 0, precision=0, timing=True, tuning=tune, viscel=ve)
    return {
        "workload": "grid_column deposition with the visco-elastic law: 200,000 spheres r~U(0.5,1.5) mm, "
                    f"tc={tc:.3e} s, en=et=0.5, phi=0.5, damping 0.2, dt={dt:.3e} s (the linear column's)",
        "value": r["contact_steps"] / r["seconds"],
        "unit": "contact-steps/s",
        "ms_per_step": r["seconds"] / steps * 1e3,
        "rebuilds": r["rebuilds"],
        "tuning": tune,
        "kernels_ms": {k: v["avg_ms"] for k, v in rt["kernels"].items()},
        "contacts_last": r["contacts_last"],
    }


def facet_column_leg(steps, warmup, log=None, cache=None):
    """The 200,000-sphere column of the headline line in an open-topped
    facet box (geom.facetBox, wallMask=31: 10 triangles) instead of its 5
    planes: the contact kernel's box/facet instantiation and the broad
    phase's closest-point tests at full size."""
    from paper_2301_00611_amd.scenes import grid_column
    spec = grid_column(n=200_000, seed=0, boundary="facets")
    tune = autotune_for(spec, 0, warmup=warmup, cache=cache)
    if log:
        log(f"facet column: {spec.n} spheres, {len(spec.facets)} facets, {steps} steps, setting {tune}")
    r = timed_run(spec, steps, warmup, precision=0, tuning=tune)
    rt = timed_run(spec, steps, 0, precision=0, timing=True, tuning=tune)
    return {
        "workload": "grid_column deposition in an open facet box: 200,000 spheres r~U(0.5,1.5) mm, "
                    "0.1x0.1 m footprint, 10 facets, E=5e7, nu=0.3, phi=0.5, damping 0.2, dt=0.5*P-wave",
        "value": r["contact_steps"] / r["seconds"],
        "unit": "contact-steps/s",
        "ms_per_step": r["seconds"] / steps * 1e3,
        "rebuilds": r["rebuilds"],
        "tuning": tune,
        "kernels_ms": {k: v["avg_ms"] for k, v in rt["kernels"].items()},
        "contacts_last": r["contacts_last"],
    }


def _periodic_scene(H, L, spec, pos, vel, angvel, precision, friction=None, track_energy=False):
    from paper_2301_00611_amd import dem
    m = spec.material
    g = dem.Scene(periodic=True, hsize=H, velgrad=L, damping=spec.damping, gravity=spec.gravity,
                  precision=precision, track_energy=track_energy)
    mg = g.add_material(m.density, m.young, m.poisson, m.friction if friction is None else friction)
    g.add_spheres(pos, spec.radius, vel=vel, angvel=angvel, default_mat=mg)
    g.set_dt(spec.dt_factor * g.pwave_dt())
    return g


PERIODIC_WORKLOADS = {
    # name: (generator, spheres, tiling of the prepared packing, description)
    "periodic_compression": ("periodic_lognormal_gas", 2_000_000, 2,
                             "periodic isotropic compression: {n} spheres, lognormal r (median 1 mm, sigma 0.3), "
                             "E=1e8, nu=0.25, phi=0.3, damping 0.3, velGrad=-0.01 I, homoDeform 2, dt=0.5*P-wave"),
    "periodic_shear": ("periodic_bidisperse_gas", 8_000_000, 2,
                       "periodic simple shear: {n} spheres, r = 0.5 and 2.0 mm (equal volumes), E=1e8, nu=0.3, "
                       "phi=0.5, damping 0.1, velGrad[0][2] = 1/s, homoDeform 2, dt=0.5*P-wave"),
}


def _workload_spec(name, n, seed=0):
    from paper_2301_00611_amd import scenes
    return getattr(scenes, PERIODIC_WORKLOADS[name][0])(n=n, seed=seed)


def prepare_periodic(name, n, seed=0, target_pressure=1e3, log=None):
    """Unmeasured preparation of a periodic workload: its lattice cloud of
    n / tile^3 spheres compressed frictionless (friction 0, same stiffness
    and damping) to a jammed packing whose relaxed mean pressure reaches the
    target, held 2000 more steps at rest, then replicated tile^3 times into
    a cell tile times wider (the same periodic packing, n spheres).  Returns
    the spec of the n-sphere workload and its prepared state (positions,
    velocities, spins, cell)."""
    import numpy as np
    from paper_2301_00611_amd.prepare import jam_isotropic, mean_pressure, tile_periodic
    tile = PERIODIC_WORKLOADS[name][2]
    n0 = n // tile ** 3
    spec0 = _workload_spec(name, n0, seed)
    vs = float((4.0 / 3.0 * math.pi * spec0.radius ** 3).sum())
    g = _periodic_scene(spec0.hsize, np.zeros((3, 3)), spec0, spec0.pos, None, None, 0, friction=0.0)
    rec = jam_isotropic(g, spec0.dt_factor * g.pwave_dt(), vs, target_pressure, log=log)
    g.step(2000)
    rec["pressure_held"] = mean_pressure(g)
    rec["coordination_held"] = g.stats()["coordination"]
    st = g.get_state()
    H, _ = g.get_cell()
    g.close()
    pos, rad, vel, ang, H2 = tile_periodic(st["pos"], spec0.radius, st["vel"], st["angvel"], H, (tile,) * 3)
    spec = _workload_spec(name, 16, seed)  # parameters of the workload
    spec.pos, spec.radius = pos, rad
    rec["prepared_spheres"] = n0
    rec["tiling"] = [tile] * 3
    rec["cell"] = H2
    return spec, {"pos": pos, "vel": vel, "angvel": ang}, H2, rec


def periodic_leg(name="periodic_compression", steps=5000, n=None, log=None, prepared_state=None):
    """A dense periodic workload (C3: isotropic compression at 0.01/s; C5:
    bidisperse simple shear at 1/s), FP64 vs FP32-mixed on the same prepared
    packing: throughput of each, kernel durations, and the FP32-mixed error
    against FP64 from the identical state (pair set, per-contact and
    per-body force) and over the run (energy terms, coordination)."""
    import numpy as np
    import torch
    log = log or (lambda m: None)
    n = n or PERIODIC_WORKLOADS[name][1]
    if prepared_state and os.path.exists(prepared_state):
        d = np.load(prepared_state)
        spec = _workload_spec(name, 16)
        spec.pos, spec.radius = d["pos"], d["radius"]
        st = {"pos": d["pos"], "vel": d["vel"], "angvel": d["angvel"]}
        H, rec = d["H"], {"loaded_from": prepared_state}
    else:
        spec, st, H, rec = prepare_periodic(name, n, log=log)
        if prepared_state:
            np.savez(prepared_state, pos=st["pos"], vel=st["vel"], angvel=st["angvel"], radius=spec.radius, H=H)
    n = len(spec.radius)
    L = spec.velgrad
    tile = PERIODIC_WORKLOADS[name][2]
    out = {"workload": PERIODIC_WORKLOADS[name][3].format(n=n)
           + f"; from a packing prepared at {n // tile ** 3} spheres and tiled {tile}x{tile}x{tile}",
           "preparation": {k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in rec.items() if k != "cell0"},
           "steps": steps}
    # identical-state one-step comparison
    one = {}
    for prec in (0, 1):
        g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], prec)
        g.step(1)
        one[prec] = (g.get_contacts(), g.get_state())
        g.close()
    c64, c32 = one[0][0], one[1][0]
    k64 = set(zip(c64["id1"].tolist(), c64["id2"].tolist(), map(tuple, c64["cell"].tolist())))
    k32 = set(zip(c32["id1"].tolist(), c32["id2"].tolist(), map(tuple, c32["cell"].tolist())))
    err = {"pair_set_differences": len(k64 ^ k32), "contacts": len(c64)}
    if len(c64) and not (k64 ^ k32):
        o64 = np.lexsort((c64["id2"], c64["id1"]))
        o32 = np.lexsort((c32["id2"], c32["id1"]))
        a, b = c64[o64], c32[o32]
        scale = a["kn"] * 4 * np.finfo(float).eps * (2 * spec.radius.max())
        fa, fb = a["fn"] + a["fs"], b["fn"] + b["fs"]
        e = np.linalg.norm(fb - fa, axis=1) / (np.linalg.norm(fa, axis=1) + scale)
        err["contact_force_rel_max"] = float(e.max())
        err["contact_force_rel_p99"] = float(np.quantile(e, 0.99))
        ssum = np.zeros(len(spec.radius))
        mag = np.linalg.norm(fa, axis=1)
        np.add.at(ssum, a["id1"], mag)
        np.add.at(ssum, a["id2"], mag)
        t = ssum > 0
        eb = np.linalg.norm(one[1][1]["force"] - one[0][1]["force"], axis=1)[t] / ssum[t]
        err["body_force_rel_max"] = float(eb.max())
    out["fp32_vs_fp64_one_step"] = err
    # timed runs (the launch setting chosen by the autotuner on a copy of the
    # same state, which it advances), then the same runs with energy
    # tracking for the statistics
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], prec)
        tune = g.autotune(probe_steps=200)
        g.close()
        g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], prec)
        g.set_tuning(**{k: v for k, v in tune.items() if k != "ms_per_step"})
        g.step(0)
        s0 = g.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s1 = g.stats()
        g.set_timing(True)
        g.step(500)
        kern = {k: g.get_timing(k)[0] for k in ("contact", "integrate", "rebuild")}
        st_t = g.stats()
        g.close()
        c_real = (s1["contact_steps"] - s0["contact_steps"]) / steps
        r = {"value": (s1["contact_steps"] - s0["contact_steps"]) / el, "unit": "contact-steps/s",
             "ms_per_step": el / steps * 1e3, "body_steps_per_s": n * steps / el, "rebuilds": s1["rebuilds"] - s0["rebuilds"],
             "contacts_mean": c_real, "candidates": s1["n_candidates"], "coordination_end": s1["coordination"],
             "kernels_ms": kern, "tuning": tune}
        # interaction-kernel rooflines (algorithmic bytes per launch)
        bpb, bpc = (80, 104) if prec == 0 else (52, 80)
        cand = st_t["n_candidates"]
        cb = bpb * n + bpc * c_real + 8 * max(cand - c_real, 0)
        ib = (INTEGRATE_BYTES_PER_BODY + (0 if prec == 0 else 28)) * n
        if kern["contact"] > 0:
            r["contact_roofline"] = {"bytes": cb, "achieved_GBs": cb / (kern["contact"] * 1e-3) / 1e9,
                                     "frac": cb / (kern["contact"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if kern["integrate"] > 0:
            r["integrate_roofline"] = {"bytes": ib, "achieved_GBs": ib / (kern["integrate"] * 1e-3) / 1e9,
                                       "frac": ib / (kern["integrate"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[name] = r
        log(f"{out['workload'][:30]} {name}: {r}")
    out["controlled_cell"] = controlled_cell_run(H, spec, st, steps, log)
    stats = {}
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], prec, track_energy=True)
        rows = []
        win = min(500, steps)
        for _ in range(max(1, steps // win)):
            g.step(win)
            e = g.get_energy()
            rows.append([e["kinetic"], e["kin_rot"], e["elastic"], e["damp_dissip"], e["plastic_dissip"],
                         g.stats()["coordination"]])
        g.close()
        stats[name] = np.array(rows)
    a, b = stats["fp64"], stats["fp32_mixed"]
    scale = np.abs(a[:, :5]).sum(axis=1, keepdims=True)
    out["fp32_vs_fp64_run"] = {
        "energy_terms_rel_to_total_max": float((np.abs(b[:, :5] - a[:, :5]) / scale).max()),
        "coordination_rel_max": float((np.abs(b[:, 5] - a[:, 5]) / np.maximum(a[:, 5], 1e-30)).max()),
        "windows": int(a.shape[0]), "window_steps": min(500, steps)}
    return out


def controlled_cell_run(H, spec, st, steps, log=None):
    """The stress-controlled cell on the prepared packing (FP64), updates
    every 5 steps on the device: `drive` steers the packing to an isotropic
    stress of twice its mean pressure; `hold` keeps it at its own pressure;
    `off` runs the same steps without the controller (zero velocity
    gradient)."""
    import numpy as np
    import torch
    from paper_2301_00611_amd.prepare import mean_pressure
    res = {}
    for mode in ("drive", "hold", "off"):
        g = _periodic_scene(H, np.zeros((3, 3)), spec, st["pos"], st["vel"], st["angvel"], 0)
        g.step(1)
        p0 = mean_pressure(g)
        goal = -(2.0 if mode == "drive" else 1.0) * max(p0, 1.0)
        if mode != "off":
            g.set_peri_triax((goal, goal, goal), 7, glob_update=5, max_strain_rate=(1.0, 1.0, 1.0), grow_damping=0.25)
        s0 = g.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s1 = g.stats()
        cs = s1["contact_steps"] - s0["contact_steps"]
        r = {"ms_per_step": el / steps * 1e3, "rebuilds": s1["rebuilds"] - s0["rebuilds"],
             "value": cs / el, "unit": "contact-steps/s", "contacts_per_step": cs / steps,
             "ns_per_contact_step": el / max(cs, 1) * 1e9}
        if mode != "off":
            c = g.get_peri_triax()
            r.update({"goal_pressure": -goal, "start_pressure": p0, "updates": c["updates"],
                      "stress_end": c["stress"], "strain_end": c["strain"], "unbalanced_end": c["unbalanced"],
                      "pressure_end": mean_pressure(g)})
        res[mode] = r
        g.close()
    # the three runs hold different contact counts (a held or driven cell
    # keeps compressing as the packing relaxes), so the cost is compared per
    # contact-step; the controller's kernels are in the kernel trace
    res["controller_overhead_per_contact_step"] = (res["hold"]["ns_per_contact_step"]
                                                   / res["off"]["ns_per_contact_step"] - 1.0)
    if log:
        log(f"controlled cell: {res}")
    return res


def _build_batch(spec, dt, precision=0):
    from paper_2301_00611_amd import dem
    params = [dem.make_params(dt=dt, gravity=s.gravity, damping=s.damping, precision=precision) for s in spec.scenes]
    b = dem.Batch(params)
    for i, s in enumerate(spec.scenes):
        v = b.scene(i)
        m = v.add_material(s.material.density, s.material.young, s.material.poisson, s.material.friction)
        for w in s.walls:
            v.add_wall(w.axis, w.position, w.sense, m)
        v.add_spheres(s.pos, s.radius, default_mat=m)
    return b


def _time_batch(b, steps):
    import torch
    b.step(1)
    s0 = b.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s1 = b.stats()
    return t, s1["contact_steps"] - s0["contact_steps"]


def batched_leg(n_scenes=512, steps=2000, sequential_steps=200, log=None):
    """C4: 512 independent deposition scenes (log-uniform sizes 500..50,000,
    per-scene friction and damping) stepped together, FP64 and FP32-mixed:
    scene-steps/s with the default launch setting and with the autotuner's
    (its probe steps are not timed), against the same scenes stepped one
    after another as single FP64 scenes (`sequential_steps` steps each)."""
    from paper_2301_00611_amd import dem
    from paper_2301_00611_amd.scenes import batched_deposition
    log = log or (lambda m: None)
    spec = batched_deposition(n_scenes=n_scenes, steps=steps)
    dt = 0.5 * spec.dt_radius * math.sqrt(2600.0 / 5e7)
    nbodies = sum(s.n for s in spec.scenes)
    out = {"unit": "scene-steps/s", "n_scenes": n_scenes, "n_spheres": nbodies, "steps": steps}
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        b = _build_batch(spec, dt, prec)
        t_def, c_def = _time_batch(b, steps)
        tune = b.autotune(probe_steps=100)
        t_tun, c_tun = _time_batch(b, steps)
        b.close()
        out[name] = {"value": n_scenes * steps / t_tun, "seconds": t_tun, "body_steps_per_s": nbodies * steps / t_tun,
                     "contact_steps_per_s": c_tun / t_tun, "default_setting_value": n_scenes * steps / t_def,
                     "tuning": tune}
        log(f"batched {name}: {out[name]}")
    out["value"] = out["fp64"]["value"]
    # the same scenes one after another through the single-scene FP64 path
    import torch
    t_seq = 0.0
    for s in spec.scenes:
        g = dem.Scene(gravity=s.gravity, damping=s.damping)
        m = g.add_material(s.material.density, s.material.young, s.material.poisson, s.material.friction)
        for w in s.walls:
            g.add_wall(w.axis, w.position, w.sense, m)
        g.add_spheres(s.pos, s.radius, default_mat=m)
        g.set_dt(dt)
        g.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(sequential_steps)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        g.close()
    out["sequential_fp64"] = {"value": n_scenes * sequential_steps / t_seq, "steps_per_scene": sequential_steps,
                              "seconds": t_seq}
    out["speedup_vs_sequential"] = out["value"] / out["sequential_fp64"]["value"]
    return out


if __name__ == "__main__":
    main()
