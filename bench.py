#!/usr/bin/env python3
"""Benchmark: the DEM timestep over a dense periodic packing on one MI355X.

Headline (N=1), the largest configuration that fits one GPU: 8,000,000
spheres, bidisperse radii 0.5 and 2.0 mm (equal volumes), periodic simple
shear at 1/s (Cell.velGrad[0][2] = 1, homoDeform 2), E = 1e8 Pa, nu = 0.3,
friction 0.5 rad, damping 0.1, dt = 0.5 x P-wave step, FP64, from a dense
packing prepared at a mean stress of 1 kPa (not timed).  A "step" is one
pass of the whole path: a broad-phase run when the Verlet budget is spent,
the contact kernel, the ordered force sum + Newton, the cell update.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--workload NAME]

W untimed steps run on the timed scene itself, then one broad-phase run
brings the pair list up to date, then exactly K steps are timed (inputs
resident in HBM, no host<->device copies in the timed region but the
per-chunk 64-byte counter read-back).  A second pass of the same scene with
per-kernel HIP events gives the kernel durations for the roofline and the
broad phase's cost per run and run rate, reported beside the timed rate as
an amortised term.  FP32-mixed runs beside it on the same prepared packing.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

# Algorithmic bytes (what the method must move):
#   contact kernel: per body gathered once x, v, w, r = 80 B (FP64 in both
#   precisions: the FP32-mixed kernel forms the relative velocity from the
#   FP64 velocities); per real contact ids 8 + shear force r/w 48 + previous
#   normal r/w 48 = 104 B (FP32-mixed: normal in FP32, 80 B); per non-real
#   candidate its ids, 8 B.
#   integrate kernel, per body: read x, v, w, q, r, m (14 doubles) + material
#   and blocked bytes = 114 B; write x, v, w, q (13 doubles) = 104 B.
CONTACT_BYTES = {0: (80, 104, 8), 1: (80, 80, 8)}
INTEGRATE_BYTES_PER_BODY = 218


def contact_algorithmic_bytes(precision, n_bodies, contacts, candidates):
    b_body, b_real, b_cand = CONTACT_BYTES[precision]
    return b_body * n_bodies + b_real * contacts + b_cand * max(candidates - contacts, 0)


def kernel_source_hash(kernel):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2301_00611_amd", "csrc")
    src = kernel.replace("k_", "") + ".hip"
    blob = open(os.path.join(csrc, src), "rb").read() + open(os.path.join(csrc, "dem_internal.hpp"), "rb").read()
    return hashlib.sha256(blob).hexdigest()[:16]


def profiled_traffic(kernel, profile, precision=0):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (profiles/<profile>.md), or None when the kernel's source
    changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", profile + ".md")
    if not os.path.exists(path):
        return None
    m = re.search(rf"traffic_bytes_per_launch {kernel} precision {precision} (\d+) source_sha256_16 (\w+)",
                  open(path).read())
    if not m or m.group(2) != kernel_source_hash(kernel):
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
    fresh scene from its initial state (its pair list built before the
    timed region).  With timing=True every contact and integrate launch is
    bracketed by HIP events."""
    import torch
    if warmup > 0:
        w = build_scene(spec, precision, timing=timing, viscel=viscel)
        w.step(warmup)
        w.close()
    s = build_scene(spec, precision, timing=timing, viscel=viscel)
    if tuning:
        s.set_tuning(**tuning)
    s.step(0)  # the initial broad-phase run, outside the timed region
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


# ------------------------------------------------------------------ periodic

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
    "periodic_shear": ("periodic_bidisperse_gas", 8_000_000, 4,
                       "periodic simple shear: {n} spheres, r = 0.5 and 2.0 mm (equal volumes), E=1e8, nu=0.3, "
                       "phi=0.5, damping 0.1, velGrad[0][2] = 1/s, homoDeform 2, dt=0.5*P-wave"),
    "periodic_compression": ("periodic_lognormal_gas", 2_000_000, 4,
                             "periodic isotropic compression: {n} spheres, lognormal r (median 1 mm, sigma 0.3), "
                             "E=1e8, nu=0.25, phi=0.3, damping 0.3, velGrad=-0.01 I, homoDeform 2, dt=0.5*P-wave"),
}


def _workload_spec(name, n, seed=0):
    from paper_2301_00611_amd import scenes
    return getattr(scenes, PERIODIC_WORKLOADS[name][0])(n=n, seed=seed)


def prepare_periodic(name, n, seed=0, target_pressure=1e3, log=None, cache=None):
    """Unmeasured preparation of a periodic workload: its lattice cloud of
    n / tile^3 spheres compressed frictionless (friction 0, same stiffness
    and damping) by a schedule of compressions and velocity resets to a
    jammed packing, settled at a mean stress of -target_pressure by the
    library's isotropic compressor, then replicated tile^3 times into a cell
    tile times wider (the same periodic packing, n spheres).  With `cache`
    (an .npz path) the small packing is loaded from it when present, else
    stored there after preparing it.  Returns the spec of the n-sphere
    workload and its prepared state (positions, velocities, spins, cell)."""
    import numpy as np
    from paper_2301_00611_amd.prepare import jam_isotropic, mean_pressure, settle_iso, tile_periodic
    tile = PERIODIC_WORKLOADS[name][2]
    n0 = n // tile ** 3
    t0 = time.perf_counter()
    if cache and os.path.exists(cache):
        d = np.load(cache)
        if len(d["radius"]) != n0:
            raise ValueError(f"{cache} holds {len(d['radius'])} spheres, the {name} preparation {n0}")
        st = {"pos": d["pos"], "vel": d["vel"], "angvel": d["angvel"]}
        radius, H = d["radius"], d["H"]
        rec = {"loaded_from": cache, "pressure_settled": float(d["pressure"]),
               "coordination_settled": float(d["coordination"]), "solid_fraction": float(d["solid_fraction"])}
    else:
        spec0 = _workload_spec(name, n0, seed)
        radius = spec0.radius
        vs = float((4.0 / 3.0 * math.pi * radius ** 3).sum())
        g = _periodic_scene(spec0.hsize, np.zeros((3, 3)), spec0, spec0.pos, None, None, 0, friction=0.0)
        rec = jam_isotropic(g, spec0.dt_factor * g.pwave_dt(), vs, target_pressure, log=log)
        rec["settle"] = settle_iso(g, target_pressure, log=log)
        g.step(1)
        rec["pressure_settled"] = mean_pressure(g)
        rec["coordination_settled"] = g.stats()["coordination"]
        st = g.get_state()
        H, _ = g.get_cell()
        rec["solid_fraction"] = vs / abs(np.linalg.det(H))
        g.close()
        if cache:
            np.savez(cache, pos=st["pos"], vel=st["vel"], angvel=st["angvel"], radius=radius, H=H,
                     pressure=rec["pressure_settled"], coordination=rec["coordination_settled"],
                     solid_fraction=rec["solid_fraction"])
    pos, rad, vel, ang, H2 = tile_periodic(st["pos"], radius, st["vel"], st["angvel"], H, (tile,) * 3)
    spec = _workload_spec(name, 16, seed)  # parameters of the workload
    spec.pos, spec.radius = pos, rad
    rec["prepared_spheres"] = n0
    rec["tiling"] = [tile] * 3
    rec["cell"] = H2
    rec["seconds"] = time.perf_counter() - t0
    return spec, {"pos": pos, "vel": vel, "angvel": ang}, H2, rec


def _fp32_vs_fp64_one_step(spec, st, H, L):
    """FP32-mixed against FP64 from the identical prepared state: pair-set
    differences, per-contact and per-body force errors."""
    import numpy as np
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
    return err


def dense_run(spec, st, H, L, precision, steps, warmup, timing_steps=1000, probe_steps=100, log=None,
              fixed_tuning=None):
    """One precision on the prepared packing: the autotuner's setting (found
    on a copy of the state, which it advances; or `fixed_tuning`), then
    `warmup` untimed steps and exactly `steps` timed steps on a fresh scene,
    then `timing_steps` more with kernel events (per-kernel durations,
    broad-phase runs)."""
    import torch
    n = len(spec.radius)
    if fixed_tuning:
        tune = dict(fixed_tuning)
    else:
        g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], precision)
        tune = g.autotune(probe_steps=probe_steps)
        g.close()
    tuning = {k: v for k, v in tune.items() if k != "ms_per_step"}
    g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], precision)
    g.set_tuning(**tuning)
    # the initial broad-phase run, timed by itself (it also allocates the
    # scene's buffers; the runs of the timing pass below do not)
    g.set_timing(True)
    g.step(0)
    rb_first_ms = g.get_timing("rebuild")[0]
    g.set_timing(False)
    sa = g.stats()
    if warmup > 0:
        g.step(warmup)
    g.step(0)  # a pending broad-phase run happens here, outside the timed region
    s0 = g.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = g.stats()
    g.set_timing(True)
    g.step(timing_steps)
    kern = {k: g.get_timing(k) for k in ("contact", "integrate", "rebuild")}
    s2 = g.stats()
    g.close()
    c_timed = (s1["contact_steps"] - s0["contact_steps"]) / steps
    c_timing = (s2["contact_steps"] - s1["contact_steps"]) / timing_steps
    # the broad phase: its measured cost per run (the mean of the runs in
    # the timing pass, else the initial run's, which is higher), and its runs
    # per step over all the steps of this scene (warm-up, timed, timing
    # pass); with no run among them the amortised term is an upper bound
    # (one run)
    runs = s2["rebuilds"] - sa["rebuilds"]
    nsteps_all = warmup + steps + timing_steps
    rb_ms = kern["rebuild"][0] if kern["rebuild"][1] > 0 else rb_first_ms
    r = {"value": (s1["contact_steps"] - s0["contact_steps"]) / el, "unit": "contact-steps/s",
         "ms_per_step": el / steps * 1e3, "body_steps_per_s": n * steps / el,
         "rebuilds_timed": s1["rebuilds"] - s0["rebuilds"], "contacts_per_step": c_timed,
         "candidates": s2["n_candidates"], "coordination": s2["coordination"],
         "kernels_ms": {k: v[0] for k, v in kern.items()},
         "kernel_launches": {k: v[1] for k, v in kern.items()},
         "broad_phase": {"ms_per_run": rb_ms, "runs_measured": kern["rebuild"][1], "first_run_ms": rb_first_ms,
                         "runs": runs, "steps": nsteps_all,
                         "amortised_ms_per_step": rb_ms * max(runs, 1) / nsteps_all,
                         "amortised_is_upper_bound": runs == 0},
         "tuning": tune}
    r["ms_per_step_with_amortised_broad_phase"] = r["ms_per_step"] + r["broad_phase"]["amortised_ms_per_step"]
    r["value_with_amortised_broad_phase"] = c_timed / (r["ms_per_step_with_amortised_broad_phase"] * 1e-3)
    rl = {}
    if kern["contact"][0] > 0:
        cb = contact_algorithmic_bytes(precision, n, c_timing, s2["n_candidates"])
        a = cb / (kern["contact"][0] * 1e-3) / 1e9
        rl["contact"] = {"bytes": cb, "achieved_GBs": a, "frac": a / HBM_PEAK_GBS}
    if kern["integrate"][0] > 0:
        ib = INTEGRATE_BYTES_PER_BODY * n
        a = ib / (kern["integrate"][0] * 1e-3) / 1e9
        rl["integrate"] = {"bytes": ib, "achieved_GBs": a, "frac": a / HBM_PEAK_GBS}
    r["rooflines"] = rl
    if log:
        log(f"{'FP64' if precision == 0 else 'FP32-mixed'}: {r}")
    return r


def periodic_leg(name="periodic_compression", steps=2000, warmup=20, n=None, log=None, prepared=None,
                 with_controller=True, with_stats=True, cache=None, fixed_tuning=None):
    """A dense periodic workload (C3: isotropic compression at 0.01/s; C5:
    bidisperse simple shear at 1/s), FP64 vs FP32-mixed on the same prepared
    packing: throughput of each, kernel durations and rooflines, and the
    FP32-mixed error against FP64 from the identical state (pair set,
    per-contact and per-body force) and over the run (energy terms,
    coordination)."""
    import numpy as np
    log = log or (lambda m: None)
    n = n or PERIODIC_WORKLOADS[name][1]
    if prepared is None:
        prepared = prepare_periodic(name, n, log=log, cache=cache)
    spec, st, H, rec = prepared
    n = len(spec.radius)
    L = spec.velgrad
    tile = PERIODIC_WORKLOADS[name][2]
    out = {"workload": PERIODIC_WORKLOADS[name][3].format(n=n)
           + f"; from a packing prepared at {n // tile ** 3} spheres and tiled {tile}x{tile}x{tile}",
           "preparation": _jsonable(rec), "steps": steps}
    out["fp32_vs_fp64_one_step"] = _fp32_vs_fp64_one_step(spec, st, H, L)
    for prec, key in ((0, "fp64"), (1, "fp32_mixed")):
        out[key] = dense_run(spec, st, H, L, prec, steps, warmup, log=log, fixed_tuning=fixed_tuning)
    if with_controller:
        out["controlled_cell"] = controlled_cell_run(H, spec, st, min(steps, 1000), log)
    if with_stats:
        stats = {}
        for prec, key in ((0, "fp64"), (1, "fp32_mixed")):
            g = _periodic_scene(H, L, spec, st["pos"], st["vel"], st["angvel"], prec, track_energy=True)
            rows = []
            win = min(500, steps)
            for _ in range(max(1, steps // win)):
                g.step(win)
                e = g.get_energy()
                rows.append([e["kinetic"], e["kin_rot"], e["elastic"], e["damp_dissip"], e["plastic_dissip"],
                             g.stats()["coordination"]])
            g.close()
            stats[key] = np.array(rows)
        a, b = stats["fp64"], stats["fp32_mixed"]
        scale = np.abs(a[:, :5]).sum(axis=1, keepdims=True)
        out["fp32_vs_fp64_run"] = {
            "energy_terms_rel_to_total_max": float((np.abs(b[:, :5] - a[:, :5]) / scale).max()),
            "coordination_rel_max": float((np.abs(b[:, 5] - a[:, 5]) / np.maximum(a[:, 5], 1e-30)).max()),
            "windows": int(a.shape[0]), "window_steps": min(500, steps)}
    return out


def _jsonable(d):
    out = {}
    for k, v in d.items():
        if isinstance(v, dict):
            out[k] = _jsonable(v)
        elif hasattr(v, "tolist"):
            out[k] = v.tolist()
        elif k != "cell0":
            out[k] = v
    return out


def cpu_model():
    """The host CPU as lscpu names it (model name, sockets x cores x threads),
    else /proc/cpuinfo's model name."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = dict(line.split(":", 1) for line in out.splitlines() if ":" in line)
        f = {k.strip(): v.strip() for k, v in f.items()}
        if "Model name" in f:
            return (f"{f['Model name']} ({f.get('Socket(s)', '?')} sockets x {f.get('Core(s) per socket', '?')} cores x "
                    f"{f.get('Thread(s) per core', '?')} threads, {f.get('CPU(s)', '?')} CPUs visible)")
    except (OSError, subprocess.SubprocessError, ValueError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=5.0, repeats=3, n=4096):
    """The FP64 oracle, one thread, on a bounded sample of the headline
    workload: a periodic cell of the same bidisperse mix (radii 0.5 and 2.0
    mm, equal volumes, same material, damping and shear rate) with n
    spheres, the generator's lattice squeezed by 0.2 % so that neighbours
    overlap (a dense state built without the GPU), stepped for about
    `budget_s` seconds, `repeats` times from the same state; the median
    rate is reported.  Its pair detection is brute force over all pairs and
    27 images, O(N^2)."""
    import numpy as np
    from oracle import OracleScene
    from paper_2301_00611_amd.scenes import periodic_bidisperse_gas
    sc = periodic_bidisperse_gas(n=n, seed=0)
    squeeze = 0.998
    m = sc.material
    rates, body_rates, per_step = [], [], []
    for _ in range(repeats):
        o = OracleScene(dt=1.0, periodic=True, hsize=sc.hsize * squeeze, velgrad=sc.velgrad,
                        damping=sc.damping, gravity=sc.gravity)
        o.add_material(m.density, m.young, m.poisson, m.friction)
        o.add_spheres(sc.pos * squeeze, sc.radius)
        dt = sc.dt_factor * o.pwave_dt()
        o = OracleScene(dt=dt, periodic=True, hsize=sc.hsize * squeeze, velgrad=sc.velgrad,
                        damping=sc.damping, gravity=sc.gravity)
        mo = o.add_material(m.density, m.young, m.poisson, m.friction)
        o.add_spheres(sc.pos * squeeze, sc.radius, default_mat=mo)
        steps, contacts = 0, 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s or steps == 0:
            o.step(1)
            steps += 1
            contacts += len(o.get_contacts())
        t = time.perf_counter() - t0
        rates.append(contacts / t)
        body_rates.append(n * steps / t)
        per_step.append(t / steps)
    return {
        "value": statistics.median(rates),
        "unit": "contact-steps/s",
        "cores": 1,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"periodic cell of the headline's bidisperse mix, {n} spheres (lattice squeezed 0.2 %), "
                   f"stepped ~{budget_s:.0f} s from the same state {repeats} times, median; O(N^2) pairs over "
                   f"27 images: {statistics.median(per_step) * 1e3:.0f} ms/step, "
                   f"{len(o.get_contacts())} contacts at the end"),
        "body_steps_per_s": statistics.median(body_rates),
        "repeats": rates,
        # its pair detection is O(N^2): the same oracle on the 8,000,000
        # spheres of the workload, extrapolated (not measured)
        "extrapolated_s_per_step_at_8M": statistics.median(per_step) * (8_000_000 / n) ** 2,
    }


def copy_bandwidth(nbytes=1 << 30, repeats=5):
    """The GPU's measured streaming bandwidth: a plain device-to-device copy
    of `nbytes` (read + write) timed with device events, best of `repeats`."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / best / 1e9


def parse_tuning(text):
    """--tuning "block_contact,block_integrate,chunk,verlet_factor" -> dict (None: autotune)."""
    if not text:
        return None
    bc, bi, ch, vf = text.split(",")
    return {"block_contact": int(bc), "block_integrate": int(bi), "chunk": int(ch), "verlet_factor": float(vf)}


def headline(args, log):
    """The N=1 line: C5 at FP64 (value), FP32-mixed beside it, the roofline
    of the dominant kernel, the CPU oracle baseline."""
    name = "periodic_shear"
    n = PERIODIC_WORKLOADS[name][1]
    log(f"preparing the {n}-sphere bidisperse packing (not timed)")
    spec, st, H, rec = prepare_periodic(name, n, log=log, cache=args.prepared_state)
    L = spec.velgrad
    log(f"prepared in {rec['seconds']:.1f} s: {_jsonable(rec)}")
    fixed = parse_tuning(args.tuning)
    r64 = dense_run(spec, st, H, L, 0, args.steps, args.warmup, timing_steps=args.timing_steps, log=log,
                    fixed_tuning=fixed)
    kern = r64["kernels_ms"]
    dom = max(("contact", "integrate"), key=lambda k: kern[k])
    rl = r64["rooflines"][dom]
    tile = PERIODIC_WORKLOADS[name][2]
    out = {
        "metric": "contact-steps/s",
        "value": r64["value"],
        "unit": "contact-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": PERIODIC_WORKLOADS[name][3].format(n=len(spec.radius))
                   + f"; dense packing prepared at 1 kPa ({n // tile ** 3} spheres, tiled {tile}x{tile}x{tile})",
                   "n_spheres": len(spec.radius), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_" + dom, "achieved": rl["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": rl["frac"],
                     "traffic": profiled_traffic("k_" + dom, "traffic_periodic_shear_8m"),
                     "algorithmic_bytes_per_launch": rl["bytes"]},
        "body_steps_per_s": r64["body_steps_per_s"],
        "contacts_per_step": r64["contacts_per_step"],
        "coordination": r64["coordination"],
        "candidates": r64["candidates"],
        "kernels_ms": kern,
        "rooflines": r64["rooflines"],
        "broad_phase": r64["broad_phase"],
        "ms_per_step_with_amortised_broad_phase": r64["ms_per_step_with_amortised_broad_phase"],
        "value_with_amortised_broad_phase": r64["value_with_amortised_broad_phase"],
        "tuning": r64["tuning"],
        "preparation": _jsonable(rec),
    }
    # the same kernel against what a plain copy reaches on this GPU
    cb = copy_bandwidth()
    out["roofline"]["copy_GBs"] = cb
    out["roofline"]["frac_of_copy"] = rl["achieved_GBs"] / cb
    if args.fp64_only:
        return out
    log("FP32-mixed on the same packing")
    r32 = dense_run(spec, st, H, L, 1, args.steps, args.warmup, timing_steps=args.timing_steps, log=log,
                    fixed_tuning=fixed)
    out["fp32_mixed"] = r32
    out["fp32_vs_fp64_one_step"] = _fp32_vs_fp64_one_step(spec, st, H, L)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads' legs (with --workload: the leg's sub-runs: controlled cell, "
                         "error statistics, the batch's sequential reference)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-only", action="store_true", help="headline: skip the FP32-mixed leg (profiling runs)")
    ap.add_argument("--timing-steps", type=int, default=1000,
                    help="steps of the pass with kernel events after the timed steps")
    ap.add_argument("--workload", default="headline",
                    choices=("headline", "column", "periodic_compression", "periodic_shear", "batched",
                             "facet_column", "viscel_column"),
                    help="headline: the N=1 line (default); the others run one leg alone")
    ap.add_argument("--prepared-state", default=None,
                    help="headline and periodic legs: .npz holding the prepared packing before it is tiled (loaded "
                         "if present, else written), so that profiled runs skip the preparation")
    ap.add_argument("--tuning", default=None,
                    help="headline and periodic legs: a fixed launch setting "
                         "'block_contact,block_integrate,chunk,verlet_factor' in place of the autotuner's (profiling runs)")
    ap.add_argument("--tuning-cache", default=None,
                    help="autotuner cache file for the column legs: reuse a stored setting, or store the one found")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy three times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs a scene on one GPU; --gpus {args.gpus} is not supported "
              "(the decomposition over several GPUs is a design note only)", file=sys.stderr)
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
        out = periodic_leg(args.workload, steps=args.steps, warmup=args.warmup, log=log,
                           with_controller=not args.no_extra, with_stats=not args.no_extra,
                           cache=args.prepared_state, fixed_tuning=parse_tuning(args.tuning))
        print(json.dumps(out), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(batched_leg(steps=args.steps, log=log, sequential=not args.no_extra)), flush=True)
        return
    if args.workload == "column":
        print(json.dumps(column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)), flush=True)
        return
    if args.workload == "facet_column":
        print(json.dumps(facet_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)), flush=True)
        return
    if args.workload == "viscel_column":
        print(json.dumps(viscel_column_leg(args.steps, args.warmup, log=log, cache=args.tuning_cache)), flush=True)
        return

    out = headline(args, log)
    if not args.no_extra:
        log("periodic compression leg (2 M spheres at 1 kPa, FP64 vs FP32-mixed)")
        out["periodic_compression"] = periodic_leg("periodic_compression", steps=1000, warmup=20, log=log,
                                                   with_stats=False)
        log("column leg (200,000 spheres, deposition)")
        out["column"] = column_leg(2000, 20, log=log)
        log("batched leg")
        out["batched"] = batched_leg(steps=1000, log=log)
        log("facet-box column leg")
        out["facet_column"] = facet_column_leg(2000, 20, log=log)
        log("visco-elastic column leg")
        out["viscel_column"] = viscel_column_leg(2000, 20, log=log)
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def column_leg(steps, warmup, log=None, cache=None):
    """The 200,000-sphere deposition column (C2) in FP64 and FP32-mixed:
    `steps` steps from the initial state (few contacts: the bottom layer on
    the floor), the integrate kernel's roofline."""
    from paper_2301_00611_amd.scenes import grid_column
    spec = grid_column(n=200_000, seed=0)
    out = {"workload": "grid_column deposition: 200,000 spheres r~U(0.5,1.5) mm, 0.1x0.1 m box with floor, "
                       "E=5e7, nu=0.3, phi=0.5, damping 0.2, dt=0.5*P-wave", "steps": steps}
    for prec, key in ((0, "fp64"), (1, "fp32_mixed")):
        tune = autotune_for(spec, prec, warmup=warmup, cache=cache)
        r = timed_run(spec, steps, warmup, precision=prec, tuning=tune)
        rt = timed_run(spec, steps, 0, precision=prec, timing=True, tuning=tune)
        kern = {k: v["avg_ms"] for k, v in rt["kernels"].items()}
        ib = INTEGRATE_BYTES_PER_BODY * spec.n
        out[key] = {"value": r["contact_steps"] / r["seconds"], "unit": "contact-steps/s",
                    "ms_per_step": r["seconds"] / steps * 1e3, "body_steps_per_s": spec.n * steps / r["seconds"],
                    "rebuilds": r["rebuilds"], "tuning": tune, "kernels_ms": kern,
                    "integrate_roofline": {"bytes": ib, "frac": ib / (kern["integrate"] * 1e-3) / 1e9 / HBM_PEAK_GBS}}
        if log:
            log(f"column {key}: {out[key]}")
    return out


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
    b.step(0)  # a pending broad-phase run, outside the timed region
    s0 = b.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s1 = b.stats()
    return t, s1["contact_steps"] - s0["contact_steps"], s1["rebuilds"] - s0["rebuilds"]


def _batch_kernels(b, steps):
    """Per-kernel durations of `steps` more batch steps with kernel events."""
    v = b.scene(0)
    v.set_timing(True)
    b.step(steps)
    out = {k: v.get_timing(k)[0] for k in ("contact", "integrate", "rebuild")}
    v.set_timing(False)
    return out


def batched_leg(n_scenes=512, steps=2000, sequential_steps=None, log=None, sequential=True):
    """C4: 512 independent deposition scenes (log-uniform sizes 500..50,000,
    per-scene friction and damping) stepped together, FP64 and FP32-mixed:
    scene-steps/s with the default launch setting and with the autotuner's
    (its probe steps are not timed), the kernel durations and the integrate
    kernel's roofline, against the same scenes stepped one after another as
    single FP64 scenes (`sequential_steps` steps each, by default as many as
    the batch)."""
    sequential_steps = sequential_steps or steps
    from paper_2301_00611_amd import dem
    from paper_2301_00611_amd.scenes import batched_deposition
    log = log or (lambda m: None)
    spec = batched_deposition(n_scenes=n_scenes, steps=steps)
    dt = 0.5 * spec.dt_radius * math.sqrt(2600.0 / 5e7)
    nbodies = sum(s.n for s in spec.scenes)
    out = {"unit": "scene-steps/s", "n_scenes": n_scenes, "n_spheres": nbodies, "steps": steps}
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        b = _build_batch(spec, dt, prec)
        t_def, c_def, _ = _time_batch(b, steps)
        tune = b.autotune(probe_steps=100)
        t_tun, c_tun, runs = _time_batch(b, steps)
        kern = _batch_kernels(b, min(steps, 500))
        b.close()
        ib = INTEGRATE_BYTES_PER_BODY * nbodies
        out[name] = {"value": n_scenes * steps / t_tun, "seconds": t_tun, "body_steps_per_s": nbodies * steps / t_tun,
                     "contact_steps_per_s": c_tun / t_tun, "default_setting_value": n_scenes * steps / t_def,
                     "tuning": tune, "kernels_ms": kern, "broad_phase_runs_timed": runs,
                     "integrate_roofline": {"bytes": ib, "frac": (ib / (kern["integrate"] * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                                  if kern["integrate"] > 0 else None)}}
        log(f"batched {name}: {out[name]}")
    out["value"] = out["fp64"]["value"]
    if not sequential:
        return out
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
        g.step(0)
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
