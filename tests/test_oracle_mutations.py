"""The oracle's pins must catch plausible slips.

Each case applies one deliberate mistake to a private copy of the oracle's
C source (a dropped term, a flipped sign, a wrong factor), builds it, and
runs the pin tests against that build: at least one pin must fail.  The
mistakes are planted in the oracle on the CPU only.  The builds and pin
runs of a table go on a few workers at once, the first time one of its
cases is asked for; each case then reports its own result.
"""
import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dem_oracle.c")
WORKERS = max(1, min(8, os.cpu_count() or 1))


def _run_c_mutant(name, before, after, pins, workdir):
    """Build the oracle with one planted slip and run a pin file against it,
    stopping at the first failure: (exit status, end of the output), or
    (None, message) when the slip's anchor is not found exactly once."""
    src = open(SRC).read()
    if src.count(before) != 1:
        return None, f"mutation anchor not found: {name}"
    d = os.path.join(workdir, name)
    os.makedirs(d, exist_ok=True)
    mutated = os.path.join(d, "dem_oracle_mutated.c")
    with open(mutated, "w") as f:
        f.write(src.replace(before, after))
    lib = os.path.join(d, "libdem_oracle_mutated.so")
    subprocess.run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "oracle"), "-o", lib, mutated, "-lm"], check=True)
    env = dict(os.environ, DEM_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", pins],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=900)
    return r.returncode, r.stdout[-2000:]


def _run_all(table, run_one):
    """Every slip of a table, run_one(name, before, after) on a few workers."""
    with ThreadPoolExecutor(WORKERS) as ex:
        futures = {name: ex.submit(run_one, name, *table[name]) for name in table}
    return {name: f.result() for name, f in futures.items()}


def _c_results(table, pin_file, tmp_path_factory):
    pins = os.path.join(ROOT, "tests", pin_file)
    work = str(tmp_path_factory.mktemp("mutants"))
    return _run_all(table, lambda name, before, after: _run_c_mutant(name, before, after, pins, work))


def _assert_caught(name, result):
    rc, out = result
    assert rc is not None, out
    assert rc != 0 and "FAILED" in out, f"no pin caught mutation {name} (exit {rc}):\n{out}"

MUTATIONS = {
    "drop_twist_term": ("cross3(fs_old, spinv, inc2);", "inc2[0] = inc2[1] = inc2[2] = 0.0;"),
    "drop_plane_rotation": ("cross3(fs_old, rot, inc1);", "inc1[0] = inc1[1] = inc1[2] = 0.0;"),
    "drop_ratcheting_factor": ("alpha = (R1 + R2) / l;", "alpha = 1.0;"),
    "shear_increment_sign": ("- ks * dt * vs[k];", "+ ks * dt * vs[k];"),
    "torque_branch_of_2": ("cross3(br2, f2, ct->t2);", "cross3(br1, f2, ct->t2);"),
    "normal_force_sign": ("fn[k] = fn_mag * n[k];", "fn[k] = -fn_mag * n[k];"),
    "damping_without_half_step": ("(v0[k] + a * dt / 2.0)", "(v0[k])"),
    "rotdamp_without_half_step": ("(b->w[k] + a * dt / 2.0)", "(b->w[k])"),
    "rotdamp_work_dropped": ("en->damp += -dtq * b->w[k] * dt;", ""),
    "damping_excludes_gravity": ("f[k] = F_in[k] + b->m * s->p.gravity[k];", "f[k] = F_in[k];"),
    "elastic_energy_factor": ("*e_el += 0.5 * (fn_mag * fn_mag / kn)", "*e_el += 1.0 * (fn_mag * fn_mag / kn)"),
    "no_image_velocity": ("for (int k = 0; k < 3; ++k) v2[k] += sv[k] / dt;", ""),
    "no_convective_term": ("(s->p.homo_deform == 2 ? a2[k] * dt : 0.0)", "0.0"),
    "kinetic_energy_missing": ("en->kin = 0.5 * b->m * dot3(b->v, b->v);", "en->kin = 0.0;"),
    "inertia_rounding": ("b->I = 2.0 * b->m * r * r / 5.0;", "b->I = 0.4 * b->m * r * r;"),
    "shear_stiffness_without_poisson": ("double s1 = (m1->young * m1->poisson) * (2.0 * R1);",
                                        "double s1 = (m1->young) * (2.0 * R1);"),
    "friction_max_not_min": ("return tan(m1->friction < m2->friction ? m1->friction : m2->friction);",
                             "return tan(m1->friction > m2->friction ? m1->friction : m2->friction);"),
    "wall_reference_radius": ("n[w->axis] = (double)wall_sign(w, sp);\n        *R1 = sp->r;",
                              "n[w->axis] = (double)wall_sign(w, sp);\n        *R1 = 0.5 * sp->r;"),
    "plastic_work_without_fmax": ("*e_plast += (fs_norm - fmax) * fmax / ks;", "*e_plast += (fs_norm - fmax) / ks;"),
    "nearest_image_only": ("    for (int a = -1; a <= 1; ++a)\n        for (int b = -1; b <= 1; ++b)\n            for (int g = -1; g <= 1; ++g) {",
                           "    for (int a = 0; a <= 0; ++a)\n        for (int b = 0; b <= 0; ++b)\n            for (int g = 0; g <= 0; ++g) {"),
    "spin_radii_swapped": ("rw[k] = R2 * w2[k] + R1 * w1[k];", "rw[k] = R1 * w2[k] + R2 * w1[k];"),
    "cell_update_on_the_right": ("matmul(M, s->H, s->H);", "matmul(s->H, M, s->H);"),
    "normal_stiffness_arithmetic_mean": ("*kn = k1 * k2 / (k1 + k2);", "*kn = 0.25 * (k1 + k2);"),
    "shear_stiffness_from_one_material": ("*ks = s1 * s2 / (s1 + s2);", "*ks = *kn * m1->poisson;"),
    "plastic_work_at_trial_force": ("*e_plast += (fs_norm - fmax) * fmax / ks;",
                                    "*e_plast += (fs_norm - fmax) * fs_norm / ks;"),
    "shear_energy_with_kn": ("*e_el += 0.5 * (fn_mag * fn_mag / kn) + 0.5 * (dot3(fs, fs) / ks);",
                             "*e_el += 0.5 * (fn_mag * fn_mag / kn) + 0.5 * (dot3(fs, fs) / kn);"),
    "shear_energy_factor": ("*e_el += 0.5 * (fn_mag * fn_mag / kn) + 0.5 * (dot3(fs, fs) / ks);",
                            "*e_el += 0.5 * (fn_mag * fn_mag / kn) + 1.0 * (dot3(fs, fs) / ks);"),
    "wall_position_sign": ("    double delta = sp->x[w->axis] - w->wpos;\n    if (!(fabs(delta) < sp->r)) return 0;",
                           "    double delta = sp->x[w->axis] + w->wpos;\n    if (!(fabs(delta) < sp->r)) return 0;"),
    "damping_estimate_a_whole_step": ("(v0[k] + a * dt / 2.0)", "(v0[k] + a * dt / 1.0)"),
    "rotdamp_estimate_a_whole_step": ("(b->w[k] + a * dt / 2.0)", "(b->w[k] + a * dt / 1.0)"),
    "twist_spin_component_subtracted": ("double wsum[3] = {w1[0] + w2[0], w1[1] + w2[1], w1[2] + w2[2]};",
                                        "double wsum[3] = {w1[0] + w2[0], w1[1] - w2[1], w1[2] + w2[2]};"),
    "cell_volume_third_cofactor_multiplier": ("                 H[2] * (H[3] * H[7] - H[4] * H[6]));",
                                              "                 H[0] * (H[3] * H[7] - H[4] * H[6]));"),
    "cell_volume_cofactor_sign": ("V = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1]",
                                  "V = fabs(H[0] * (H[4] * H[8] + H[5] * H[7]) - H[1]"),
    "contact_point_on_the_first_surface": ("for (int k = 0; k < 3; ++k) pt[k] = b1->x[k] + (R1 - 0.5 * pen) * n[k];",
                                           "for (int k = 0; k < 3; ++k) pt[k] = b1->x[k] + R1 * n[k];"),
    "wall_contact_point_on_the_sphere": ("for (int k = 0; k < 3; ++k) pt[k] = b2->x[k] - (b2->r - 0.5 * pen) * n[k];",
                                         "for (int k = 0; k < 3; ++k) pt[k] = b2->x[k] - b2->r * n[k];"),
    "rotation_composed_on_the_right": ("        qmul(dq, b->q, q);", "        qmul(b->q, dq, q);"),
    "pwave_step_of_the_first_material": ("        const mat_t* m = &s->mats[b->mat];\n        double dt = b->r / sqrt(m->young / m->density);",
                                         "        const mat_t* m = &s->mats[0];\n        double dt = b->r / sqrt(m->young / m->density);"),
    "rotation_angle_doubled": ("double half = 0.5 * wn * dt;", "double half = wn * dt;"),
    "overlap_dependent_branch": ("rw[k] = R2 * w2[k] + R1 * w1[k];",
                                 "rw[k] = (R2 - 0.5 * pen) * w2[k] + (R1 - 0.5 * pen) * w1[k];"),
    "stress_transposed": ("acc[3 * i + j] += ct->f2[i] * (-ct->det_d[j]);",
                          "acc[3 * i + j] += ct->f2[j] * (-ct->det_d[i]);"),
    "stress_volume_signed": ("        V = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +",
                             "        V = (H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +"),
    "stress_volume_from_the_diagonal": ("        V = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +\n"
                                        "                 H[2] * (H[3] * H[7] - H[4] * H[6]));",
                                        "        V = H[0] * H[4] * H[8];"),
    "stress_branch_sign": ("acc[3 * i + j] += ct->f2[i] * (-ct->det_d[j]);",
                           "acc[3 * i + j] += ct->f2[i] * (ct->det_d[j]);"),
    "gravity_work_sign": ("en->grav += -b->m * s->p.gravity[k] * v0[k] * dt;",
                          "en->grav += b->m * s->p.gravity[k] * v0[k] * dt;"),
}


@pytest.fixture(scope="module")
def pins_results(tmp_path_factory):
    return _c_results(MUTATIONS, "test_oracle_pins.py", tmp_path_factory)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, pins_results):
    _assert_caught(name, pins_results[name])


# slips in the box and facet boundaries, caught by tests/test_oracle_boundaries.py
BOUNDARY_MUTATIONS = {
    "facet_reference_radius": ("*R1 = 2.0 * sp->r;", "*R1 = sp->r;"),
    "box_inside_overlap": ("*pen = sp->r + depth;", "*pen = sp->r - depth;"),
    "box_edge_as_two_planes": ("if (!(dist < sp->r)) return 0;\n            for (int k = 0; k < 3; ++k) n[k] = d[k] / dist;",
                               "if (!(dist < sp->r * 1.5)) return 0;\n            for (int k = 0; k < 3; ++k) n[k] = d[k] / dist;"),
    "facet_edge_clamp": ("if (t > 1.0) t = 1.0;", ""),
    "facet_one_sided": ("if (dot3(c, nn) < 0.0) inside = 0;", "if (dot3(c, nn) > 0.0) inside = 0;"),
    "triangle_edges_from_the_origin": ("        e1[k] = v[1][k] - v[0][k];\n        e2[k] = v[2][k] - v[0][k];",
                                       "        e1[k] = v[1][k] + v[0][k];\n        e2[k] = v[2][k] + v[0][k];"),
    "triangle_plane_height_sign": ("double h = (x[0] - v[0][0]) * nn[0] + (x[1] - v[0][1]) * nn[1]",
                                   "double h = (x[0] - v[0][0]) * nn[0] - (x[1] - v[0][1]) * nn[1]"),
    "facet_closest_point_vector": ("    closest_on_triangle(w->fv, sp->x, p);\n    double d[3] = {sp->x[0] - p[0], sp->x[1] - p[1], sp->x[2] - p[2]};",
                                   "    closest_on_triangle(w->fv, sp->x, p);\n    double d[3] = {sp->x[0] - p[0], sp->x[1] - p[1], sp->x[2] + p[2]};"),
    "box_inside_low_face_pushed_inwards": ("                depth = dl;\n                ax = k;\n                sg = -1;",
                                           "                depth = dl;\n                ax = k;\n                sg = 1;"),
    "segment_lower_clamp_dropped": ("    if (t < 0.0) t = 0.0;\n", ""),
    "triangle_inside_test_two_edges": ("    for (int i = 0; i < 3; ++i) {\n        const double* a = v[i];",
                                       "    for (int i = 0; i < 2; ++i) {\n        const double* a = v[i];"),
    "facet_face_normal_reversed": ("        cross3(e1, e2, n);\n        double len = sqrt(dot3(n, n));",
                                   "        cross3(e2, e1, n);\n        double len = sqrt(dot3(n, n));"),
}


@pytest.fixture(scope="module")
def boundary_results(tmp_path_factory):
    return _c_results(BOUNDARY_MUTATIONS, "test_oracle_boundaries.py", tmp_path_factory)


@pytest.mark.parametrize("name", sorted(BOUNDARY_MUTATIONS))
def test_boundary_pins_catch_mutation(name, boundary_results):
    _assert_caught(name, boundary_results[name])


# slips in the visco-elastic law, caught by tests/test_oracle_viscel.py
VISCEL_MUTATIONS = {
    "viscel_sphere_mass_not_reduced": ("double m = b1->m * b2->m / (b1->m + b2->m);", "double m = b2->m;"),
    "viscel_fixed_sphere_mass": ("if (fixed2 && !fixed1) m = b1->m;", ""),
    "viscel_tangential_without_two_sevenths": ("*ks = 2.0 / 7.0 * m * (pi * pi + let * let) / (tc * tc);",
                                               "*ks = m * (pi * pi + let * let) / (tc * tc);"),
    "viscel_normal_dashpot_sign": ("fn_mag = kn * pen - cn * un;", "fn_mag = kn * pen + cn * un;"),
    "viscel_dashpot_work_halved": ("*e_visc += (cn * un * un", "*e_visc += (0.5 * cn * un * un"),
    "viscel_shear_dashpot_dropped": ("fsv[k] = -cs * vs[k];", "fsv[k] = 0.0 * vs[k];"),
    "viscel_tension_cut_off": ("double fmax = (fn_mag > 0.0 ? fn_mag : 0.0) * tanphi;",
                               "if (fn_mag < 0.0) fn_mag = 0.0;\n        double fmax = fn_mag * tanphi;"),
    "viscel_restitution_product": ("double len = log(0.5 * (m1->en + m2->en));",
                                   "double len = log(m1->en * m2->en);"),
    "viscel_contact_time_max": ("double tc = 0.5 * (m1->tc + m2->tc);",
                                "double tc = (m1->tc > m2->tc ? m1->tc : m2->tc);"),
    "viscel_shear_dashpot_while_sliding": ("        if (!slide)\n            for (int k = 0; k < 3; ++k) fsv[k] = -cs * vs[k];",
                                           "        for (int k = 0; k < 3; ++k) fsv[k] = -cs * vs[k];"),
    "viscel_shear_dashpot_work_dropped": ("(slide ? 0.0 : cs * dot3(vs, vs))", "0.0"),
}


@pytest.fixture(scope="module")
def viscel_results(tmp_path_factory):
    return _c_results(VISCEL_MUTATIONS, "test_oracle_viscel.py", tmp_path_factory)


@pytest.mark.parametrize("name", sorted(VISCEL_MUTATIONS))
def test_viscel_pins_catch_mutation(name, viscel_results):
    _assert_caught(name, viscel_results[name])


# slips in the controllers (oracle/controls.py, Python), caught by
# tests/test_oracle_controls.py: the mutated source is executed into the
# module in a child process before the pins are collected there
CONTROL_MUTATIONS = {
    "control_no_grow_damping": ("rate = (1.0 - self.grow_damping) * err / (M[i] * T)",
                                "rate = err / (M[i] * T)"),
    "control_period_without_interval": ("T = self.glob_update * sc.dt", "T = sc.dt"),
    "control_linear_strain": ("self.strain[i] = math.log(float(trsf[i, i]))",
                              "self.strain[i] = float(trsf[i, i]) - 1.0"),
    "control_goal_ignores_unbalanced": ("        if not (self.unbalanced <= self.max_unbalanced):\n"
                                        "            reached = False\n", ""),
    "control_tolerance_min": ("if abs(err) > max(self.abs_tol, self.rel_tol * abs(self.goal[i])):",
                              "if abs(err) > min(self.abs_tol, self.rel_tol * abs(self.goal[i])):"),
    "control_strain_tolerance_inverted": ("                if abs(err) > STRAIN_TOL:", "                if abs(err) < STRAIN_TOL:"),
    "control_strain_tolerance_without_abs": ("                if abs(err) > STRAIN_TOL:", "                if (err) > STRAIN_TOL:"),
    "control_rate_not_capped": ("rates[i] = max(-self.max_rate[i], min(self.max_rate[i], rate))",
                                "rates[i] = rate"),
    "modulus_branch_not_squared": ('M[i] += float(c["kn"]) * (di * ni) * (di * ni)',
                                   'M[i] += float(c["kn"]) * (di * ni)'),
    "iso_modulus_sum_not_mean": ("self.stiff = (M[0] + M[1] + M[2]) / 3.0", "self.stiff = (M[0] + M[1] + M[2])"),
    "iso_tolerance_min": ("return (abs(goal - self.sigma) <= max(self.abs_tol, self.rel_tol * abs(goal))",
                          "return (abs(goal - self.sigma) <= min(self.abs_tol, self.rel_tol * abs(goal))"),
    "iso_next_stress_a_period_late": ("        if reached and self.state + 1 < len(self.stresses):\n"
                                      "            self.state += 1\n            reached = False\n",
                                      "        if reached and self.state + 1 < len(self.stresses):\n"
                                      "            self.state += 1\n            reached = False\n"
                                      "            self.done = False\n            self.strain_rate = 0.0\n"
                                      "            sc.set_velgrad(np.eye(3) * 0.0)\n            self.updates += 1\n"
                                      "            return\n"),
    "unbalanced_always_max": ("top = max(body) if use_max else sum(body) / len(body)", "top = max(body)"),
    "unbalanced_counts_blocked": ("if sc.is_wall[i] or sc.blocked[i] == 63:", "if sc.is_wall[i]:"),
    "stiffness_dt_without_sqrt2": ("best = min(best, math.sqrt(2.0) * math.sqrt(m[b] / K[b][i]))",
                                   "best = min(best, math.sqrt(m[b] / K[b][i]))"),
    "stiffness_without_tangential_term": ("K[body][i] += (kn - ks) * nv[i] * nv[i] + ks",
                                          "K[body][i] += kn * nv[i] * nv[i]"),
    "rotational_stiffness_without_lever": ("R[body][i] += ks * r * r * (1.0 - nv[i] * nv[i])",
                                           "R[body][i] += ks * (1.0 - nv[i] * nv[i])"),
}

_CONTROL_DRIVER = """
import json, sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle.controls as C
before, after = json.loads(sys.argv[1])
src = open(C.__file__).read()
exec(compile(src.replace(before, after), C.__file__, "exec"), C.__dict__)
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", {pins!r}]))
"""


def _run_control_mutant(name, before, after, workdir):
    src = open(os.path.join(ROOT, "oracle", "controls.py")).read()
    if src.count(before) != 1:
        return None, f"mutation anchor not found: {name}"
    driver = os.path.join(workdir, name + "_driver.py")
    with open(driver, "w") as f:
        f.write(_CONTROL_DRIVER.format(root=ROOT, tests=os.path.join(ROOT, "tests"),
                                       pins=os.path.join(ROOT, "tests", "test_oracle_controls.py")))
    r = subprocess.run([sys.executable, driver, json.dumps([before, after])], capture_output=True, text=True,
                       cwd=workdir, timeout=900)
    # 1: the pins ran and one failed (not a crash of the harness)
    return (r.returncode if r.returncode in (0, 1) else None), r.stdout[-2000:] + r.stderr[-500:]


@pytest.fixture(scope="module")
def control_results(tmp_path_factory):
    work = str(tmp_path_factory.mktemp("control_mutants"))
    return _run_all(CONTROL_MUTATIONS, lambda name, before, after: _run_control_mutant(name, before, after, work))


@pytest.mark.parametrize("name", sorted(CONTROL_MUTATIONS))
def test_control_pins_catch_mutation(name, control_results):
    _assert_caught(name, control_results[name])
