"""Oracle versions of the quantities and controllers around the timestep:
unbalanced force, the stiffness-based critical timestep and the
stress/strain-controlled periodic cell (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library.  Everything here is computed in plain
Python/NumPy (FP64) from what the C oracle reports after a step (resultant
forces, contact records, masses, the cell), in the order the documentation
describes.

Readings of the documentation (each is listed in the design notes):
  * unbalanced force (utils.unbalancedForce, section 5 utility reference):
    mean (or largest) magnitude of the resultant contact force over the
    dynamic spheres (a sphere with all six DOFs blocked is not dynamic;
    walls are not dynamic; gravity is not part of the resultant), divided
    by the mean of |F_n + F_s| over the real contacts.  NaN when either set
    is empty.
  * stiffness timestep (GlobalStiffnessTimeStepper, section 2.2.x, eqs.
    2.12-2.14): per dynamic sphere the diagonal of its translational
    stiffness, K_ii = sum over its contacts of (k_n - k_s) n_i^2 + k_s
    (eq. 2.14), and of its rotational stiffness, R_ii = sum of
    k_s r^2 (1 - n_i^2) (a tangential spring at lever arm r, the sphere's
    radius); each unblocked DOF with positive stiffness gives
    sqrt(2) sqrt(m / K_ii) (eq. 2.12; I / R_ii for rotations); the timestep
    is the safety factor times the smallest of these.  Without any contact
    it is the safety factor times the P-wave timestep.
  * stress/strain-controlled cell (PeriTriaxController with the packing
    stiffness, dynCell off): every `glob_update` steps, from the stress of
    the last step's contacts and the modulus M_i = (1/V) sum over
    sphere-sphere contacts of k_n (d_i n_i)^2 (d the centre distance
    vector; the stress change per unit strain of the normal springs), each
    stress axis gets the strain rate (1 - grow_damping) (goal_i - sigma_ii) /
    (M_i T), T = glob_update * dt (the full rate towards the goal's sign
    when M_i = 0), each strain axis (strain = log of the cell
    transformation's diagonal) the rate (goal_i - strain_i) / T; rates are
    capped at max_strain_rate; the velocity gradient is diag(rates).  The
    goal is reached when every stress axis is within
    max(abs_stress_tol, rel_stress_tol |goal_i|), every strain axis within
    1e-6, and the unbalanced force at most max_unbalanced; the cell then
    stops (zero velocity gradient).
"""
from __future__ import annotations

import math

import numpy as np

STRAIN_TOL = 1e-6


def unbalanced_force(sc, use_max=False):
    """utils.unbalancedForce of an oracle scene after a step."""
    st = sc.get_state()
    body = []
    for i in range(sc.num_bodies):
        if sc.is_wall[i] or sc.blocked[i] == 63:
            continue
        f = st["force"][i]
        body.append(math.sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]))
    contacts = sc.get_contacts()
    cf = []
    for c in contacts:
        f = np.asarray(c["fn"]) + np.asarray(c["fs"])
        cf.append(math.sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]))
    if not body or not cf:
        return float("nan")
    mean_contact = sum(cf) / len(cf)
    top = max(body) if use_max else sum(body) / len(body)
    return top / mean_contact


def stiffness_dt(sc, safety=0.8):
    """GlobalStiffnessTimeStepper's timestep from the last step's contacts."""
    n = sc.num_bodies
    m, inertia = sc.get_mass()
    K = [[0.0, 0.0, 0.0] for _ in range(n)]
    R = [[0.0, 0.0, 0.0] for _ in range(n)]
    for c in sc.get_contacts():
        nv = [float(x) for x in c["normal"]]
        kn, ks = float(c["kn"]), float(c["ks"])
        for body in (int(c["id1"]), int(c["id2"])):
            if sc.is_wall[body]:
                continue
            r = sc.radius[body]
            for i in range(3):
                K[body][i] += (kn - ks) * nv[i] * nv[i] + ks
                R[body][i] += ks * r * r * (1.0 - nv[i] * nv[i])
    best = math.inf
    for b in range(n):
        if sc.is_wall[b] or sc.blocked[b] == 63:
            continue
        for i in range(3):
            if not (sc.blocked[b] & (1 << i)) and K[b][i] > 0.0:
                best = min(best, math.sqrt(2.0) * math.sqrt(m[b] / K[b][i]))
            if not (sc.blocked[b] & (8 << i)) and R[b][i] > 0.0:
                best = min(best, math.sqrt(2.0) * math.sqrt(inertia[b] / R[b][i]))
    if math.isinf(best):
        return safety * sc.pwave_dt()
    return safety * best


def contact_modulus(sc, volume):
    """M_i = (1/V) sum over sphere-sphere contacts of k_n (d_i n_i)^2."""
    M = [0.0, 0.0, 0.0]
    for c in sc.get_contacts():
        if c["is_wall"]:
            continue
        a, b = int(c["id1"]), int(c["id2"])
        dist = (sc.radius[a] + sc.radius[b]) - float(c["pen"])
        for i in range(3):
            ni = float(c["normal"][i])
            di = dist * ni
            M[i] += float(c["kn"]) * (di * ni) * (di * ni)
    return [x / volume for x in M]


class PeriTriax:
    """The stress/strain-controlled periodic cell driving an oracle scene."""

    def __init__(self, sc, goal, stress_mask, glob_update=5, max_strain_rate=(1.0, 1.0, 1.0),
                 grow_damping=0.25, max_unbalanced=1e-4, abs_stress_tol=1e3, rel_stress_tol=3e-5):
        self.sc = sc
        self.goal = [float(g) for g in goal]
        self.mask = int(stress_mask)
        self.glob_update = int(glob_update)
        self.max_rate = [float(r) for r in max_strain_rate]
        self.grow_damping = float(grow_damping)
        self.max_unbalanced = float(max_unbalanced)
        self.abs_tol = float(abs_stress_tol)
        self.rel_tol = float(rel_stress_tol)
        self.stress = [0.0, 0.0, 0.0]
        self.strain = [0.0, 0.0, 0.0]
        self.strain_rate = [0.0, 0.0, 0.0]
        self.stiff = [0.0, 0.0, 0.0]
        self.unbalanced = float("nan")
        self.updates = 0
        self.done = False

    def update(self):
        sc = self.sc
        H, trsf = sc.get_cell()
        V = abs(float(np.linalg.det(H)))
        sigma = sc.get_stress(V)
        M = contact_modulus(sc, V)
        T = self.glob_update * sc.dt
        rates = [0.0, 0.0, 0.0]
        reached = True
        for i in range(3):
            self.stress[i] = float(sigma[i, i])
            self.strain[i] = math.log(float(trsf[i, i]))
            self.stiff[i] = M[i]
            if self.mask & (1 << i):
                err = self.goal[i] - self.stress[i]
                if M[i] > 0.0:
                    rate = (1.0 - self.grow_damping) * err / (M[i] * T)
                else:
                    rate = math.copysign(self.max_rate[i], err) if err != 0.0 else 0.0
                if abs(err) > max(self.abs_tol, self.rel_tol * abs(self.goal[i])):
                    reached = False
            else:
                err = self.goal[i] - self.strain[i]
                rate = err / T
                if abs(err) > STRAIN_TOL:
                    reached = False
            rates[i] = max(-self.max_rate[i], min(self.max_rate[i], rate))
        self.unbalanced = unbalanced_force(sc)
        if not (self.unbalanced <= self.max_unbalanced):
            reached = False
        self.done = reached
        if reached:
            rates = [0.0, 0.0, 0.0]
        self.strain_rate = rates
        sc.set_velgrad(np.diag(rates))
        self.updates += 1

    def run(self, nsteps, stop_when_done=False):
        """Step one at a time; after every step that makes the iteration
        count a multiple of glob_update, update the cell.  Returns the number
        of steps run."""
        done_steps = 0
        for _ in range(int(nsteps)):
            self.sc.step(1)
            done_steps += 1
            it, _t = self.sc.counters()
            if it % self.glob_update == 0:
                self.update()
                if self.done and stop_when_done:
                    break
        return done_steps


class PeriIsoCompressor:
    """Isotropic compression of a periodic cell through a series of mean
    stresses (PeriIsoCompressor with keepProportions): after every
    global_update_int-th step the mean stress sigma_m = tr(sigma)/3 and the
    mean normal-spring modulus M_m = (M_1 + M_2 + M_3)/3 (contact_modulus)
    give one strain rate for all three axes,
        (1 - grow_damping)(goal - sigma_m)/(M_m T),  T = global_update_int dt,
    or +-max_strain_rate towards the goal while M_m = 0, capped at
    max_strain_rate (the law of the stress-controlled cell above, applied to
    the mean).  A stress counts as reached when |goal - sigma_m| <=
    max(abs_stress_tol, rel_stress_tol |goal|) and the unbalanced force is at
    most max_unbalanced; then the next stress of the series becomes the goal
    (its rate is set in the same update), and after the last one the cell
    stops (done)."""

    def __init__(self, sc, stresses, global_update_int=20, max_strain_rate=1.0, grow_damping=0.25,
                 max_unbalanced=1e-4, abs_stress_tol=1e3, rel_stress_tol=3e-5):
        self.sc = sc
        self.stresses = [float(x) for x in stresses]
        if not self.stresses:
            raise ValueError("PeriIsoCompressor: empty stress series")
        self.global_update_int = int(global_update_int)
        self.max_rate = float(max_strain_rate)
        self.grow_damping = float(grow_damping)
        self.max_unbalanced = float(max_unbalanced)
        self.abs_tol = float(abs_stress_tol)
        self.rel_tol = float(rel_stress_tol)
        self.state = 0
        self.sigma = 0.0
        self.stiff = 0.0
        self.strain_rate = 0.0
        self.unbalanced = float("nan")
        self.updates = 0
        self.done = False

    def _rate(self, goal):
        err = goal - self.sigma
        T = self.global_update_int * self.sc.dt
        if self.stiff > 0.0:
            rate = (1.0 - self.grow_damping) * err / (self.stiff * T)
        else:
            rate = math.copysign(self.max_rate, err) if err != 0.0 else 0.0
        return max(-self.max_rate, min(self.max_rate, rate))

    def _reached(self, goal):
        return (abs(goal - self.sigma) <= max(self.abs_tol, self.rel_tol * abs(goal))
                and self.unbalanced <= self.max_unbalanced)

    def update(self):
        sc = self.sc
        H, _trsf = sc.get_cell()
        V = abs(float(np.linalg.det(H)))
        sigma = sc.get_stress(V)
        M = contact_modulus(sc, V)
        self.sigma = (float(sigma[0, 0]) + float(sigma[1, 1]) + float(sigma[2, 2])) / 3.0
        self.stiff = (M[0] + M[1] + M[2]) / 3.0
        self.unbalanced = unbalanced_force(sc)
        reached = self._reached(self.stresses[self.state])
        if reached and self.state + 1 < len(self.stresses):
            self.state += 1
            reached = False
        self.done = reached
        self.strain_rate = 0.0 if reached else self._rate(self.stresses[self.state])
        sc.set_velgrad(np.eye(3) * self.strain_rate)
        self.updates += 1

    def run(self, nsteps, stop_when_done=False):
        """Step one at a time, updating after every global_update_int-th
        step; returns the number of steps run."""
        done_steps = 0
        for _ in range(int(nsteps)):
            self.sc.step(1)
            done_steps += 1
            it, _t = self.sc.counters()
            if it % self.global_update_int == 0:
                self.update()
                if self.done and stop_when_done:
                    break
        return done_steps


def run_with_timestepper(sc, nsteps, safety=0.8, interval=1):
    """Step with the stiffness timestepper: before every step whose
    iteration count is a multiple of `interval`, dt = stiffness_dt."""
    for _ in range(int(nsteps)):
        it, _t = sc.counters()
        if it % interval == 0:
            sc.set_dt(stiffness_dt(sc, safety))
        sc.step(1)
