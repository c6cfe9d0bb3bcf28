"""Pins of the oracle's visco-elastic law (Law2_ScGeom_ViscElPhys_Basic with
Ip2_ViscElMat_ViscElMat_ViscElPhys from contact time and restitution
coefficients) against the mechanics of a collision.

The closed forms of k_n, c_n, k_s and c_s are built so that a two-body
collision lasts t_c and ends with the normal relative velocity reversed and
scaled by e_n; with the sphere's tangential effective mass 2/7 m the
tangential velocity of the contact point follows a damped oscillator whose
state after t_c has a closed form in e_t.  These tests measure those
outcomes from simulated collisions (the expected values are t_c, e_n and
the oscillator's solution, not the coefficient formulas), to within the
leapfrog's O(dt / t_c) error: a wrong mass (the sphere's instead of the reduced one),
a lost 2/7, a flipped dashpot sign or a wrong dashpot work fails one of them.
"""
import math

import numpy as np
import pytest

from oracle import OracleScene
from oracle.oracle import OracleError

R = 2.0 ** -10
RHO = 2600.0
TC = 2e-4
STEPS_PER_TC = 2000


def _mass(r):
    return 4.0 / 3.0 * math.pi * r ** 3 * RHO


def _run_collision(s, max_steps):
    """Step until the contact list has been non-empty and is empty again;
    returns (first step with a contact, first step without one after it)."""
    start = end = None
    for i in range(max_steps):
        s.step(1)
        c = s.get_contacts()
        if len(c) and start is None:
            start = i
        if start is not None and not len(c):
            end = i
            break
    assert start is not None and end is not None, "the collision did not finish"
    return start, end


def _pair(r1, r2, v, en, et=1.0, friction=0.3):
    s = OracleScene(dt=TC / STEPS_PER_TC, gravity=(0.0, 0.0, 0.0), damping=0.0)
    m = s.add_viscel_material(RHO, TC, en, et, friction)
    gap = 1e-3 * R
    pos = np.array([[0.0, 0.0, 0.0], [r1 + r2 + gap, 0.0, 0.0]])
    vel = np.array([[v, 0.0, 0.0], [-v, 0.0, 0.0]])
    s.add_spheres(pos, [r1, r2], vel=vel, default_mat=m)
    return s


@pytest.mark.parametrize("en", [0.9, 0.5, 0.2])
def test_head_on_equal_spheres_duration_and_restitution(en):
    """Equal spheres approaching at 2v: the contact lasts t_c and the
    relative velocity leaves at -e_n times the incoming one."""
    v = 0.05
    s = _pair(R, R, v, en)
    start, end = _run_collision(s, 3 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(TC, abs=3 * dt)
    vel = s.get_state()["vel"]
    e = (vel[1, 0] - vel[0, 0]) / (2 * v)
    assert e == pytest.approx(en, rel=3e-3)
    # momentum is conserved exactly up to rounding
    assert abs(_mass(R) * (vel[0, 0] + vel[1, 0])) <= 1e-15 * _mass(R) * v


def test_unequal_spheres_use_the_reduced_mass():
    """Radii r and 2r (mass ratio 8): still t_c and e_n, which holds only
    with the reduced mass m1 m2/(m1 + m2) in k_n and c_n."""
    v, en = 0.05, 0.6
    s = _pair(R, 2 * R, v, en)
    start, end = _run_collision(s, 3 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(TC, abs=3 * dt)
    vel = s.get_state()["vel"]
    e = (vel[1, 0] - vel[0, 0]) / (-2 * v)
    assert -e == pytest.approx(en, rel=3e-3)
    m1, m2 = _mass(R), _mass(2 * R)
    assert abs(m1 * vel[0, 0] + m2 * vel[1, 0] - (m1 - m2) * v) <= 1e-13 * m2 * v


@pytest.mark.parametrize("fixed", [0, 1])
def test_collision_with_a_fixed_sphere_uses_the_moving_mass(fixed):
    """A sphere hitting a sphere with all six DOFs blocked (as #1 or as #2
    of the pair): t_c and e_n with the moving sphere's own mass (the fixed
    one acts as a boundary); the fixed sphere does not move."""
    v, en = 0.05, 0.5
    s = OracleScene(dt=TC / STEPS_PER_TC, gravity=(0.0, 0.0, 0.0), damping=0.0)
    m = s.add_viscel_material(RHO, TC, en, 1.0, 0.3)
    pos = np.array([[0.0, 0.0, 0.0], [2 * R * (1 + 1e-3), 0.0, 0.0]])
    moving = 1 - fixed
    vel = np.zeros((2, 3))
    vel[moving, 0] = v if moving == 0 else -v
    blocked = [0, 0]
    blocked[fixed] = 63
    s.add_spheres(pos, [R, R], vel=vel, default_mat=m, blocked=blocked)
    start, end = _run_collision(s, 3 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(TC, abs=3 * dt)
    st = s.get_state()
    assert -st["vel"][moving, 0] / vel[moving, 0] == pytest.approx(en, rel=3e-3)
    assert np.array_equal(st["pos"][fixed], pos[fixed])


def _wall_bounce(en, et, vn, vt, friction=1.5):
    s = OracleScene(dt=TC / STEPS_PER_TC, gravity=(0.0, 0.0, 0.0), damping=0.0)
    m = s.add_viscel_material(RHO, TC, en, et, friction)
    s.add_wall(2, 0.0, 1, m)
    s.add_spheres(np.array([[0.0, 0.0, R * (1 + 1e-3)]]), [R], vel=np.array([[vt, 0.0, -vn]]), default_mat=m)
    return s


def test_wall_bounce_uses_the_sphere_mass():
    """A sphere on a wall: t_c and e_n with the sphere's own mass (the wall
    does not move)."""
    vn, en = 0.1, 0.4
    s = _wall_bounce(en, 1.0, vn, 0.0)
    start, end = _run_collision(s, 3 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(TC, abs=3 * dt)
    assert s.get_state()["vel"][1, 2] / vn == pytest.approx(en, rel=3e-3)


def test_wall_bounce_energy_balance():
    """A sphere bouncing on a wall with e_n = 0.4: the dashpot work is
    (1 - e_n^2) of the incoming kinetic energy (the wall takes none)."""
    vn, en = 0.1, 0.4
    s = _wall_bounce(en, 1.0, vn, 0.0)
    _run_collision(s, 3 * STEPS_PER_TC)
    e0 = 0.5 * _mass(R) * vn * vn
    assert s.get_energy()["visc_dissip"] / e0 == pytest.approx(1 - en * en, rel=5e-3)


@pytest.mark.parametrize("et", [0.9, 0.5])
def test_oblique_sticking_impact_tangential_closed_form(et):
    """Oblique impact on a wall with e_n = 1 (no normal dashpot, so the
    normal force stays compressive and the contact lasts t_c) and a
    friction angle large enough to stick throughout.  The contact point's
    tangential velocity u = v_x - r w_y obeys m_t u'' = -k_s u - c_s u' with
    the sphere's tangential effective mass m_t = 2/7 m (1/m + r^2/I = 7/(2m)).
    With the printed k_s and c_s, gamma = c_s/(2 m_t) = -ln(e_t)/(2 t_c) and
    omega t_c = theta = sqrt(pi^2 + 3/4 ln^2 e_t), so after t_c
    u/u0 = exp(-gamma t_c) (cos theta - (gamma t_c/theta) sin theta), about
    -sqrt(e_t) (the printed c_t carries half the damping that would make
    the tangential restitution e_t itself).  Translation and spin share the
    impulse as 2/7 and 5/7."""
    vn, vt = 0.1, 0.05
    s = _wall_bounce(1.0, et, vn, vt, friction=1.55)
    start, end = _run_collision(s, 3 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(TC, abs=3 * dt)
    st = s.get_state()
    v, w = st["vel"][1], st["angvel"][1]
    # contact point at x - r e_z: its velocity v + w x (-r e_z), x component v_x - r w_y
    uc = v[0] - R * w[1]
    g = -math.log(et) / 2.0
    theta = math.sqrt(math.pi ** 2 + 0.75 * math.log(et) ** 2)
    expected = math.exp(-g) * (math.cos(theta) - (g / theta) * math.sin(theta))
    assert uc / vt == pytest.approx(expected, rel=2e-3)
    assert v[2] / vn == pytest.approx(1.0, rel=3e-3)
    # impulse J along x: m (v_x - vt) = J, I w_y = -r J (I = 2/5 m r^2)
    J = _mass(R) * (v[0] - vt)
    assert 0.4 * _mass(R) * R * R * w[1] == pytest.approx(-R * J, rel=1e-9)


def test_energy_balance_with_dashpots():
    """Over a lossy head-on collision (e_n = 0.5) the kinetic energy lost
    equals the dashpots' work: kinetic + elastic + visc_dissip stays at the
    initial kinetic energy (the leapfrog's O(dt) aside); at the end the
    dissipated share is 1 - e_n^2."""
    v, en = 0.05, 0.5
    s = _pair(R, R, v, en)
    e0 = 2 * 0.5 * _mass(R) * v * v
    worst = 0.0
    start = None
    for i in range(3 * STEPS_PER_TC):
        s.step(1)
        e = s.get_energy()
        bal = e["kinetic"] + e["elastic"] + e["visc_dissip"]
        worst = max(worst, abs(bal - e0) / e0)
        c = s.get_contacts()
        if len(c) and start is None:
            start = i
        if start is not None and not len(c):
            break
    assert worst <= 5e-3
    e = s.get_energy()
    assert e["visc_dissip"] / e0 == pytest.approx(1 - en * en, rel=5e-3)
    assert e["total"] == pytest.approx(e["kinetic"] + e["kin_rot"] + e["elastic"] + e["visc_dissip"], rel=1e-12)


def test_two_contact_times_collide_over_their_mean():
    """Equal spheres of two visco-elastic materials whose contact times are
    t_c and 3 t_c: the pair takes the mean of the two (2 t_c), so the
    collision lasts 2 t_c and still restitutes e_n."""
    v, en = 0.05, 0.5
    s = OracleScene(dt=TC / STEPS_PER_TC, gravity=(0.0, 0.0, 0.0), damping=0.0)
    m1 = s.add_viscel_material(RHO, TC, en, 1.0, 0.3)
    m2 = s.add_viscel_material(RHO, 3 * TC, en, 1.0, 0.3)
    pos = np.array([[0.0, 0.0, 0.0], [2 * R + 1e-3 * R, 0.0, 0.0]])
    s.add_spheres(pos, [R, R], vel=[[v, 0.0, 0.0], [-v, 0.0, 0.0]], mat=[m1, m2])
    start, end = _run_collision(s, 6 * STEPS_PER_TC)
    dt = TC / STEPS_PER_TC
    assert (end - start) * dt == pytest.approx(2 * TC, abs=3 * dt)
    vel = s.get_state()["vel"]
    assert (vel[1, 0] - vel[0, 0]) / (2 * v) == pytest.approx(en, rel=3e-3)


def test_prescribed_slip_with_the_shear_dashpot():
    """A sphere at a fixed overlap d on a visco-elastic floor, driven along
    it at v0 with its translations and its spins about x and y blocked (the
    spin about z is left free, so that the sphere is not an immovable body,
    and stays zero: the friction's torque is about y); the floor is fixed,
    so the pair's mass is the sphere's.  No normal motion, so F_n = k_n d; while the
    shear spring holds, the reported shear force is the spring's
    k_s v0 t plus the dashpot's c_s v0 and the dashpot works c_s v0^2 per
    unit time; once the spring passes tan(phi) F_n the contact slides at
    exactly that force with the dashpot idle, and the plastic work is
    c (v0 t - c/k_s) as for the linear law.  Guards the slider's series
    arrangement (dashpot off while sliding) and the dashpot's work."""
    en, et, phi = 0.6, 0.4, 0.35
    dt = TC / STEPS_PER_TC
    m = _mass(R)
    kn = m * (math.pi ** 2 + math.log(en) ** 2) / TC ** 2
    ks = 2.0 / 7.0 * m * (math.pi ** 2 + math.log(et) ** 2) / TC ** 2
    cs = -2.0 / 7.0 * m * math.log(et) / TC
    d = 1e-3 * R
    cap = kn * d * math.tan(phi)
    v0 = cap / (ks * 100.5 * dt)  # the spring passes the cap between steps 100 and 101
    s = OracleScene(dt=dt, gravity=(0.0, 0.0, 0.0), damping=0.0)
    mat = s.add_viscel_material(RHO, TC, en, et, phi)
    s.add_wall(2, 0.0, 1, mat)
    s.add_spheres([[0.0, 0.0, R - d]], [R], vel=[[v0, 0.0, 0.0]], default_mat=mat, blocked=[31])
    for k in (40, 80):
        s.step(40)
        t = k * dt
        c, e = s.get_contacts(), s.get_energy()
        assert len(c) == 1 and c["fs"][0][0] < 0.0
        assert np.linalg.norm(c["fs"][0]) == pytest.approx(ks * v0 * t + cs * v0, rel=1e-11)
        assert np.linalg.norm(c["fn"][0]) == pytest.approx(kn * d, rel=1e-11)
        assert e["visc_dissip"] == pytest.approx(cs * v0 * v0 * t, rel=1e-11)
        assert e["plastic_dissip"] == 0.0
    s.step(420)
    t = 500 * dt
    c, e = s.get_contacts(), s.get_energy()
    assert np.linalg.norm(c["fs"][0]) == pytest.approx(cap, rel=1e-11)
    assert e["visc_dissip"] == pytest.approx(cs * v0 * v0 * 100 * dt, rel=1e-11)
    assert e["plastic_dissip"] == pytest.approx(cap * (v0 * t - cap / ks), rel=1e-9)
    assert np.array_equal(s.get_state()["angvel"][1], [0.0, 0.0, 0.0])


def test_contact_reports_the_dashpot_force():
    """Mid-collision the reported normal force is k_n pen - c_n (v2 - v1).n
    along n: at the first contact step of a head-on approach it exceeds the
    spring's k_n pen by the dashpot's c_n |u_n| > 0."""
    v, en = 0.05, 0.3
    s = _pair(R, R, v, en)
    for _ in range(10 * STEPS_PER_TC):
        s.step(1)
        c = s.get_contacts()
        if len(c):
            break
    fn = c["fn"][0] @ c["normal"][0]
    assert fn > c["kn"][0] * c["pen"][0]


def test_mixed_material_kinds_are_refused():
    s = OracleScene(dt=1e-7)
    a = s.add_material(RHO, 1e7, 0.3, 0.5)
    b = s.add_viscel_material(RHO, TC, 0.5, 0.5, 0.3)
    s.add_spheres(np.array([[0.0, 0.0, 0.0], [3 * R, 0.0, 0.0]]), [R, R], mat=[a, b])
    with pytest.raises(OracleError):
        s.step(1)
    with pytest.raises(OracleError):
        s.add_viscel_material(RHO, TC, 0.0, 0.5, 0.3)
    with pytest.raises(OracleError):
        s.add_viscel_material(RHO, -1.0, 0.5, 0.5, 0.3)
