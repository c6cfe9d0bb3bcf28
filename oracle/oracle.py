"""ctypes wrapper around libdem_oracle.so (test infrastructure only).

Argument marshalling only: every number is computed by the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdem_oracle.so")
_lib = None

_DP = C.POINTER(C.c_double)
_LP = C.POINTER(C.c_long)
_IP = C.POINTER(C.c_int)
_UP = C.POINTER(C.c_ubyte)


class OrcParams(C.Structure):
    _fields_ = [
        ("dt", C.c_double),
        ("gravity", C.c_double * 3),
        ("damping", C.c_double),
        ("damp_rot", C.c_int),
        ("periodic", C.c_int),
        ("hsize", C.c_double * 9),
        ("velgrad", C.c_double * 9),
        ("homo_deform", C.c_int),
    ]


class OrcContact(C.Structure):
    _fields_ = [
        ("id1", C.c_long),
        ("id2", C.c_long),
        ("cell", C.c_int * 3),
        ("is_wall", C.c_int),
        ("normal", C.c_double * 3),
        ("pen", C.c_double),
        ("point", C.c_double * 3),
        ("fn", C.c_double * 3),
        ("fs", C.c_double * 3),
        ("kn", C.c_double),
        ("ks", C.c_double),
    ]


CONTACT_DTYPE = np.dtype([
    ("id1", np.int64), ("id2", np.int64), ("cell", np.int32, 3), ("is_wall", np.int32),
    ("normal", np.float64, 3), ("pen", np.float64), ("point", np.float64, 3),
    ("fn", np.float64, 3), ("fs", np.float64, 3), ("kn", np.float64), ("ks", np.float64),
])
assert CONTACT_DTYPE.itemsize == C.sizeof(OrcContact)

ENERGY_KEYS = ("kinetic", "kin_rot", "elastic", "grav_work", "damp_dissip", "plastic_dissip", "total", "visc_dissip")


class OracleError(RuntimeError):
    pass


def load_library(path: str | None = None):
    """Load (building first if absent) the oracle shared library.  The
    environment variable DEM_ORACLE_LIB may name another build of the same
    source (used to check that the pins catch deliberate slips)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("DEM_ORACLE_LIB", _LIB_PATH)
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    lib = C.CDLL(path)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [C.POINTER(OrcParams)]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_last_error.restype = C.c_char_p
    sigs = {
        "orc_add_material": [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, _IP],
        "orc_add_viscel_material": [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _IP],
        "orc_add_spheres": [C.c_void_p, C.c_long, _DP, _DP, _DP, _DP, _IP, C.c_int, _UP, _LP],
        "orc_add_wall": [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int, _LP],
        "orc_pwave_dt": [C.c_void_p, _DP],
        "orc_step": [C.c_void_p, C.c_long],
        "orc_get_counters": [C.c_void_p, _LP, _DP],
        "orc_get_state": [C.c_void_p, _DP, _DP, _DP, _DP, _DP, _DP],
        "orc_set_state": [C.c_void_p, _DP, _DP, _DP, _DP],
        "orc_get_mass": [C.c_void_p, _DP, _DP],
        "orc_get_contacts": [C.c_void_p, C.c_long, C.POINTER(OrcContact), _LP],
        "orc_set_contacts": [C.c_void_p, C.c_long, _LP, _LP, _IP, _DP, _DP],
        "orc_get_energy": [C.c_void_p, _DP],
        "orc_get_cell": [C.c_void_p, _DP, _DP],
        "orc_get_stress": [C.c_void_p, C.c_double, _DP],
        "orc_detect_pairs": [C.c_void_p, C.c_long, _LP, _LP, _IP, _LP],
        "orc_spot_step": [C.c_void_p, C.c_long, _LP, _DP, _DP, _DP, _DP, _DP, _DP, _LP, _DP],
        "orc_set_dt": [C.c_void_p, C.c_double],
        "orc_add_box": [C.c_void_p, _DP, _DP, C.c_int, _LP],
        "orc_add_facet": [C.c_void_p, _DP, _DP, _DP, C.c_int, _LP],
        "orc_set_velgrad": [C.c_void_p, _DP],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.orc_num_bodies.argtypes = [C.c_void_p]
    lib.orc_num_bodies.restype = C.c_long
    lib.orc_num_contacts.argtypes = [C.c_void_p]
    lib.orc_num_contacts.restype = C.c_long
    _lib = lib
    return lib


def _ptr(a, t=_DP):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleScene:
    """One oracle scene.  Mirrors the GPU library's calls in spirit but not
    in code: the two share nothing beyond the data handed to both."""

    def __init__(self, dt, gravity=(0.0, 0.0, 0.0), damping=0.0, damp_rot=True,
                 periodic=False, hsize=None, velgrad=None, homo_deform=2):
        self.lib = load_library()
        p = OrcParams()
        p.dt = float(dt)
        p.gravity[:] = [float(g) for g in gravity]
        p.damping = float(damping)
        p.damp_rot = 1 if damp_rot else 0
        p.periodic = 1 if periodic else 0
        h = np.eye(3) if hsize is None else np.asarray(hsize, dtype=np.float64).reshape(3, 3)
        L = np.zeros((3, 3)) if velgrad is None else np.asarray(velgrad, dtype=np.float64).reshape(3, 3)
        p.hsize[:] = [float(x) for x in h.ravel()]
        p.velgrad[:] = [float(x) for x in L.ravel()]
        p.homo_deform = int(homo_deform)
        self._h = self.lib.orc_create(C.byref(p))
        if not self._h:
            raise OracleError(self.lib.orc_last_error().decode())
        # what the callers handed over, kept for the quantities computed in
        # Python from the C oracle's outputs (oracle/controls.py)
        self.dt = float(dt)
        self.periodic = bool(periodic)
        self.radius = []     # by id; 0 for a wall
        self.blocked = []    # by id; a wall counts as fully blocked (63)
        self.is_wall = []

    def close(self):
        if getattr(self, "_h", None):
            self.lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise OracleError(f"{what}: code {rc}: {self.lib.orc_last_error().decode()}")

    # -- construction -----------------------------------------------------
    def add_material(self, density, young, poisson, friction_angle):
        out = C.c_int()
        self._check(self.lib.orc_add_material(self._h, density, young, poisson, friction_angle, C.byref(out)),
                    "add_material")
        return out.value

    def add_viscel_material(self, density, tc, en, et, friction_angle):
        """ViscElMat from contact time and restitution coefficients
        (Law2_ScGeom_ViscElPhys_Basic)."""
        out = C.c_int()
        self._check(self.lib.orc_add_viscel_material(self._h, density, tc, en, et, friction_angle, C.byref(out)),
                    "add_viscel_material")
        return out.value

    def add_spheres(self, pos, radius, vel=None, angvel=None, mat=None, default_mat=0, blocked=None):
        radius = _f64(radius).ravel()
        n = radius.size
        pos = _f64(pos, (n, 3))
        vel = _f64(vel, (n, 3))
        angvel = _f64(angvel, (n, 3))
        mat_a = None if mat is None else np.ascontiguousarray(mat, dtype=np.int32).ravel()
        blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8).ravel()
        first = C.c_long()
        self._check(self.lib.orc_add_spheres(self._h, n, _ptr(pos), _ptr(radius), _ptr(vel), _ptr(angvel),
                                             _ptr(mat_a, _IP), int(default_mat), _ptr(blk, _UP), C.byref(first)),
                    "add_spheres")
        self.radius.extend(radius.tolist())
        self.blocked.extend([0] * n if blk is None else [int(b) & 63 for b in blk])
        self.is_wall.extend([False] * n)
        return first.value

    def add_wall(self, axis, position, sense=0, mat=0):
        out = C.c_long()
        self._check(self.lib.orc_add_wall(self._h, int(axis), float(position), int(sense), int(mat), C.byref(out)),
                    "add_wall")
        self.radius.append(0.0)
        self.blocked.append(63)
        self.is_wall.append(True)
        return out.value

    def add_box(self, center, half, mat=0):
        out = C.c_long()
        c, h = _f64(center, (3,)), _f64(half, (3,))
        self._check(self.lib.orc_add_box(self._h, _ptr(c), _ptr(h), int(mat), C.byref(out)), "add_box")
        self.radius.append(0.0)
        self.blocked.append(63)
        self.is_wall.append(True)
        return out.value

    def add_facet(self, v0, v1, v2, mat=0):
        out = C.c_long()
        a, b, c = _f64(v0, (3,)), _f64(v1, (3,)), _f64(v2, (3,))
        self._check(self.lib.orc_add_facet(self._h, _ptr(a), _ptr(b), _ptr(c), int(mat), C.byref(out)), "add_facet")
        self.radius.append(0.0)
        self.blocked.append(63)
        self.is_wall.append(True)
        return out.value

    # -- stepping ---------------------------------------------------------
    def pwave_dt(self):
        out = C.c_double()
        self._check(self.lib.orc_pwave_dt(self._h, C.byref(out)), "pwave_dt")
        return out.value

    def step(self, n=1):
        self._check(self.lib.orc_step(self._h, int(n)), "step")

    def set_dt(self, dt):
        self._check(self.lib.orc_set_dt(self._h, float(dt)), "set_dt")
        self.dt = float(dt)

    def set_velgrad(self, L):
        L = _f64(L, (3, 3))
        self._check(self.lib.orc_set_velgrad(self._h, _ptr(L)), "set_velgrad")

    # -- reading ----------------------------------------------------------
    @property
    def num_bodies(self):
        return self.lib.orc_num_bodies(self._h)

    def counters(self):
        it, t = C.c_long(), C.c_double()
        self._check(self.lib.orc_get_counters(self._h, C.byref(it), C.byref(t)), "get_counters")
        return it.value, t.value

    def get_state(self):
        n = self.num_bodies
        out = {k: np.zeros((n, 3)) for k in ("pos", "vel", "angvel", "force", "torque")}
        out["ori"] = np.zeros((n, 4))
        self._check(self.lib.orc_get_state(self._h, _ptr(out["pos"]), _ptr(out["vel"]), _ptr(out["angvel"]),
                                           _ptr(out["ori"]), _ptr(out["force"]), _ptr(out["torque"])),
                    "get_state")
        return out

    def get_mass(self):
        n = self.num_bodies
        m, i = np.zeros(n), np.zeros(n)
        self._check(self.lib.orc_get_mass(self._h, _ptr(m), _ptr(i)), "get_mass")
        return m, i

    def set_state(self, pos=None, vel=None, angvel=None, ori=None):
        n = self.num_bodies
        self._check(self.lib.orc_set_state(self._h, _ptr(_f64(pos, (n, 3))), _ptr(_f64(vel, (n, 3))),
                                           _ptr(_f64(angvel, (n, 3))), _ptr(_f64(ori, (n, 4)))), "set_state")

    def get_contacts(self):
        n = self.lib.orc_num_contacts(self._h)
        arr = np.zeros(max(n, 1), dtype=CONTACT_DTYPE)
        cnt = C.c_long()
        self._check(self.lib.orc_get_contacts(self._h, n, arr.ctypes.data_as(C.POINTER(OrcContact)), C.byref(cnt)),
                    "get_contacts")
        return arr[: cnt.value]

    def set_contacts(self, id1, id2, fs, nprev, cell=None):
        id1 = np.ascontiguousarray(id1, dtype=np.int64).ravel()
        id2 = np.ascontiguousarray(id2, dtype=np.int64).ravel()
        n = id1.size
        fs = _f64(fs, (n, 3))
        nprev = _f64(nprev, (n, 3))
        cell_a = None if cell is None else np.ascontiguousarray(cell, dtype=np.int32).reshape(n, 3)
        self._check(self.lib.orc_set_contacts(self._h, n, _ptr(id1, _LP), _ptr(id2, _LP), _ptr(cell_a, _IP),
                                              _ptr(fs), _ptr(nprev)), "set_contacts")

    def get_energy(self):
        out = np.zeros(8)
        self._check(self.lib.orc_get_energy(self._h, _ptr(out)), "get_energy")
        return dict(zip(ENERGY_KEYS, out.tolist()))

    def get_stress(self, volume=0.0):
        out = np.zeros(9)
        self._check(self.lib.orc_get_stress(self._h, float(volume), _ptr(out)), "get_stress")
        return out.reshape(3, 3)

    def get_cell(self):
        h, t = np.zeros(9), np.zeros(9)
        self._check(self.lib.orc_get_cell(self._h, _ptr(h), _ptr(t)), "get_cell")
        return h.reshape(3, 3), t.reshape(3, 3)

    def detect_pairs(self):
        cnt = C.c_long()
        rc = self.lib.orc_detect_pairs(self._h, 0, None, None, None, C.byref(cnt))
        if rc not in (0, 4):
            self._check(rc, "detect_pairs")
        n = cnt.value
        id1 = np.zeros(max(n, 1), dtype=np.int64)
        id2 = np.zeros(max(n, 1), dtype=np.int64)
        cell = np.zeros((max(n, 1), 3), dtype=np.int32)
        self._check(self.lib.orc_detect_pairs(self._h, n, _ptr(id1, _LP), _ptr(id2, _LP), _ptr(cell, _IP),
                                              C.byref(cnt)), "detect_pairs")
        return id1[:n], id2[:n], cell[:n]

    def spot_step(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.int64).ravel()
        k = ids.size
        out = {key: np.zeros((k, 3)) for key in ("force", "torque", "pos", "vel", "angvel")}
        out["ori"] = np.zeros((k, 4))
        out["n_contacts"] = np.zeros(k, dtype=np.int64)
        out["fmag_sum"] = np.zeros(k)
        self._check(self.lib.orc_spot_step(self._h, k, _ptr(ids, _LP), _ptr(out["force"]), _ptr(out["torque"]),
                                           _ptr(out["pos"]), _ptr(out["vel"]), _ptr(out["angvel"]),
                                           _ptr(out["ori"]), _ptr(out["n_contacts"], _LP),
                                           _ptr(out["fmag_sum"])), "spot_step")
        return out
