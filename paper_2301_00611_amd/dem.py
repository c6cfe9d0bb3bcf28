"""ctypes binding of libdem_hip.so (declared in include/dem.h).

Argument marshalling only: every step of the method runs in the HIP
library.  There is no fallback: if the compiled library is missing, loading
raises ImportError (build it with ``python -m paper_2301_00611_amd.build``).

The raw entry points keep their C names (``dem_create``, ``dem_step``, ...);
``Scene`` and ``Batch`` are thin conveniences that hold the handle and turn
host buffers into numpy arrays.  PyTorch appears only as an optional source
of device buffers (``get_state_device``) and streams (``dem_params.stream``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .geom import aabb_walls, facet_box_triangles, packing_extrema  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdem_hip.so")

DEM_OK, DEM_EINVAL, DEM_ERANGE, DEM_ENOENT, DEM_ECAPACITY, DEM_ENOMEM, DEM_EDEVICE = range(7)
DEM_ENONFINITE, DEM_EPERIODIC, DEM_EUNSTABLE, DEM_EBUSY = 7, 8, 9, 10
DEM_FP64, DEM_FP32_MIXED = 0, 1

_DP = C.POINTER(C.c_double)
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_U8P = C.POINTER(C.c_uint8)


class dem_params(C.Structure):
    _fields_ = [
        ("dt", C.c_double),
        ("gravity", C.c_double * 3),
        ("damping", C.c_double),
        ("damp_rot", C.c_int32),
        ("verlet_dist", C.c_double),
        ("precision", C.c_int32),
        ("periodic", C.c_int32),
        ("hsize", C.c_double * 9),
        ("velgrad", C.c_double * 9),
        ("homo_deform", C.c_int32),
        ("track_energy", C.c_int32),
        ("device", C.c_int32),
        ("stream", C.c_void_p),
    ]


class dem_contact(C.Structure):
    _fields_ = [
        ("id1", C.c_int64), ("id2", C.c_int64), ("cell", C.c_int32 * 3), ("is_wall", C.c_int32),
        ("normal", C.c_double * 3), ("pen", C.c_double), ("point", C.c_double * 3),
        ("fn", C.c_double * 3), ("fs", C.c_double * 3), ("kn", C.c_double), ("ks", C.c_double),
    ]


class dem_history(C.Structure):
    _fields_ = [
        ("id1", C.c_int64), ("id2", C.c_int64), ("cell", C.c_int32 * 3), ("pad", C.c_int32),
        ("fs", C.c_double * 3), ("nprev", C.c_double * 3),
    ]


class dem_energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("kinetic", "kin_rot", "elastic", "grav_work", "damp_dissip", "plastic_dissip", "total",
                 "visc_dissip")]


class dem_stats(C.Structure):
    _fields_ = [
        ("iter", C.c_int64), ("time", C.c_double), ("n_spheres", C.c_int64), ("n_walls", C.c_int64),
        ("n_contacts_ss", C.c_int64), ("n_contacts_sw", C.c_int64), ("n_candidates", C.c_int64),
        ("rebuilds", C.c_int64), ("contact_steps", C.c_int64), ("coordination", C.c_double),
        ("verlet_dist", C.c_double), ("max_overlap_ratio", C.c_double),
    ]


class dem_tuning(C.Structure):
    _fields_ = [("block_contact", C.c_int32), ("block_integrate", C.c_int32), ("chunk", C.c_int32),
                ("pad", C.c_int32), ("verlet_factor", C.c_double), ("ms_per_step", C.c_double)]


class dem_peri_triax(C.Structure):
    _fields_ = [("goal", C.c_double * 3), ("stress_mask", C.c_int32), ("glob_update", C.c_int32),
                ("max_strain_rate", C.c_double * 3), ("grow_damping", C.c_double),
                ("max_unbalanced", C.c_double), ("abs_stress_tol", C.c_double), ("rel_stress_tol", C.c_double),
                ("stop_when_done", C.c_int32), ("pad", C.c_int32)]


class dem_peri_triax_state(C.Structure):
    _fields_ = [("stress", C.c_double * 3), ("strain", C.c_double * 3), ("strain_rate", C.c_double * 3),
                ("stiff", C.c_double * 3), ("unbalanced", C.c_double), ("updates", C.c_int64),
                ("done", C.c_int32), ("active", C.c_int32)]


class dem_peri_iso(C.Structure):
    _fields_ = [("n_stresses", C.c_int32), ("global_update", C.c_int32), ("stresses", C.c_double * 8),
                ("max_strain_rate", C.c_double), ("grow_damping", C.c_double), ("max_unbalanced", C.c_double),
                ("abs_stress_tol", C.c_double), ("rel_stress_tol", C.c_double), ("stop_when_done", C.c_int32),
                ("pad_", C.c_int32)]


class dem_peri_iso_state(C.Structure):
    _fields_ = [("state", C.c_int32), ("done", C.c_int32), ("sigma", C.c_double), ("stiff", C.c_double),
                ("strain_rate", C.c_double), ("unbalanced", C.c_double), ("updates", C.c_int64),
                ("active", C.c_int32), ("pad_", C.c_int32)]


def _tuning_dict(t):
    return {k: getattr(t, k) for k, _ in dem_tuning._fields_ if k != "pad"}


def _tuning_struct(d):
    t = dem_tuning()
    for k, v in d.items():
        setattr(t, k, v)
    return t


CONTACT_DTYPE = np.dtype([
    ("id1", np.int64), ("id2", np.int64), ("cell", np.int32, 3), ("is_wall", np.int32),
    ("normal", np.float64, 3), ("pen", np.float64), ("point", np.float64, 3),
    ("fn", np.float64, 3), ("fs", np.float64, 3), ("kn", np.float64), ("ks", np.float64),
])
HISTORY_DTYPE = np.dtype([
    ("id1", np.int64), ("id2", np.int64), ("cell", np.int32, 3), ("pad", np.int32),
    ("fs", np.float64, 3), ("nprev", np.float64, 3),
])
assert CONTACT_DTYPE.itemsize == C.sizeof(dem_contact)
assert HISTORY_DTYPE.itemsize == C.sizeof(dem_history)

# name -> (restype, argtypes), exactly the declarations of include/dem.h
SIGNATURES = {
    "dem_abi_version": (C.c_int32, []),
    "dem_last_error": (C.c_char_p, []),
    "dem_params_default": (None, [C.POINTER(dem_params)]),
    "dem_create": (C.c_int32, [C.POINTER(dem_params), C.POINTER(C.c_void_p)]),
    "dem_destroy": (C.c_int32, [C.c_void_p]),
    "dem_add_material": (C.c_int32, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, _I32P]),
    "dem_add_viscel_material": (C.c_int32, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                            _I32P]),
    "dem_add_spheres": (C.c_int32, [C.c_void_p, C.c_int64, _DP, _DP, _DP, _DP, _I32P, C.c_int32, _U8P, _I64P]),
    "dem_add_wall": (C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_int32, _I64P]),
    "dem_pwave_dt": (C.c_int32, [C.c_void_p, _DP]),
    "dem_set_dt": (C.c_int32, [C.c_void_p, C.c_double]),
    "dem_set_velgrad": (C.c_int32, [C.c_void_p, _DP]),
    "dem_get_cell": (C.c_int32, [C.c_void_p, _DP, _DP]),
    "dem_step": (C.c_int32, [C.c_void_p, C.c_int64]),
    "dem_step_async": (C.c_int32, [C.c_void_p, C.c_int64]),
    "dem_wait": (C.c_int32, [C.c_void_p]),
    "dem_get_state": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int64, _DP, _DP, _DP, _DP, _DP, _DP]),
    "dem_get_state_device": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int64, _DP, _DP, _DP, _DP]),
    "dem_set_state": (C.c_int32, [C.c_void_p, _DP, _DP, _DP, _DP]),
    "dem_get_mass": (C.c_int32, [C.c_void_p, _DP, _DP]),
    "dem_get_contacts": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(dem_contact), _I64P]),
    "dem_get_interaction": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int64, _I32P, C.POINTER(dem_contact)]),
    "dem_get_history": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(dem_history), _I64P]),
    "dem_set_history": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(dem_history)]),
    "dem_get_energy": (C.c_int32, [C.c_void_p, C.POINTER(dem_energy)]),
    "dem_get_stress": (C.c_int32, [C.c_void_p, C.c_double, _DP]),
    "dem_get_stress_noalloc": (C.c_int32, [C.c_void_p, C.c_double, _DP]),
    "dem_get_stats": (C.c_int32, [C.c_void_p, C.POINTER(dem_stats)]),
    "dem_set_timing": (C.c_int32, [C.c_void_p, C.c_int32]),
    "dem_get_timing": (C.c_int32, [C.c_void_p, C.c_char_p, _DP, _I64P]),
    "dem_batch_create": (C.c_int32, [C.c_int32, C.POINTER(dem_params), C.POINTER(C.c_void_p)]),
    "dem_batch_scene": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "dem_batch_step": (C.c_int32, [C.c_void_p, C.c_int64]),
    "dem_batch_stats": (C.c_int32, [C.c_void_p, C.POINTER(dem_stats)]),
    "dem_batch_destroy": (C.c_int32, [C.c_void_p]),
    "dem_get_tuning": (C.c_int32, [C.c_void_p, C.POINTER(dem_tuning)]),
    "dem_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(dem_tuning)]),
    "dem_autotune": (C.c_int32, [C.c_void_p, C.c_int64, C.c_char_p, C.POINTER(dem_tuning)]),
    "dem_batch_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(dem_tuning)]),
    "dem_batch_autotune": (C.c_int32, [C.c_void_p, C.c_int64, C.c_char_p, C.POINTER(dem_tuning)]),
    "dem_add_box": (C.c_int32, [C.c_void_p, _DP, _DP, C.c_int32, _I64P]),
    "dem_add_facet": (C.c_int32, [C.c_void_p, _DP, _DP, _DP, C.c_int32, _I64P]),
    "dem_get_unbalanced_force": (C.c_int32, [C.c_void_p, C.c_int32, _DP]),
    "dem_stiffness_dt": (C.c_int32, [C.c_void_p, C.c_double, _DP]),
    "dem_set_stiffness_timestepper": (C.c_int32, [C.c_void_p, C.c_double, C.c_int64]),
    "dem_peri_triax_default": (None, [C.POINTER(dem_peri_triax)]),
    "dem_set_peri_triax": (C.c_int32, [C.c_void_p, C.POINTER(dem_peri_triax)]),
    "dem_get_peri_triax": (C.c_int32, [C.c_void_p, C.POINTER(dem_peri_triax_state)]),
    "dem_peri_iso_default": (None, [C.POINTER(dem_peri_iso)]),
    "dem_set_peri_iso": (C.c_int32, [C.c_void_p, C.POINTER(dem_peri_iso)]),
    "dem_get_peri_iso": (C.c_int32, [C.c_void_p, C.POINTER(dem_peri_iso_state)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libdem_hip.so.  Raises ImportError when it is missing: the
    product path has no CPU fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2301_00611_amd.build`")
    # PyTorch ships its own HIP runtime library; loading it first makes this
    # library bind to the same one, so both share one HIP runtime in the
    # process (a second runtime initialised later finds no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dem error {code}: {msg}")
        self.code = code


def check(rc, what=""):
    if rc != DEM_OK:
        raise DemError(rc, f"{what}: {load().dem_last_error().decode()}")


def _p(a, t=_DP):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64).reshape(shape)


def make_params(dt=0.0, gravity=(0.0, 0.0, 0.0), damping=0.2, damp_rot=True, verlet_dist=-0.5,
                precision=DEM_FP64, periodic=False, hsize=None, velgrad=None, homo_deform=2,
                track_energy=False, device=0, stream=None):
    p = dem_params()
    load().dem_params_default(C.byref(p))
    p.dt = float(dt)
    p.gravity[:] = [float(g) for g in gravity]
    p.damping = float(damping)
    p.damp_rot = 1 if damp_rot else 0
    p.verlet_dist = float(verlet_dist)
    p.precision = int(precision)
    p.periodic = 1 if periodic else 0
    if hsize is not None:
        p.hsize[:] = [float(x) for x in np.asarray(hsize, dtype=np.float64).ravel()]
    if velgrad is not None:
        p.velgrad[:] = [float(x) for x in np.asarray(velgrad, dtype=np.float64).ravel()]
    p.homo_deform = int(homo_deform)
    p.track_energy = 1 if track_energy else 0
    p.device = int(device)
    p.stream = stream
    return p


class Scene:
    """One scene (owning), or a non-owning view of a batch scene."""

    def __init__(self, handle=None, owner=True, **params):
        self.lib = load()
        if handle is None:
            h = C.c_void_p()
            p = make_params(**params)
            check(self.lib.dem_create(C.byref(p), C.byref(h)), "dem_create")
            handle = h
        self.h = handle
        self.owner = owner

    def close(self):
        if self.owner and self.h:
            check(self.lib.dem_destroy(self.h), "dem_destroy")
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # construction
    def add_material(self, density, young, poisson, friction_angle):
        m = C.c_int32()
        check(self.lib.dem_add_material(self.h, density, young, poisson, friction_angle, C.byref(m)),
              "dem_add_material")
        return m.value

    def add_viscel_material(self, density, tc, en, et, friction_angle):
        """ViscElMat from contact time and restitution coefficients
        (Law2_ScGeom_ViscElPhys_Basic)."""
        m = C.c_int32()
        check(self.lib.dem_add_viscel_material(self.h, density, tc, en, et, friction_angle, C.byref(m)),
              "dem_add_viscel_material")
        return m.value

    def add_spheres(self, pos, radius, vel=None, angvel=None, mat=None, default_mat=0, blocked=None):
        radius = np.ascontiguousarray(radius, dtype=np.float64).ravel()
        n = radius.size
        pos, vel, angvel = _f64(pos, (n, 3)), _f64(vel, (n, 3)), _f64(angvel, (n, 3))
        mat_a = None if mat is None else np.ascontiguousarray(mat, dtype=np.int32).ravel()
        blk = None if blocked is None else np.ascontiguousarray(blocked, dtype=np.uint8).ravel()
        first = C.c_int64()
        check(self.lib.dem_add_spheres(self.h, n, _p(pos), _p(radius), _p(vel), _p(angvel), _p(mat_a, _I32P),
                                       int(default_mat), _p(blk, _U8P), C.byref(first)), "dem_add_spheres")
        return first.value

    def add_wall(self, axis, position, sense=0, mat=0):
        out = C.c_int64()
        check(self.lib.dem_add_wall(self.h, int(axis), float(position), int(sense), int(mat), C.byref(out)),
              "dem_add_wall")
        return out.value

    def add_box(self, center, half, mat=0):
        c, h = _f64(center, (3,)), _f64(half, (3,))
        out = C.c_int64()
        check(self.lib.dem_add_box(self.h, _p(c), _p(h), int(mat), C.byref(out)), "dem_add_box")
        return out.value

    def add_facet(self, v0, v1, v2, mat=0):
        a, b, c = _f64(v0, (3,)), _f64(v1, (3,)), _f64(v2, (3,))
        out = C.c_int64()
        check(self.lib.dem_add_facet(self.h, _p(a), _p(b), _p(c), int(mat), C.byref(out)), "dem_add_facet")
        return out.value

    def add_facet_box(self, center, half, mat=0, wall_mask=63):
        """geom.facetBox: the faces of an axis-aligned box as two facets
        each; wall_mask bits 1, 2, 4, 8, 16, 32 keep the x-, x+, y-, y+, z-,
        z+ faces.  Returns the facets' ids."""
        return [self.add_facet(*tri, mat=mat) for tri in facet_box_triangles(center, half, wall_mask)]

    def add_aabb_walls(self, extrema, mat=0, thickness=None, oversize_factor=1.5):
        """utils.aabbWalls: six boxes wrapping the packing whose bounding box
        is extrema = (lo, hi) (see geom.aabb_walls for the placement), in the
        order min x, max x, min y, max y, min z, max z.  Returns their ids."""
        return [self.add_box(c, h, mat) for c, h in aabb_walls(extrema, thickness, oversize_factor)]

    def pwave_dt(self):
        out = C.c_double()
        check(self.lib.dem_pwave_dt(self.h, C.byref(out)), "dem_pwave_dt")
        return out.value

    def set_dt(self, dt):
        check(self.lib.dem_set_dt(self.h, float(dt)), "dem_set_dt")

    def set_velgrad(self, L):
        a = _f64(L, (9,))
        check(self.lib.dem_set_velgrad(self.h, _p(a)), "dem_set_velgrad")

    def get_cell(self):
        h, t = np.zeros(9), np.zeros(9)
        check(self.lib.dem_get_cell(self.h, _p(h), _p(t)), "dem_get_cell")
        return h.reshape(3, 3), t.reshape(3, 3)

    # stepping
    def step(self, n=1):
        check(self.lib.dem_step(self.h, int(n)), "dem_step")

    def step_async(self, n=1):
        check(self.lib.dem_step_async(self.h, int(n)), "dem_step_async")

    def wait(self):
        check(self.lib.dem_wait(self.h), "dem_wait")

    # reading
    def stats(self):
        s = dem_stats()
        check(self.lib.dem_get_stats(self.h, C.byref(s)), "dem_get_stats")
        return {k: getattr(s, k) for k, _ in dem_stats._fields_}

    @property
    def num_bodies(self):
        st = self.stats()
        return st["n_spheres"] + st["n_walls"]

    def get_state(self, first=0, count=None):
        if count is None:
            count = self.num_bodies - first
        out = {k: np.zeros((count, 3)) for k in ("pos", "vel", "angvel", "force", "torque")}
        out["ori"] = np.zeros((count, 4))
        check(self.lib.dem_get_state(self.h, int(first), int(count), _p(out["pos"]), _p(out["vel"]),
                                     _p(out["angvel"]), _p(out["ori"]), _p(out["force"]), _p(out["torque"])),
              "dem_get_state")
        return out

    def get_state_device(self, pos, vel=None, angvel=None, ori=None, first=0):
        """Fill caller-owned device tensors (torch, float64, contiguous)."""
        count = pos.shape[0]
        ptr = (lambda t: None if t is None else C.cast(C.c_void_p(t.data_ptr()), _DP))
        check(self.lib.dem_get_state_device(self.h, int(first), int(count), ptr(pos), ptr(vel), ptr(angvel),
                                            ptr(ori)), "dem_get_state_device")

    def set_state(self, pos=None, vel=None, angvel=None, ori=None):
        n = self.num_bodies
        check(self.lib.dem_set_state(self.h, _p(_f64(pos, (n, 3))), _p(_f64(vel, (n, 3))),
                                     _p(_f64(angvel, (n, 3))), _p(_f64(ori, (n, 4)))), "dem_set_state")

    def get_mass(self):
        n = self.num_bodies
        m, i = np.zeros(n), np.zeros(n)
        check(self.lib.dem_get_mass(self.h, _p(m), _p(i)), "dem_get_mass")
        return m, i

    def get_contacts(self):
        cnt = C.c_int64()
        rc = self.lib.dem_get_contacts(self.h, 0, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_ECAPACITY):
            check(rc, "dem_get_contacts")
        arr = np.zeros(max(cnt.value, 1), dtype=CONTACT_DTYPE)
        check(self.lib.dem_get_contacts(self.h, cnt.value, arr.ctypes.data_as(C.POINTER(dem_contact)),
                                        C.byref(cnt)), "dem_get_contacts")
        return arr[: cnt.value]

    def get_interaction(self, id1, id2, cell=None):
        """The real contact between id1 and id2 (either order) as a
        CONTACT_DTYPE record; DemError with code DEM_ENOENT if none."""
        out = np.zeros(1, dtype=CONTACT_DTYPE)
        c = None if cell is None else np.ascontiguousarray(cell, dtype=np.int32).reshape(3)
        check(self.lib.dem_get_interaction(self.h, int(id1), int(id2), _p(c, _I32P),
                                           out.ctypes.data_as(C.POINTER(dem_contact))), "dem_get_interaction")
        return out[0]

    def get_history(self):
        cnt = C.c_int64()
        rc = self.lib.dem_get_history(self.h, 0, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_ECAPACITY):
            check(rc, "dem_get_history")
        arr = np.zeros(max(cnt.value, 1), dtype=HISTORY_DTYPE)
        check(self.lib.dem_get_history(self.h, cnt.value, arr.ctypes.data_as(C.POINTER(dem_history)),
                                       C.byref(cnt)), "dem_get_history")
        return arr[: cnt.value]

    def set_history(self, id1, id2, fs, nprev, cell=None):
        id1 = np.asarray(id1, dtype=np.int64).ravel()
        n = id1.size
        arr = np.zeros(max(n, 1), dtype=HISTORY_DTYPE)[:n]
        arr["id1"] = id1
        arr["id2"] = np.asarray(id2, dtype=np.int64).ravel()
        arr["fs"] = np.asarray(fs, dtype=np.float64).reshape(n, 3)
        arr["nprev"] = np.asarray(nprev, dtype=np.float64).reshape(n, 3)
        if cell is not None:
            arr["cell"] = np.asarray(cell, dtype=np.int32).reshape(n, 3)
        arr = np.ascontiguousarray(arr)
        check(self.lib.dem_set_history(self.h, n, arr.ctypes.data_as(C.POINTER(dem_history))), "dem_set_history")

    def get_energy(self):
        e = dem_energy()
        check(self.lib.dem_get_energy(self.h, C.byref(e)), "dem_get_energy")
        return {k: getattr(e, k) for k, _ in dem_energy._fields_}

    def get_stress(self, volume=0.0):
        out = np.zeros(9)
        check(self.lib.dem_get_stress(self.h, float(volume), _p(out)), "dem_get_stress")
        return out.reshape(3, 3)

    def get_stress_noalloc(self, volume=0.0):
        out = np.zeros(9)
        check(self.lib.dem_get_stress_noalloc(self.h, float(volume), _p(out)), "dem_get_stress_noalloc")
        return out.reshape(3, 3)

    def unbalanced_force(self, use_max=False):
        out = C.c_double()
        check(self.lib.dem_get_unbalanced_force(self.h, 1 if use_max else 0, C.byref(out)), "dem_get_unbalanced_force")
        return out.value

    def stiffness_dt(self, safety=0.8):
        out = C.c_double()
        check(self.lib.dem_stiffness_dt(self.h, float(safety), C.byref(out)), "dem_stiffness_dt")
        return out.value

    def set_stiffness_timestepper(self, safety=0.8, interval=1):
        check(self.lib.dem_set_stiffness_timestepper(self.h, float(safety), int(interval)),
              "dem_set_stiffness_timestepper")

    def set_peri_triax(self, goal=None, stress_mask=7, **kw):
        """Switch the stress-controlled cell on (goal: 3 values) or off
        (goal None).  Keywords: glob_update, max_strain_rate (3),
        grow_damping, max_unbalanced, abs_stress_tol, rel_stress_tol,
        stop_when_done."""
        if goal is None:
            check(self.lib.dem_set_peri_triax(self.h, None), "dem_set_peri_triax")
            return
        c = dem_peri_triax()
        self.lib.dem_peri_triax_default(C.byref(c))
        c.goal[:] = [float(g) for g in goal]
        c.stress_mask = int(stress_mask)
        for k, v in kw.items():
            if k == "max_strain_rate":
                c.max_strain_rate[:] = [float(x) for x in v]
            elif k in ("glob_update", "stop_when_done"):
                setattr(c, k, int(v))
            else:
                setattr(c, k, float(v))
        check(self.lib.dem_set_peri_triax(self.h, C.byref(c)), "dem_set_peri_triax")

    def set_peri_iso(self, stresses=None, **kw):
        """PeriIsoCompressor (keepProportions): drive the mean stress to each
        of `stresses` in turn (None switches the controller off).  Keywords:
        global_update, max_strain_rate, grow_damping, max_unbalanced,
        abs_stress_tol, rel_stress_tol, stop_when_done."""
        if stresses is None:
            check(self.lib.dem_set_peri_iso(self.h, None), "dem_set_peri_iso")
            return
        c = dem_peri_iso()
        self.lib.dem_peri_iso_default(C.byref(c))
        st = [float(x) for x in stresses]
        c.n_stresses = len(st)
        for j, x in enumerate(st[:8]):
            c.stresses[j] = x
        for k, v in kw.items():
            setattr(c, k, int(v) if k in ("global_update", "stop_when_done") else float(v))
        check(self.lib.dem_set_peri_iso(self.h, C.byref(c)), "dem_set_peri_iso")

    def get_peri_iso(self):
        st = dem_peri_iso_state()
        check(self.lib.dem_get_peri_iso(self.h, C.byref(st)), "dem_get_peri_iso")
        return {k: getattr(st, k) for k, _ in dem_peri_iso_state._fields_ if k != "pad_"}

    def get_peri_triax(self):
        st = dem_peri_triax_state()
        check(self.lib.dem_get_peri_triax(self.h, C.byref(st)), "dem_get_peri_triax")
        out = {}
        for k, _ in dem_peri_triax_state._fields_:
            v = getattr(st, k)
            out[k] = list(v) if hasattr(v, "__len__") else v
        return out

    def get_tuning(self):
        t = dem_tuning()
        check(self.lib.dem_get_tuning(self.h, C.byref(t)), "dem_get_tuning")
        return _tuning_dict(t)

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _tuning_struct(cur)
        check(self.lib.dem_set_tuning(self.h, C.byref(t)), "dem_set_tuning")

    def autotune(self, probe_steps=200, cache_path=None):
        t = dem_tuning()
        check(self.lib.dem_autotune(self.h, int(probe_steps), None if cache_path is None else cache_path.encode(),
                                    C.byref(t)), "dem_autotune")
        return _tuning_dict(t)

    def set_timing(self, on=True):
        check(self.lib.dem_set_timing(self.h, 1 if on else 0), "dem_set_timing")

    def get_timing(self, name):
        ms, n = C.c_double(), C.c_int64()
        check(self.lib.dem_get_timing(self.h, name.encode(), C.byref(ms), C.byref(n)), "dem_get_timing")
        return ms.value, n.value


class Batch:
    """Independent scenes advanced together by the same kernels."""

    def __init__(self, params_list):
        self.lib = load()
        arr = (dem_params * len(params_list))(*params_list)
        h = C.c_void_p()
        check(self.lib.dem_batch_create(len(params_list), arr, C.byref(h)), "dem_batch_create")
        self.h = h
        self.n = len(params_list)

    def scene(self, i):
        v = C.c_void_p()
        check(self.lib.dem_batch_scene(self.h, int(i), C.byref(v)), "dem_batch_scene")
        return Scene(handle=v, owner=False)

    def step(self, n=1):
        check(self.lib.dem_batch_step(self.h, int(n)), "dem_batch_step")

    def stats(self):
        s = dem_stats()
        check(self.lib.dem_batch_stats(self.h, C.byref(s)), "dem_batch_stats")
        return {k: getattr(s, k) for k, _ in dem_stats._fields_}

    def get_tuning(self):
        return self.scene(0).get_tuning()

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _tuning_struct(cur)
        check(self.lib.dem_batch_set_tuning(self.h, C.byref(t)), "dem_batch_set_tuning")

    def autotune(self, probe_steps=200, cache_path=None):
        t = dem_tuning()
        check(self.lib.dem_batch_autotune(self.h, int(probe_steps),
                                          None if cache_path is None else cache_path.encode(), C.byref(t)),
              "dem_batch_autotune")
        return _tuning_dict(t)

    def close(self):
        if self.h:
            check(self.lib.dem_batch_destroy(self.h), "dem_batch_destroy")
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
