"""MI355X-native soft-sphere DEM timestep (spheres + axis-aligned walls).

The compute path lives in ``libdem_hip.so`` (hand-written HIP for gfx950,
C ABI declared in ``include/dem.h``); ``paper_2301_00611_amd.dem`` is a thin
ctypes binding with the same names.  ``paper_2301_00611_amd.scenes`` holds
the seeded synthetic input generators.  Submodules are imported lazily so
that the generators can be used without the compiled library.
"""
import importlib

__all__ = ["dem", "scenes"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
