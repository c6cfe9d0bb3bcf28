"""FP64 reference oracle for the DEM timestep (test infrastructure only).

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.
"""
from .oracle import OracleScene, load_library  # noqa: F401
