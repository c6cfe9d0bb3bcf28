"""C-ABI checks that need no GPU: the library is built, loads, exports every
function include/dem.h declares, and the ctypes structures match the C
layouts (checked against a tiny C program compiled from the header).
No call here touches the HIP runtime."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "dem.h")
LIB = os.path.join(ROOT, "paper_2301_00611_amd", "libdem_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_]+)\s*\(", text)))


def test_library_built():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (dem_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_header():
    from paper_2301_00611_amd import dem
    assert sorted(dem.SIGNATURES) == declared_functions()


def test_pure_host_calls():
    from paper_2301_00611_amd import dem
    lib = dem.load()
    assert lib.dem_abi_version() == 1
    p = dem.dem_params()
    lib.dem_params_default(ctypes.byref(p))
    assert p.damping == 0.2 and p.verlet_dist == -0.5 and p.homo_deform == 2 and p.damp_rot == 1
    assert p.precision == dem.DEM_FP64 and p.track_energy == 0 and list(p.hsize) == [1, 0, 0, 0, 1, 0, 0, 0, 1]
    assert isinstance(lib.dem_last_error(), bytes)


LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "dem.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("dem_params %zu\ndem_contact %zu\ndem_history %zu\ndem_energy %zu\ndem_stats %zu\n",
         sizeof(dem_params), sizeof(dem_contact), sizeof(dem_history), sizeof(dem_energy), sizeof(dem_stats));
  printf("dem_peri_triax %zu\ndem_peri_triax_state %zu\ndem_peri_iso %zu\ndem_peri_iso_state %zu\n",
         sizeof(dem_peri_triax), sizeof(dem_peri_triax_state), sizeof(dem_peri_iso), sizeof(dem_peri_iso_state));
  P(dem_energy, visc_dissip); P(dem_peri_iso, stresses); P(dem_peri_iso, max_strain_rate);
  P(dem_peri_iso, stop_when_done); P(dem_peri_iso_state, sigma); P(dem_peri_iso_state, updates);
  P(dem_peri_iso_state, active);
  P(dem_params, verlet_dist); P(dem_params, precision); P(dem_params, hsize); P(dem_params, homo_deform);
  P(dem_params, stream); P(dem_contact, normal); P(dem_contact, kn); P(dem_history, fs); P(dem_stats, coordination);
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    from paper_2301_00611_amd import dem
    src = tmp_path / "probe.c"
    src.write_text(LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    lines = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    assert int(lines["dem_params"]) == ctypes.sizeof(dem.dem_params)
    assert int(lines["dem_contact"]) == ctypes.sizeof(dem.dem_contact)
    assert int(lines["dem_history"]) == ctypes.sizeof(dem.dem_history)
    assert int(lines["dem_energy"]) == ctypes.sizeof(dem.dem_energy)
    assert int(lines["dem_stats"]) == ctypes.sizeof(dem.dem_stats)
    for name in ("dem_peri_triax", "dem_peri_triax_state", "dem_peri_iso", "dem_peri_iso_state"):
        assert int(lines[name]) == ctypes.sizeof(getattr(dem, name)), name
    for key, val in lines.items():
        if "." in key:
            cls, field = key.split(".")
            assert getattr(getattr(dem, cls), field).offset == int(val), key


def test_missing_library_fails_loudly(tmp_path):
    from paper_2301_00611_amd import dem
    with pytest.raises(ImportError):
        dem._lib_backup = dem._lib
        try:
            dem._lib = None
            dem.load(str(tmp_path / "absent.so"))
        finally:
            dem._lib = dem._lib_backup
