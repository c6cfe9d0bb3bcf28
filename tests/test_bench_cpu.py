"""Host logic of bench.py that needs no GPU: the algorithmic byte model of
the contact kernel (the per-unit figures of the survey's byte table), the
reading of a committed counter summary (a figure is used only while the
kernel's sources are the ones it was taken on), and the refusal of more
than one GPU."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_contact_bytes_per_unit():
    # FP64: 80 B per body gathered once, 104 B per touching pair (ids 8,
    # shear force r/w 48, previous normal r/w 48), 8 B per other candidate
    assert bench.contact_algorithmic_bytes(0, 1, 0, 0) == 80
    assert bench.contact_algorithmic_bytes(0, 0, 1, 1) == 104
    assert bench.contact_algorithmic_bytes(0, 0, 0, 1) == 8
    # FP32-mixed: the previous normal in FP32, 80 B per touching pair
    assert bench.contact_algorithmic_bytes(1, 0, 1, 1) == 80
    # more contacts than candidates never yields negative candidate bytes
    assert bench.contact_algorithmic_bytes(0, 10, 7, 5) == 800 + 7 * 104
    n, c, cand = 8_000_000, 17_000_000, 33_000_000
    assert bench.contact_algorithmic_bytes(0, n, c, cand) == 80 * n + 104 * c + 8 * (cand - c)


def _profile(tmp_path, kernel, digest, value=123456789):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    (d / "p.md").write_text(f"# x\n\ntraffic_bytes_per_launch {kernel} precision 0 {value} "
                            f"source_sha256_16 {digest}\n")


def test_traffic_used_only_on_the_profiled_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: "00aa11bb22cc33dd")
    assert bench.profiled_traffic("k_contact", "p") is None  # no summary
    _profile(tmp_path, "k_contact", "00aa11bb22cc33dd")
    assert bench.profiled_traffic("k_contact", "p") == 123456789.0
    assert bench.profiled_traffic("k_contact", "p", precision=1) is None  # not profiled
    assert bench.profiled_traffic("k_integrate", "p") is None
    _profile(tmp_path, "k_contact", "ffffffffffffffff")  # taken on other sources
    assert bench.profiled_traffic("k_contact", "p") is None


def test_source_hash_covers_the_shared_header(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2301_00611_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "contact.hip").write_text("kernel")
    (csrc / "dem_internal.hpp").write_text("layout")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash("k_contact")
    (csrc / "dem_internal.hpp").write_text("layout changed")
    assert bench.kernel_source_hash("k_contact") != h0
    (csrc / "dem_internal.hpp").write_text("layout")
    assert bench.kernel_source_hash("k_contact") == h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
