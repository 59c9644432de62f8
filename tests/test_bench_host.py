"""Host-side parts of bench.py (no GPU): the one-GPU guard, and how
roofline.traffic is taken from a committed counter summary only while the
kernel's sources still hash to the value recorded beside the counters."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _summary(tmp_path, sha):
    line = ("counter-summary: kernel=k_wave_flat workload=w precision=fp64 fetch_bytes=1000 write_bytes=24 "
            f"sources=device.hpp,krylov_tiled.hpp sha256_16={sha}\n")
    (tmp_path / "k.md").write_text("# a profile\n\n" + line)


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    good = bench.sources_hash(["device.hpp", "krylov_tiled.hpp"])
    _summary(tmp_path, good)
    tr = bench.measured_traffic("k_wave_flat", "w", "fp64")
    assert tr == {"bytes_per_launch": 1024, "source": os.path.relpath(str(tmp_path / "k.md"), ROOT)}
    # another workload, precision or kernel has no summary
    assert bench.measured_traffic("k_wave_flat", "w", "fp32_mixed") is None
    assert bench.measured_traffic("k_bellman_wave", "w", "fp64") is None
    # counters taken from other sources are not reported
    _summary(tmp_path, "0" * 16)
    assert bench.measured_traffic("k_wave_flat", "w", "fp64") is None


@pytest.mark.parametrize("names", [["device.hpp"], ["device.hpp", "kernels_bellman.hip"]])
def test_source_hash_depends_on_every_file(names):
    h = bench.sources_hash(names)
    assert len(h) == 16 and h != bench.sources_hash(names[:1] + ["krylov.hpp"])
