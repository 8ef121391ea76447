"""Host logic of bench.py (no GPU): the one-GPU contract and the lookup of
the profiled HBM traffic, which must be dropped (null) once the kernel
source, the tile or the workload differ from what the counters measured."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def _profile(tmp_path, sha, tile="16x16x16", traffic="2.5e9"):
    p = tmp_path / "profile.md"
    p.write_text("# summary\n\n    kernel_source_sha256_prefix: %s\n    tile: %s\n"
                 "    traffic_bytes_per_launch: %s\n" % (sha, tile, traffic))
    return str(p)


def test_profiled_traffic_follows_source_tile_and_workload(tmp_path, monkeypatch):
    with open(bench.KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    tile = dict(tx=16, ty=16, zchunk=16)
    monkeypatch.setattr(bench, "PROFILE", _profile(tmp_path, sha))
    assert bench.profiled_traffic(tile, 256, "f32") == pytest.approx(2.5e9)
    # another tile, grid, precision or kernel source: not what was measured
    assert bench.profiled_traffic(dict(tile, zchunk=32), 256, "f32") is None
    assert bench.profiled_traffic(tile, 512, "f32") is None
    assert bench.profiled_traffic(tile, 256, "f64") is None
    assert bench.profiled_traffic(None, 256, "f32") is None
    monkeypatch.setattr(bench, "PROFILE", _profile(tmp_path, "0" * 16))
    assert bench.profiled_traffic(tile, 256, "f32") is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic(tile, 256, "f32") is None


def test_committed_profile_is_readable():
    """The committed FP32 summary carries the three fields the lookup reads."""
    fields = {}
    with open(bench.PROFILE) as f:
        for line in f:
            k, _, v = line.strip().partition(": ")
            if v:
                fields[k] = v
    assert len(fields["kernel_source_sha256_prefix"]) == 16
    assert fields["tile"].count("x") == 2
    assert 1e9 < float(fields["traffic_bytes_per_launch"]) < 1e10
