"""Host-side logic of bench.py (no GPU): the one-GPU rule, the profile
traffic lookup that must go stale when a kernel source changes, and the
seeded medoid pair list."""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def _profile(tmp_path, src_text, sha=None, traffic=12345):
    src = tmp_path / "kern.hip"
    src.write_text(src_text)
    digest = sha or hashlib.sha256(src_text.encode()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / "lab_test.md").write_text(
        "# t\n\nkernel_sources: kern.hip\nkernel_source_sha256: %s\n\ntraffic_bytes_per_launch: %d\n" % (digest, traffic))
    return src


def test_recorded_traffic_tracks_the_kernel_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = _profile(tmp_path, "kernel v1\n")
    assert bench.recorded_traffic("lab") == 12345
    src.write_text("kernel v2\n")  # the kernel changed after the counters were taken
    assert bench.recorded_traffic("lab") is None
    assert bench.recorded_traffic("other") is None


def test_recorded_traffic_needs_all_fields(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _profile(tmp_path, "k\n", sha="0" * 64)
    assert bench.recorded_traffic("lab") is None


def test_medoid_pairs_are_seeded_and_complete():
    p = bench.medoid_pairs(100, 10)
    q = bench.medoid_pairs(100, 10)
    assert np.array_equal(p, q)
    assert p.shape == (1000, 2)
    medoids = np.unique(p[:, 1])
    assert len(medoids) == 10
    for m in medoids:
        assert np.array_equal(np.sort(p[p[:, 1] == m, 0]), np.arange(100))
