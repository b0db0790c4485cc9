"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that the HBM byte
count of the main kernel is reported only when its counter summary was taken on the current
kernel source."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_main_cfg3_eps1e-06_hbm_bytes.txt").write_text(
        "# comment: ignored\nhbm_bytes_per_launch: 1.5e+13\nkernel_source_sha256: abc123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc123")
    assert bench.measured_traffic(1e-6) == 1.5e13
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "changed")
    assert bench.measured_traffic(1e-6) is None
    assert bench.measured_traffic(1e-4) is None  # no summary for this workload


def test_kernel_source_digest_covers_the_main_kernel_sources():
    d = bench.kernel_source_digest()
    assert len(d) == 64 and int(d, 16) >= 0
