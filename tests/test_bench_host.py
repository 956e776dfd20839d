"""Host-side logic of bench.py (no GPU): the one-GPU guard and the counter
traffic it reports only for the kernel source the counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _summary(tmp_path, sha):
    p = tmp_path / "push_kernel_x_pmc.txt"
    p.write_text("# header: not a key\n"
                 "kernel: push_kernel<float>\n"
                 f"kernel_source_sha256_16: {sha}\n"
                 "fetch_bytes_per_launch: 1000\n"
                 "write_bytes_per_launch: 234\n")
    return str(tmp_path / "push_kernel_{}_pmc.txt")


def test_traffic_is_reported_for_the_measured_source_only(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_FILE", _summary(tmp_path, bench.kernel_sha()))
    assert bench.pmc_traffic("x") == 1234.0
    monkeypatch.setattr(bench, "PMC_FILE", _summary(tmp_path, "0" * 16))
    assert bench.pmc_traffic("x") is None
    assert bench.pmc_traffic("missing") is None

