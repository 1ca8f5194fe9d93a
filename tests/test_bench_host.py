"""Host-side checks of bench.py: the one-GPU guard and the reading of the
committed HBM-traffic summary (no GPU needed)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _sha(src):
    path = os.path.join(ROOT, "paper_1707_00023_amd", "csrc", src)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def test_traffic_is_ratio_times_this_runs_bytes(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    f.write_text("text\n"
                 f"    traffic_ratio k_gemm_cols 1.2500 source_sha256_16 {_sha('kry_block.hip')}\n"
                 f"    traffic_ratio k_stencil_axpby 1.1000 source_sha256_16 0000000000000000\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("block_gemm", "c2", 4.0e9) == pytest.approx(5.0e9)
    # the summary names another build of the kernel: no figure
    assert bench.measured_traffic("operator", "c2", 1.0e9) is None
    # not in the summary, or another workload: no figure
    assert bench.measured_traffic("block_gram", "c2", 1.0e9) is None
    assert bench.measured_traffic("block_gemm", "c5", 1.0e9) is None
    assert bench.measured_traffic("combine", "c2", 1.0e9) is None
