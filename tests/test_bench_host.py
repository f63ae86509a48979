"""Host logic of bench.py that needs no GPU: the one-GPU guard and the
gating of the stored profiler figures on the kernel sources, the tile
variant, the domain and the state form."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_figures_follow_the_kernel_sources(monkeypatch):
    m = dict(bench.MEASURED_TRAFFIC)
    here = bench.kernel_source_hash()
    monkeypatch.setitem(m, "source_sha256", here)
    v, nx, ny = m["variant"], m["nx"], m["ny"]
    assert bench.measured_for(m, "bytes_per_launch", v, nx, ny) == m["bytes_per_launch"]
    assert bench.measured_for(m, "bytes_per_launch", "tile8x8_t128", nx, ny) is None
    assert bench.measured_for(m, "bytes_per_launch", v, nx // 2, ny) is None
    assert bench.measured_for(m, "bytes_per_launch", v, nx, ny, storage=1) is None
    monkeypatch.setitem(m, "source_sha256", "0" * 16)
    assert bench.measured_for(m, "bytes_per_launch", v, nx, ny) is None


def test_valu_ceiling_constant():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, no packed float32
    assert bench.VALU_ISSUE_PEAK == pytest.approx(39.3216e12)
    assert bench.MEASURED_VALU["source_sha256"] == bench.MEASURED_TRAFFIC["source_sha256"]
