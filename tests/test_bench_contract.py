"""CPU checks of bench.py's contract pieces that need no GPU: the one-GPU
refusal, and the lookup of counter figures in the committed profile
summaries, which is void once the kernel sources change."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("digest_ok", [True, False])
def test_counter_figures_follow_the_source_digest(tmp_path, monkeypatch, digest_ok):
    d = bench.source_digest() if digest_ok else "0" * 16
    f = tmp_path / "counters.md"
    f.write_text(f"text\nsource_digest: {d}\nhbm_bytes_per_launch[fp32]: 3.6e9\n"
                 f"valu_lane_ops_per_cell[mom32_256]: 450.0\n")
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    monkeypatch.setattr(bench, "MOM_COUNTERS_FILE", str(f))
    if digest_ok:
        assert bench.measured_traffic("fp32") == 3.6e9
        r = bench.alu_roofline(256, 50.0)
        assert r["bound"] == "alu" and r["valu_lane_ops_per_cell"] == 450.0
        assert abs(r["frac"] - 450.0 * 50e9 / bench.VALU_PEAK_LANE_OPS) < 1e-4
        assert bench.measured_traffic("fp16") is None  # no figure for that key
    else:
        assert bench.measured_traffic("fp32") is None
        assert bench.alu_roofline(256, 50.0) is None
