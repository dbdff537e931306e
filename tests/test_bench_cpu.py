"""CPU checks of the benchmark script's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.committed_traffic("varcoef") is None
    (tmp_path / "assemble_varcoef_hbm.txt").write_text(f"source_sha256: {h}\nhbm_bytes_per_launch: 1.5e+08\n")
    assert bench.committed_traffic("varcoef") == 1.5e8
    (tmp_path / "assemble_varcoef_hbm.txt").write_text("source_sha256: 0000000000000000\nhbm_bytes_per_launch: 1.5e+08\n")
    assert bench.committed_traffic("varcoef") is None


def test_algorithmic_op_counts_are_stated_for_every_family():
    for kind in ("poisson", "varcoef", "amplitude", "lut"):
        assert bench.ALG_OPS[kind] > 50 and bench.FP32_FLOP[kind] > 0
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
