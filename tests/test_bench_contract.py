"""Host-side parts of the benchmark contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stored_traffic_requires_matching_sources_and_tile(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    name = prof / "traffic_k_pipe_sub2_fp64_512cubed.txt"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for f in bench.KERNEL_SOURCES:
        d = tmp_path / os.path.dirname(f)
        d.mkdir(parents=True, exist_ok=True)
        (tmp_path / f).write_text("kernel source " + f)
    h = bench.kernel_source_hash()
    name.write_text(f"# header\nsource_sha256: {h}\ntile: 16x8x8/2+ring\ntraffic_bytes_per_launch: 1.5e10\n")
    assert bench.stored_traffic(8, 512, "16x8x8/2+ring") == 1.5e10
    assert bench.stored_traffic(8, 512, "32x4x4/1+ring") is None      # other tile
    assert bench.stored_traffic(4, 512, "16x8x8/2+ring") is None      # no FP32 file
    (tmp_path / bench.KERNEL_SOURCES[0]).write_text("changed")
    assert bench.stored_traffic(8, 512, "16x8x8/2+ring") is None      # kernel changed
