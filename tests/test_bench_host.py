"""Host logic of bench.py that needs no GPU: the one-GPU guard and the rule that
measured HBM traffic is reported only for the kernel sources it was taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_measured_kernel_sources(tmp_path, monkeypatch):
    import bench
    sha = bench.kernel_sources_sha()
    good = tmp_path / "good.md"
    good.write_text(f"kernel_sources_sha256: {sha}\ntraffic_bytes_per_launch: 123456\n")
    stale = tmp_path / "stale.md"
    stale.write_text("kernel_sources_sha256: 0000000000000000\ntraffic_bytes_per_launch: 123456\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic() == 123456.0
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None

