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



def test_dense_model_bytes_per_slot_update():
    """The dense forward-step model bench.py prices the roofline with gives the
    bytes per slot update of the workloads' table: 69 / 111 B (64^3 RR and the
    batch, FP32 / FP64) and 48 / 90 B (128^3 shadow set-up)."""
    import bench
    from paper_1311_0182_amd import inputs as I
    for k, f32, want in ((2, True, 69), (2, False, 111), (4, True, 69), (4, False, 111), (3, True, 48),
                         (3, False, 90)):
        cfg = I.config(k)
        total, per_slot, slots = bench.dense_bytes_per_hop(cfg, f32)
        assert abs(per_slot - want) < 0.6, (k, f32, per_slot)
        assert slots == cfg["pos"].shape[0] * cfg["params"]["n_rc"] * cfg["params"]["n_freq"]
