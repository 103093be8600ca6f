"""The seeded input generators: shapes, and the slicing of a batch into its
instances (data movement only)."""
import numpy as np

from paper_1311_0182_amd import inputs as I


def test_instances_partition_the_batch():
    cfg = I.batched(n_inst=5, side_lo=6, side_hi=10, n_ngb=32, n_steps=3)
    parts = [I.instance(cfg, k) for k in range(5)]
    for key in ("pos", "nH", "NH", "xHI", "T"):
        assert np.array_equal(np.concatenate([p[key] for p in parts]), cfg[key])
    for k, p in enumerate(parts):
        n = int(cfg["inst_off"][k + 1] - cfg["inst_off"][k])
        assert list(p["inst_off"]) == [0, n]
        assert np.array_equal(p["box"][0], cfg["box"][k])
        sel = cfg["sources"]["inst"] == k
        assert np.all(p["sources"]["inst"] == 0)
        assert np.array_equal(p["sources"]["pos"], cfg["sources"]["pos"][sel])
        assert np.array_equal(p["sources"]["rate"], cfg["sources"]["rate"][sel])
        assert p["params"] == cfg["params"]
        lo, hi = p["box"][0, :3], p["box"][0, 3:]
        assert np.all(p["pos"] >= lo) and np.all(p["pos"] <= hi)
    assert sum(len(p["sources"]["inst"]) for p in parts) == len(cfg["sources"]["inst"])
