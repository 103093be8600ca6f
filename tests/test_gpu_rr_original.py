"""The predecessor scheme of emitting recombination radiation (section 2.2) on
the HIP path: every particle with recombination photons emits them like a
point source, through N_EC emission cones rotated per particle and emission
sub-step, into its own neighbours; empty cones become virtual particles.

Against the oracle's same scheme: FP64 with exact counters and x_HI, T within
1e-6; FP32 within its bars; with several emission sub-steps and with the
barrier disk.  At the 64^3 Stromgren size, FP32 against the FP64 GPU path, and
the two schemes side by side (section 2.2: nearly the same ionization state,
the same RR photons emitted).
"""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_0182_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def residual(led):
    E, A, X, R, F = np.moveaxis(led, -1, 0)
    return np.abs(E - A - X - R - F) / np.maximum(E, 1e-300)


def rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def _cfg(n_em=10, **kw):
    cfg = I.stromgren(12, rr=True, n_ngb=32, dt_myr=0.5, n_em=n_em, **kw)
    cfg["params"]["recomb_mode"] = I.RR_ORIGINAL
    return cfg


@pytest.mark.parametrize("precision,n_em", [("fp64", 10), ("fp64", 1), ("fp32", 10)])
def test_rr_original_against_oracle(precision, n_em):
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = _cfg(n_em)
    steps = 8
    say("predecessor RR scheme, Stromgren 12^3,", precision, "n_em", n_em)
    s = O.OracleSim(cfg)
    s.step(steps)
    ctx = RT.Context(cfg, precision=precision)
    ctx.step(steps)
    so, sg = s.state(), ctx.state()
    say("counters oracle", so["counters"], "gpu", sg["counters"], "RR emitted", so["ledger"][0, 1, 0],
        "max |dx_HI|", np.max(np.abs(sg["xHI"] - so["xHI"])), "residual", np.max(residual(sg["ledger"])))
    assert so["ledger"][0, 1, 0] > 0 and so["A"][:, 1].sum() > 0     # RR photons emitted and absorbed
    if precision == "fp64":
        assert np.array_equal(so["counters"], sg["counters"])
        assert rel(sg["xHI"], so["xHI"]) < 1e-6
        assert rel(sg["T"], so["T"]) < 1e-6
        assert np.max(residual(sg["ledger"])) < 1e-12
        assert rel(sg["ledger"][..., 0], so["ledger"][..., 0]) < 1e-12
        lit = so["A"] > 1e-12 * so["A"].max()
        assert rel(sg["A"][lit], so["A"][lit]) < 1e-6
    else:
        assert np.max(np.abs(sg["xHI"] - so["xHI"])) <= 1e-3
        assert np.max(residual(sg["ledger"])) <= 1e-6
    ctx.close()
    s.close()


def test_rr_original_with_barrier_against_oracle():
    # the disk removes legs of the particles' own emission and of their
    # virtual particles too
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = _cfg(2)
    L = float(cfg["box"][0][3])
    cfg["barrier"] = dict(inst=0, center=np.array([0.3, 0.5, 0.5]) * L, radius=0.25 * L)
    steps = 6
    s = O.OracleSim(cfg)
    s.step(steps)
    ctx = RT.Context(cfg, precision="fp64")
    ctx.step(steps)
    so, sg = s.state(), ctx.state()
    say("predecessor RR + barrier: counters", so["counters"], sg["counters"], "removed RR",
        so["ledger"][0, 1, 3], sg["ledger"][0, 1, 3])
    assert so["ledger"][0, 1, 3] > 0
    assert np.array_equal(so["counters"], sg["counters"])
    assert rel(sg["xHI"], so["xHI"]) < 1e-6
    assert np.max(residual(sg["ledger"])) < 1e-12
    assert rel(sg["ledger"][0, :, 3], so["ledger"][0, :, 3]) < 1e-9
    ctx.close()
    s.close()


def test_rr_schemes_side_by_side_full_size():
    # 64^3 Stromgren with RR (262,144 particles, 10 emission sub-steps): the
    # predecessor scheme in FP32 against FP64 on the GPU, and both schemes'
    # cost per RT step on the same steps
    import torch
    from paper_1311_0182_amd import traphic_rt as RT
    base = I.config(2)
    W, K = 3, 4
    out = {}
    for mode in (I.RR_TRANSPORT, I.RR_ORIGINAL):
        for prec in ("fp64", "fp32"):
            cfg = dict(base)
            cfg["params"] = dict(base["params"], recomb_mode=mode)
            ctx = RT.Context(cfg, precision=prec)
            ctx.step(W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.step(K)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / K * 1e3
            out[(mode, prec)] = ctx.state()
            say("mode", mode, prec, f"{ms:.2f} ms/step", "counters", out[(mode, prec)]["counters"],
                "residual", np.max(residual(out[(mode, prec)]["ledger"])))
            ctx.close()
    a, b = out[(I.RR_ORIGINAL, "fp32")], out[(I.RR_ORIGINAL, "fp64")]
    assert np.max(residual(b["ledger"])) < 1e-12 and np.max(residual(a["ledger"])) < 1e-6
    assert np.max(np.abs(a["xHI"] - b["xHI"])) <= 1e-3
    # the schemes: RR photons emitted agree closely, ionization nearly the same
    t = out[(I.RR_TRANSPORT, "fp64")]
    assert abs(t["ledger"][0, 1, 0] / b["ledger"][0, 1, 0] - 1) < 1e-2
    assert np.max(np.abs(t["xHI"] - b["xHI"])) < 0.05
