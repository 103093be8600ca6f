"""The large clustered workload on the HIP path: equal-mass particles sampled
from a lognormal density, many point sources at the densest particles, a 1e5 K
blackbody in four grey bins plus the recombination bin (three empty bins pad a
particle's packet slots to one wavefront), N_TC = N_EC = 32, photoheating and
cooling from 100 K.

Small (16^3 in a 20 kpc box, 16 sources, where the sources ionize within the
test's steps): FP64 against the oracle (counters exact) and FP32 within its
bars.  128^3 in a 160 kpc box (the same particle spacing): FP32 against the
FP64 GPU path.  The full 256^3 field in its 10 Mpc box is a bench row.
"""
import sys

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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_clustered_small_against_oracle(precision):
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.clustered(n_side=16, n_src=16, box_mpc=0.02)
    steps = 10
    s = O.OracleSim(cfg)
    s.step(steps)
    so = s.state()
    assert so["xHI"].min() < 0.5 and so["T"].max() > 1e4      # the sources ionize and heat
    ctx = RT.Context(cfg, precision=precision)
    ctx.step(steps)
    sg = ctx.state()
    say("clustered 16^3", precision, "counters", so["counters"], sg["counters"], "max |dx_HI|",
        np.max(np.abs(sg["xHI"] - so["xHI"])), "residual", np.max(residual(sg["ledger"])))
    if precision == "fp64":
        assert np.array_equal(so["counters"], sg["counters"])
        assert rel(sg["xHI"], so["xHI"]) < 1e-6
        assert rel(sg["T"], so["T"]) < 1e-6
        assert np.max(residual(sg["ledger"])) < 1e-12
        assert rel(sg["ledger"][..., 0], so["ledger"][..., 0]) < 1e-12
    else:
        assert np.max(np.abs(sg["xHI"] - so["xHI"])) <= 1e-3
        assert np.max(residual(sg["ledger"])) <= 1e-6
    ctx.close()
    s.close()


def test_clustered_128_fp32_against_fp64_gpu():
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.clustered(n_side=128, box_mpc=0.16)
    steps = 3
    out = {}
    for prec in ("fp64", "fp32"):
        ctx = RT.Context(cfg, precision=prec)
        assert ctx.step(steps) == RT.RT_OK
        out[prec] = ctx.state()
        say("clustered 128^3", prec, "counters", out[prec]["counters"], "residual",
            np.max(residual(out[prec]["ledger"])))
        ctx.close()
    a, b = out["fp32"], out["fp64"]
    dx = np.abs(a["xHI"] - b["xHI"])
    say("max |dx_HI|", dx.max(), "min x_HI", b["xHI"].min())
    assert np.max(residual(b["ledger"])) < 1e-12 and np.max(residual(a["ledger"])) < 1e-6
    assert b["xHI"].min() < 0.9                  # the sources ionize something
    assert dx.max() <= 1e-3
    assert rel(a["ledger"][0, :4, 0], b["ledger"][0, :4, 0]) < 1e-12   # the sources emit the same
