"""The shadow set-up (section 4, scaled) on the HIP path: a plane-parallel front
from the x = 0 face, a 1e5 K blackbody in three grey bins plus the
recombination bin (N_RC = 16: 64 packet slots per particle, one particle per
wavefront tile), a dense clump, photoheating and cooling.

Small: FP64 against the oracle (counters exact, x_HI and T within 1e-6
relative, ledger residual 1e-12) and FP32 within its bars.  Full size (128^3
particles, 134 M slots): too large for the oracle in a test, so FP32 transport
is checked against the FP64 GPU path on the same inputs (ledger residuals 1e-6
and 1e-12, totals, slab means and max |dx_HI| <= 1e-3).

With recombination radiation from outside the box (appendix B): isotropic
boundary sources on the four faces parallel to the front, switched on between
steps once the I-front has passed them, in a bin of their own; checked against
the oracle, with the cylindrical-shell profiles of the three components.

Section 4's own obstacle: the artificial barrier disk in uniform gas at
N_TC = 128, where virtual particles carry most legs; FP64 and FP32 against the
oracle at 12^3, and at the paper's 32^3 FP32 against FP64 on the GPU.
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


def small():
    return I.shadow(n_side=12, n_pp=16, n_ngb=32)


def test_shadow_small_fp64_against_oracle():
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = small()
    steps = 4
    say("shadow 12^3, G = 64, fp64,", steps, "steps")
    s = O.OracleSim(cfg)
    s.step(steps)
    ctx = RT.Context(cfg, precision="fp64")
    ctx.step(steps)
    so, sg = s.state(), ctx.state()
    say("counters oracle", so["counters"], "gpu", sg["counters"])
    assert np.array_equal(so["counters"], sg["counters"])
    assert np.array_equal(s.ngb()[0], ctx.neighbours()[0])
    assert rel(sg["xHI"], so["xHI"]) < 1e-6
    assert rel(sg["T"], so["T"]) < 1e-6
    assert np.max(so["T"]) > 2e4           # the front heated the gas
    assert np.max(residual(sg["ledger"])) < 1e-12
    assert rel(sg["ledger"][..., 0], so["ledger"][..., 0]) < 1e-12


def test_shadow_small_fp32_within_bars():
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = small()
    steps = 4
    say("shadow 12^3, G = 64, fp32,", steps, "steps")
    s = O.OracleSim(cfg)
    s.step(steps)
    ctx = RT.Context(cfg, precision="fp32")
    ctx.step(steps)
    so, sg = s.state(), ctx.state()
    dx = np.max(np.abs(sg["xHI"] - so["xHI"]))
    say("max |dx_HI|", dx, "residual", np.max(residual(sg["ledger"])))
    assert dx <= 1e-3
    assert np.max(residual(sg["ledger"])) <= 1e-6


def test_shadow_full_size_fp32_against_fp64_gpu():
    """Full size, FP32 transport against the FP64 GPU path on the same inputs.
    Photon ledgers close in both; max |dx_HI| <= 1e-3 over every particle, and
    totals and slab means agree to far below it.  The FP32 transport takes its
    cone-membership and reception-cone decisions near their thresholds in FP64
    (a guard band), so a decision flips between the precisions only through the
    FP32 rounding of the packet's own direction."""
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.config(3)
    steps = 2
    out = {}
    for prec in ("fp64", "fp32"):
        say("shadow 128^3 full size,", prec, steps, "steps")
        ctx = RT.Context(cfg, precision=prec)
        assert ctx.step(steps) == RT.RT_OK
        out[prec] = ctx.state()
        ctx.close()
        say(prec, "counters", out[prec]["counters"], "residual", np.max(residual(out[prec]["ledger"])))
    s64, s32 = out["fp64"], out["fp32"]
    assert np.max(residual(s64["ledger"])) < 1e-12
    assert np.max(residual(s32["ledger"])) < 1e-6
    assert s64["counters"][0] == s32["counters"][0] == steps
    x64, x32 = s64["xHI"], s32["xHI"]
    assert np.min(x64) < 0.5                 # the front entered the box
    d = np.abs(x32 - x64)
    say("max |dx_HI|", d.max(), "99.99% quantile", np.quantile(d, 0.9999), "beyond 1e-3", int(np.sum(d > 1e-3)))
    assert d.max() <= 1e-3
    ion64, ion32 = np.sum(1.0 - x64), np.sum(1.0 - x32)
    assert abs(ion32 - ion64) <= 1e-6 * ion64
    A64, A32 = s64["A"].sum(axis=0), s32["A"].sum(axis=0)
    lit = A64 > 0
    assert np.all(np.abs(A32[lit] - A64[lit]) <= 1e-5 * A64[lit])
    xs = cfg["pos"][:, 0] / (cfg["box"][0, 3] - cfg["box"][0, 0])
    for k in range(6):
        m = (xs >= k / 6) & (xs < (k + 1) / 6)
        assert abs(np.mean(x32[m]) - np.mean(x64[m])) <= 1e-5


def _passed(cfg, xHI):
    """Boundary sources the I-front has passed: their nearest particle is mostly ionized."""
    b = cfg["boundary"]["pos"]
    d2 = ((b[:, None, :] - cfg["pos"][None, :, :]) ** 2).sum(-1)
    return xHI[np.argmin(d2, axis=1)] < 0.5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_boundary_rr_sources_against_oracle(precision):
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.shadow_boundary(n_side=12, n_pp=16, n_bd=6, n_ngb=32)
    say("shadow with boundary sources, 12^3,", precision)
    s = O.OracleSim(cfg)
    s.step(6)
    # the switch is decided on the oracle's state and handed to both sides
    on = _passed(cfg, s.state()["xHI"])
    assert 0 < on.sum() < on.size
    src = I.boundary_sources(cfg, on)
    s.add_sources(src)
    s.step(3)
    ctx = RT.Context(cfg, precision=precision)
    ctx.step(6)
    ctx.add_sources(src)
    ctx.step(3)
    so, sg = s.state(), ctx.state()
    say("on", int(on.sum()), "of", on.size, "max |dx_HI|", np.max(np.abs(sg["xHI"] - so["xHI"])),
        "residual", np.max(residual(sg["ledger"])))
    assert np.all(so["ledger"][0, 2, 0] > 0) and so["A"][:, 2].sum() > 0
    if precision == "fp64":
        assert np.array_equal(so["counters"], sg["counters"])
        assert rel(sg["xHI"], so["xHI"]) < 1e-6
        assert rel(sg["T"], so["T"]) < 1e-6
        assert np.max(residual(sg["ledger"])) < 1e-12
        assert rel(sg["ledger"][..., 0], so["ledger"][..., 0]) < 1e-12
    else:
        assert np.max(np.abs(sg["xHI"] - so["xHI"])) <= 1e-3
        assert np.max(residual(sg["ledger"])) <= 1e-6
    # section 4's diagnostic: mean intensity in cylindrical shells around the
    # shadow's axis behind the clump, per component (source, RR from inside and
    # from outside the box)
    L = float(cfg["box"][0][3])
    g = dict(center=(0.6 * L, 0.5 * L, 0.5 * L), r_max=0.5 * L, n_shells=6, axis=(1.0, 0.0, 0.0),
             half_height=0.3 * L, mean=True)
    pg, cg = ctx.shell_profile(**g)
    po, co = O.shell_profile(cfg["pos"], so["P"], cfg["params"]["dt"], g["center"], g["r_max"], g["n_shells"],
                             axis=g["axis"], half_height=g["half_height"], mean=True)
    assert np.array_equal(cg, co)
    assert po[:, 2].max() > 0
    if precision == "fp64":
        scale = np.maximum(np.max(np.abs(po), axis=0), 1e-300)
        assert np.all(np.abs(pg - po) <= 1e-6 * scale)
    ctx.close()
    s.close()


def test_boundary_rr_sources_full_size_fp32_against_fp64_gpu():
    # section 4's size: 32^3 particles, 50^2 boundary sources per face, 100^2
    # front emitters; too large for the oracle, so FP32 transport is checked
    # against the FP64 GPU path on the same inputs and the same switch schedule
    import time
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.shadow_boundary()
    dt = cfg["params"]["dt"]
    s1, s2 = 6, 4
    on = I.boundary_schedule(cfg, s1 * dt)
    say("shadow with boundary sources, 32^3,", int(on.sum()), "of", on.size, "boundary sources on after", s1, "steps")
    assert 0 < on.sum() < on.size
    src = I.boundary_sources(cfg, on)
    out = {}
    for prec in ("fp64", "fp32"):
        ctx = RT.Context(cfg, precision=prec)
        ctx.step(s1)
        ctx.add_sources(src)
        ctx.step(1)
        import torch
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(s2 - 1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / (s2 - 1) * 1e3
        tm = ctx.timing()
        out[prec] = ctx.state()
        say(prec, f"{ms:.2f} ms/step (every launch timed) with", len(src["inst"]), "sources;",
            {k: round(v / (s2 - 1), 2) for k, v in tm.items() if k.endswith("_ms")}, "ms per step;",
            tm["hop_launches"] / (s2 - 1), "forward steps per step")
        ctx.close()
    a, b = out["fp32"], out["fp64"]
    r32, r64 = np.max(residual(a["ledger"])), np.max(residual(b["ledger"]))
    dx = np.abs(a["xHI"] - b["xHI"])
    say("residuals", r32, r64, "max |dx_HI|", dx.max())
    assert r64 < 1e-12 and r32 < 1e-6
    # the sources emit the same photons; the gas's recombination photons follow its state
    assert rel(a["ledger"][0, [0, 2], 0], b["ledger"][0, [0, 2], 0]) < 1e-12
    assert rel(a["ledger"][0, 1, 0], b["ledger"][0, 1, 0]) < 1e-5
    A32, A64 = a["A"].sum(0), b["A"].sum(0)
    assert np.all(np.abs(A32 - A64) <= 1e-5 * np.maximum(A64, 1e-300))  # absorbed per bin
    assert A64[2] > 0                                                    # the outside-box bin arrives
    assert dx.max() <= 1e-3
    assert abs(np.mean(a["xHI"]) - np.mean(b["xHI"])) < 1e-5


# --- section 4's own set-up: the artificial barrier disk at N_TC = 128 --------

def _shadow_mask(cfg):
    """Particles in the ideal shadow's core behind the disk, and well beside it."""
    L = float(cfg["box"][0][3])
    x = cfg["pos"]
    rho = np.hypot(x[:, 1] - 0.5 * L, x[:, 2] - 0.5 * L)
    return (rho < 0.12 * L) & (x[:, 0] > 0.4 * L), rho > 0.3 * L


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_barrier_shadow_against_oracle(precision):
    # the disk (radius 0.2 L at (0.27, 0.5, 0.5) L) removes every packet whose
    # leg meets it, on every kind of leg: particle to neighbour, emitter to
    # neighbour, to and from virtual particles (most legs at N_TC = 128)
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.shadow_barrier(n_side=12, n_pp=16, n_bd=6, n_ngb=32)
    say("barrier shadow 12^3, N_TC = 128,", precision)
    s = O.OracleSim(cfg)
    s.step(6)
    on = _passed(cfg, s.state()["xHI"])
    assert 0 < on.sum() < on.size
    src = I.boundary_sources(cfg, on)
    s.add_sources(src)
    s.step(3)
    ctx = RT.Context(cfg, precision=precision)
    ctx.step(6)
    ctx.add_sources(src)
    ctx.step(3)
    so, sg = s.state(), ctx.state()
    Eo, Ro = so["ledger"][0, :, 0], so["ledger"][0, :, 3]
    say("counters oracle", so["counters"], "gpu", sg["counters"], "removed/emitted", Ro[:3] / Eo[:3],
        "max |dx_HI|", np.max(np.abs(sg["xHI"] - so["xHI"])), "residual", np.max(residual(sg["ledger"])))
    assert Ro[0] > 0.02 * Eo[0] and Ro[2] > 0          # the disk removed source and outside-box photons
    sh, out = _shadow_mask(cfg)
    assert np.mean(so["xHI"][sh]) > 0.99 > 0.9 > np.mean(so["xHI"][out])   # it casts a shadow
    if precision == "fp64":
        assert np.array_equal(so["counters"], sg["counters"])
        assert rel(sg["xHI"], so["xHI"]) < 1e-6
        assert rel(sg["T"], so["T"]) < 1e-6
        assert np.max(residual(sg["ledger"])) < 1e-12
        assert rel(sg["ledger"][..., 0], so["ledger"][..., 0]) < 1e-12
        assert rel(sg["ledger"][0, :3, 3], Ro[:3]) < 1e-9           # removed
    else:
        assert np.max(np.abs(sg["xHI"] - so["xHI"])) <= 1e-3
        assert np.max(residual(sg["ledger"])) <= 1e-6
        assert rel(sg["ledger"][0, [0, 2], 3], Ro[[0, 2]]) < 1e-4
    ctx.close()
    s.close()


def test_barrier_rejects_bad_arguments_and_can_be_removed():
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.shadow_barrier(n_side=10, n_pp=12, n_bd=4, n_ngb=32, n_tc=16)
    b = cfg["barrier"]
    ctx = RT.Context(cfg, precision="fp64")
    for args in ((1, b["center"], b["radius"]), (-1, b["center"], b["radius"]), (0, b["center"], -1.0),
                 (0, b["center"], float("nan")), (0, (float("inf"), 0.0, 0.0), 1.0)):
        with pytest.raises(RT.RTError) as e:
            ctx.set_barrier(*args)
        assert e.value.status == RT.RT_EINVAL
    # radius 0 takes the disk away: the run then matches the oracle without one
    ctx.set_barrier(0, b["center"], 0.0)
    ctx.step(3)
    cfg0 = dict(cfg)
    cfg0.pop("barrier")
    s = O.OracleSim(cfg0)
    s.step(3)
    so, sg = s.state(), ctx.state()
    assert so["ledger"][0, 0, 3] == 0.0 and sg["ledger"][0, 0, 3] == 0.0
    assert np.array_equal(so["counters"], sg["counters"])
    assert rel(sg["xHI"], so["xHI"]) < 1e-6
    ctx.close()
    s.close()


def test_barrier_full_size_fp32_against_fp64_gpu():
    # section 4's run: 32^3 particles, N_TC = 128, N_RC = 8, 100^2 front
    # emitters, 50^2 boundary sources per face switched on as the front passes
    import time
    from paper_1311_0182_amd import traphic_rt as RT
    cfg = I.shadow_barrier()
    dt = cfg["params"]["dt"]
    s1, s2 = 6, 3
    on = I.boundary_schedule(cfg, s1 * dt)
    src = I.boundary_sources(cfg, on)
    say("barrier shadow 32^3, N_TC = 128:", int(on.sum()), "of", on.size, "boundary sources on after", s1, "steps")
    out = {}
    for prec in ("fp64", "fp32"):
        ctx = RT.Context(cfg, precision=prec)
        ctx.step(s1)
        ctx.add_sources(src)
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(s2)
        torch.cuda.synchronize()
        out[prec] = ctx.state()
        say(prec, f"{(time.perf_counter() - t0) / s2 * 1e3:.2f} ms/step, counters", out[prec]["counters"],
            "removed/emitted", out[prec]["ledger"][0, :3, 3] / np.maximum(out[prec]["ledger"][0, :3, 0], 1e-300))
        ctx.close()
    a, b = out["fp32"], out["fp64"]
    r32, r64 = np.max(residual(a["ledger"])), np.max(residual(b["ledger"]))
    dx = np.abs(a["xHI"] - b["xHI"])
    say("residuals", r32, r64, "max |dx_HI|", dx.max())
    assert r64 < 1e-12 and r32 < 1e-6
    assert rel(a["ledger"][0, [0, 2], 0], b["ledger"][0, [0, 2], 0]) < 1e-12
    assert rel(a["ledger"][0, [0, 2], 3], b["ledger"][0, [0, 2], 3]) < 1e-4
    assert dx.max() <= 1e-3
    sh, far = _shadow_mask(cfg)
    assert np.mean(b["xHI"][sh]) > np.mean(b["xHI"][far]) + 0.1   # the shadow lags the open front
