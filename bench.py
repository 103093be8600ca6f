"""Benchmark of one TRAPHIC RT step with recombination radiation on one MI355X.

Headline workload (the metric's own): the batched HII regions, 64 independent
instances of 512..97,336 particles (1.36 M in all) in the same launches,
recombination radiation transported (N_ngb = 48, N_TC = N_RC = N_EC = 8, a
source bin and an RR bin, dt = 0.1 Myr).  A step is one RT step of every
instance: emission, all forward steps until no packet moves, chemistry, RR
emission and the photon ledger.

  value     particle-packet updates/s of the FP32-transport run (forward steps
            replayed from captured graphs), W warm-up steps then K timed; the
            work is the packet updates of the FP64 run over the same steps.
            The forward step's launch configuration is the one the library's
            autotuner picks in an untimed pass over the same W + K steps (per
            precision); the timed runs start with it fixed.
  accuracy  the FP32 and FP64 runs side by side over the same W + K steps:
            max |dx_HI| after every step, which must stay <= 1e-3 (the bar);
            the ledger residuals.  If the bar is missed, value is 0 and the
            measured rate is kept under "value_bar_missed".
  roofline  the forward-step kernel k_hop<float>: its launches timed with HIP
            events on the library's stream (a separate run with per-launch
            events); algorithmic bytes per launch = the dense model's bytes per
            slot update (every slot, edge list and per-particle datum of a
            forward step touched once, divided by the slots) x the active packet
            updates per launch.  The kernel's own device-counted bytes and the
            dense bytes per forward step are given beside it.  traffic: HBM
            bytes per launch from hardware counters (profiles/), if they were
            taken on the current kernel sources.

Extra rows: the 64^3 Stromgren workload (FP32 vs FP64), the two schemes of
emitting recombination radiation on it (section 2.2), the 256^3 clustered field
(FP32 only: its FP64 state would not fit beside it), the 128^3 shadow
set-up (three blackbody bins + RR, N_TC = N_RC = N_EC = 16, heating and
cooling; FP32 vs FP64), the batch solved one instance at a time in FP64, the
intensity-profile diagnostic and the CPU oracle (the baseline, not the
target).  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DX_BAR = 1e-3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_hop_float_batched64_hbm_bytes.md")


def kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("rt_kernels.hpp", "rt_device.hpp"):
        with open(os.path.join(ROOT, "paper_1311_0182_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per forward-step launch on the headline window from the
    committed counter summary, valid only for the kernel sources measured."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    sha = re.search(r"kernel_sources_sha256:\s*([0-9a-f]+)", txt)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9]+)", txt)
    if not sha or not val or sha.group(1) != kernel_sources_sha():
        return None
    return float(val.group(1))


def dense_bytes_per_hop(cfg, fp32):
    """The dense model of one forward step: every packet slot read and written
    (photons, direction, clock: 20 B in FP32, 40 B in FP64), a one-byte cone
    count per slot, and per particle its forward and reverse neighbour lists
    (8 N_ngb B), position (24 B), x_HI n_H (8 B) and absorbed/passing photons
    read and written (4 N_freq s, s the transport's float size)."""
    p = cfg["params"]
    n = int(cfg["pos"].shape[0])
    k, nf = int(p["n_ngb"]), int(p["n_freq"])
    slots = n * int(p["n_rc"]) * nf
    s = 4 if fp32 else 8
    per_slot = 2 * 5 * s + 1
    per_particle = 8 * k + 24 + 8 + 4 * nf * s
    total = slots * per_slot + n * per_particle
    return total, total / slots, slots


FORCE_SHAPE = -1   # --hop-shape
CLUSTERED_LABEL = ("256^3 clustered field (16.8 M particles from a lognormal density in a 10 Mpc box, 1024 "
                   "sources, 4 blackbody bins + RR padded to 8, N_ngb=48, N_TC=N_EC=32, N_RC=8, heating and cooling)")


def tuned_shape(cfg, steps, precision="fp32"):
    """The library's autotuner run over the same workload in an untimed
    pass (steps RT steps, at least 3; if the tuner has not finished by the last
    3 of them, it is made to time the configurations on those 3, the number of
    RT steps it times them over).  Returns rt_get_hop_shape's report; the
    timed runs then use the chosen one."""
    from paper_1311_0182_amd import traphic_rt as RT
    if FORCE_SHAPE >= 0:
        return dict(shape=FORCE_SHAPE, tuned=False, ms_per_launch=[0.0] * 6)
    ctx = RT.Context(cfg, precision=precision)
    ctx.step(max(0, steps - 3))
    if not ctx.hop_shape()["tuned"]:
        ctx.set_hop_shape(-2)
        ctx.step(3)
    out = ctx.hop_shape()
    ctx.close()
    return out


def run_timed(cfg, precision, W, K, timing=False, shape=None, step_graphs=False):
    import torch
    from paper_1311_0182_amd import traphic_rt as RT
    ctx = RT.Context(cfg, precision=precision)
    if FORCE_SHAPE >= 0:
        shape = FORCE_SHAPE
    if shape is not None:
        ctx.set_hop_shape(shape)
    if step_graphs:
        ctx.set_step_graphs(True)
    if W:
        ctx.step(W)
    s0 = ctx.state()
    ctx.set_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(K)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = ctx.state()
    out = dict(t=t, updates=int(st["counters"][3] - s0["counters"][3]),
               hops=int(st["counters"][1] - s0["counters"][1]), state=st, shape=ctx.hop_shape(),
               timing=ctx.timing() if timing else None, ctx=ctx)
    return out


def side_by_side(cfg, steps):
    """FP32 and FP64 runs stepped together: max |dx_HI| after every step."""
    import numpy as np
    from paper_1311_0182_amd import traphic_rt as RT
    a, b = RT.Context(cfg, precision="fp32"), RT.Context(cfg, precision="fp64")
    if FORCE_SHAPE >= 0:
        a.set_hop_shape(FORCE_SHAPE)
        b.set_hop_shape(FORCE_SHAPE)
    worst, at = 0.0, 0
    res32 = res64 = 0.0
    for k in range(steps):
        a.step(1)
        b.step(1)
        sa, sb = a.state(), b.state()
        d = float(np.max(np.abs(sa["xHI"] - sb["xHI"])))
        if d > worst:
            worst, at = d, k + 1
        res32 = max(res32, residual(sa["ledger"]))
        res64 = max(res64, residual(sb["ledger"]))
    a.close()
    b.close()
    return dict(max_abs_dx_HI=worst, at_step=at, steps_checked=steps, bar=DX_BAR, met=worst <= DX_BAR,
                ledger_residual_fp32=res32, ledger_residual_fp64=res64)


def residual(led):
    import numpy as np
    E, A, X, R, F = np.moveaxis(led, -1, 0)
    return float(np.max(np.abs(E - A - X - R - F) / np.maximum(E, 1e-300)))


def cpu_baseline(cfg, budget_s):
    """The FP64 oracle (single thread) on the headline workload from step 0,
    for as many whole steps as fit in the budget."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    s = O.OracleSim(cfg)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    steps = 0
    while True:
        s.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 50:
            break
    dt = time.perf_counter() - t0
    upd = int(s.state()["counters"][3])
    s.close()
    return dict(value=upd / dt, unit="particle-packet updates/s", cores=1, kind="oracle",
                sample=f"first {steps} steps of the same batched workload ({upd} packet updates, {dt:.1f} s; "
                       f"neighbour search {t_init:.1f} s not counted)")


def shell_profile_timing(ctx, cfg, reps=50):
    """The intensity-profile diagnostic: wall time per call (stream sync, two
    fills, the kernel and the copy of the histogram back included)."""
    import numpy as np
    box = np.asarray(cfg["box"][0], dtype=float)
    L = float(box[3] - box[0])
    src = np.asarray(cfg["sources"]["pos"][0], dtype=float)
    mid = 0.5 * (box[:3] + box[3:])
    out = {}
    for name, kw in (("sphere_128", dict(center=src, r_max=0.5 * L, n_shells=128)),
                     ("cylinder_64", dict(center=mid, r_max=0.5 * L, n_shells=64, axis=(1.0, 0.0, 0.0),
                                          half_height=0.25 * L, mean=True))):
        ctx.shell_profile(**kw)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.shell_profile(**kw)
        out[name + "_ms_per_call"] = (time.perf_counter() - t0) / reps * 1e3
    n, nf = int(cfg["pos"].shape[0]), int(cfg["params"]["n_freq"])
    out["particles"] = n
    out["algorithmic_bytes_per_call"] = n * (24 + 8 * nf)
    return out


def rr_scheme_row(cfg, W, K):
    """Section 2.2's comparison on one workload: recombination photons emitted
    into the reception cones against the predecessor scheme (every particle a
    point source with its own rotated emission cones on every emission
    sub-step), FP32 transport, the same steps; the emission's share of the step
    (time split with every launch timed) and the ionization state reached."""
    import numpy as np
    from paper_1311_0182_amd import inputs as I
    out = {}
    states = {}
    for name, mode in (("reception_cones", I.RR_TRANSPORT), ("predecessor", I.RR_ORIGINAL)):
        c = dict(cfg)
        c["params"] = dict(cfg["params"], recomb_mode=mode)
        sh = tuned_shape(c, W + K)["shape"]
        r = run_timed(c, "fp32", W, K, shape=sh)
        r["ctx"].close()
        rt = run_timed(c, "fp32", W, K, timing=True, shape=sh)
        tm = rt["timing"]
        rt["ctx"].close()
        states[name] = r["state"]
        out[name] = {"ms_per_step": r["t"] / K * 1e3, "updates_per_s": r["updates"] / r["t"],
                     "rr_photons_emitted": float(r["state"]["ledger"][0, 1, 0]),
                     "time_split_ms_per_step": {k: tm[k] / K for k in ("hop_ms", "vip_ms", "chem_ms", "emit_ms",
                                                                       "ledger_ms")}}
        print(f"RR scheme {name}: {r['t'] / K * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    out["predecessor_over_reception_cones_time"] = (out["predecessor"]["ms_per_step"] /
                                                    out["reception_cones"]["ms_per_step"])
    out["max_abs_dx_HI_between_schemes"] = float(np.max(np.abs(states["predecessor"]["xHI"] -
                                                                states["reception_cones"]["xHI"])))
    out["steps"] = f"{W}..{W + K - 1}"
    return out


def fp32_row(cfg, W, K, label):
    """FP32 transport only (the FP64 state of the full clustered field would not
    fit beside it): rate, per-step split and the forward step's launches."""
    import torch
    sh = tuned_shape(cfg, W + K)["shape"]
    torch.cuda.reset_peak_memory_stats()
    r = run_timed(cfg, "fp32", W, K, shape=sh)
    peak = torch.cuda.max_memory_allocated()
    st = r["state"]
    r["ctx"].close()
    rt = run_timed(cfg, "fp32", W, K, timing=True, shape=sh)
    tm = rt["timing"]
    rt["ctx"].close()
    launches = max(1.0, tm["hop_launches"])
    print(f"{label}: fp32 {r['t']:.3f} s over {K} steps", file=sys.stderr, flush=True)
    return {
        "workload": label,
        "steps": f"{W}..{W + K - 1}",
        "fp32_updates_per_s": r["updates"] / r["t"],
        "fp32_ms_per_step": r["t"] / K * 1e3,
        "ledger_residual_fp32": residual(st["ledger"]),
        "forward_steps_per_step": r["hops"] / K,
        "device_memory_peak_GB": peak / 1e9,
        "k_hop_float_avg_launch_ms": tm["hop_ms"] / launches,
        "time_split_ms_per_step": {k: tm[k] / K for k in ("hop_ms", "vip_ms", "chem_ms", "emit_ms", "ledger_ms")},
    }


def pair_row(cfg, W, K, label):
    """FP32 and FP64 over the same window: rates (work counted on FP64), the
    forward-step kernel's time per launch and the dense-model bandwidth, and
    max |dx_HI| at the window's end."""
    import numpy as np
    sh32 = tuned_shape(cfg, W + K)["shape"]
    r32 = run_timed(cfg, "fp32", W, K, shape=sh32)
    r32["ctx"].close()
    sh64 = tuned_shape(cfg, W + K, "fp64")["shape"]
    r64 = run_timed(cfg, "fp64", W, K, shape=sh64)
    r64["ctx"].close()
    rt = run_timed(cfg, "fp32", W, K, timing=True, shape=sh32)
    tm = rt["timing"]
    rt["ctx"].close()
    work = r64["updates"]
    launches = max(1.0, tm["hop_launches"])
    avg_ms = tm["hop_ms"] / launches
    dense, per_slot, slots = dense_bytes_per_hop(cfg, True)
    upl = rt["updates"] / launches
    print(f"{label}: fp32 {r32['t']:.3f} s, fp64 {r64['t']:.3f} s over {K} steps", file=sys.stderr, flush=True)
    return {
        "workload": label,
        "steps": f"{W}..{W + K - 1}",
        "fp32_updates_per_s": work / r32["t"],
        "fp32_ms_per_step": r32["t"] / K * 1e3,
        "fp64_updates_per_s": work / r64["t"],
        "fp64_ms_per_step": r64["t"] / K * 1e3,
        "speedup_fp32_over_fp64": r64["t"] / r32["t"],
        "max_abs_dx_HI_at_end": float(np.max(np.abs(r32["state"]["xHI"] - r64["state"]["xHI"]))),
        "ledger_residual_fp32": residual(r32["state"]["ledger"]),
        "forward_steps_per_step": r64["hops"] / K,
        "hop_shape": {"fp32": sh32, "fp64": sh64},
        "k_hop_float": {
            "avg_launch_ms": avg_ms,
            "launches": int(tm["hop_launches"]),
            "active_updates_per_launch": upl,
            "model_bytes_per_slot_update": per_slot,
            "achieved_GBs_model": per_slot * upl / (avg_ms * 1e-3) / 1e9,
            "achieved_GBs_dense_hop": dense / (avg_ms * 1e-3) / 1e9,
            "achieved_GBs_device_counted": tm["hop_bytes_total"] / launches / (avg_ms * 1e-3) / 1e9,
        },
        "time_split_ms_per_step": {k: tm[k] / K for k in ("hop_ms", "vip_ms", "chem_ms", "emit_ms", "ledger_ms")},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip the extra rows")
    ap.add_argument("--hop-shape", type=int, default=-1,
                    help="forward-step launch configuration 0..5 for every run (-1: the library's tuner picks)")
    ap.add_argument("--only", choices=["stromgren64_rr", "shadow128", "rr_schemes", "clustered256"], default=None,
                    help="run one extra row alone and print it (for profiling); no headline line")
    ap.add_argument("--c3-warmup", type=int, default=2)
    ap.add_argument("--c3-steps", type=int, default=3)
    ap.add_argument("--calib-copy-mb", type=float, default=0.0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU decomposition is designed, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1311_0182_amd import inputs as I

    torch.cuda.set_device(0)
    if args.calib_copy_mb > 0:
        # a plain device copy of known size, so that hardware byte counters of a
        # profiled run can be scaled to bytes
        n = int(args.calib_copy_mb * (1 << 20)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    K, W = args.steps, args.warmup
    global FORCE_SHAPE
    FORCE_SHAPE = args.hop_shape
    if args.only == "stromgren64_rr":
        print(json.dumps({"stromgren64_rr": pair_row(I.config(2), W, K, "64^3 Stromgren with RR")}), flush=True)
        return
    if args.only == "clustered256":
        print(json.dumps({"clustered256": fp32_row(I.config(5), 1, 2, CLUSTERED_LABEL)}), flush=True)
        return
    if args.only == "rr_schemes":
        print(json.dumps({"rr_schemes_stromgren64": rr_scheme_row(I.config(2), W, K)}), flush=True)
        return
    if args.only == "shadow128":
        print(json.dumps({"shadow128": pair_row(I.config(3), args.c3_warmup, args.c3_steps, "128^3 shadow set-up")}),
              flush=True)
        return
    cfg = I.config(4)
    n_inst = len(cfg["inst_off"]) - 1
    import numpy as np
    sizes = np.diff(cfg["inst_off"])

    shape = tuned_shape(cfg, W + K)
    r32 = run_timed(cfg, "fp32", W, K, shape=shape["shape"])
    r32["ctx"].close()
    print(f"batched fp32: {K} steps in {r32['t']:.3f} s, {r32['updates']} updates", file=sys.stderr, flush=True)
    r64 = run_timed(cfg, "fp64", W, K, shape=tuned_shape(cfg, W + K, "fp64")["shape"])
    r64["ctx"].close()
    print(f"batched fp64: {K} steps in {r64['t']:.3f} s, {r64['updates']} updates", file=sys.stderr, flush=True)
    acc = side_by_side(cfg, W + K)
    print(f"batched fp32 vs fp64 over {W + K} steps: max |dx_HI| {acc['max_abs_dx_HI']:.3e}", file=sys.stderr,
          flush=True)
    rt = run_timed(cfg, "fp32", W, K, timing=True, shape=shape["shape"])
    tm = rt["timing"]
    rt["ctx"].close()
    work = r64["updates"]
    rate = work / r32["t"]
    launches = max(1.0, tm["hop_launches"])
    avg_ms = tm["hop_ms"] / launches
    upl = rt["updates"] / launches
    dense, per_slot, slots = dense_bytes_per_hop(cfg, True)
    achieved = per_slot * upl / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": "particle-packet updates/s per RT step, FP32-batched vs FP64 at x_HI err<=1e-3",
        "value": rate if acc["met"] else 0.0,
        "unit": "particle-packet updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": r32["t"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched HII regions: {n_inst} instances, {int(sizes.sum())} particles "
                        f"({int(sizes.min())}..{int(sizes.max())} per instance), recombination radiation "
                        f"transported, N_ngb=48, N_TC=N_RC=N_EC=8, 2 bins, dt=0.1 Myr, steps {W}..{W + K - 1}",
            "particles": int(sizes.sum()),
            "slots": slots,
            "transport": "fp32 with TwoSum merge sums, decisions near thresholds in fp64; chemistry and ledger fp64",
            "hop_shape": shape,
        },
        "accuracy": acc,
        "roofline": {
            "kernel": "k_hop<float> (forward step: gather, merge, cone tests)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "avg_launch_ms": avg_ms,
            "launches": int(tm["hop_launches"]),
            "active_updates_per_launch": upl,
            "model_bytes_per_slot_update": per_slot,
            "bytes_per_launch_model": per_slot * upl,
            "dense_bytes_per_hop": dense,
            "achieved_dense_hop": dense / (avg_ms * 1e-3) / 1e9,
            "bytes_per_launch_device_counted": tm["hop_bytes_total"] / launches,
            "achieved_device_counted": tm["hop_bytes_total"] / launches / (avg_ms * 1e-3) / 1e9,
        },
        "fp64": {
            "updates_per_s": work / r64["t"],
            "ms_per_step": r64["t"] / K * 1e3,
            "fp32_speedup": r64["t"] / r32["t"],
            "fp32_updates": r32["updates"],
            "fp64_updates": r64["updates"],
        },
        "time_split_ms_per_step": {k: tm[k] / K for k in ("hop_ms", "vip_ms", "chem_ms", "emit_ms", "ledger_ms")},
        "forward_steps_per_step": r64["hops"] / K,
    }
    if not acc["met"]:
        out["value_bar_missed"] = rate
    if not args.headline_only:
        # the same timed steps with whole-step graphs (one host check per call)
        rg = run_timed(cfg, "fp32", W, K, shape=shape["shape"], step_graphs=True)
        rg["ctx"].close()
        out["whole_step_graphs"] = {"ms_per_step": rg["t"] / K * 1e3, "updates_per_s": work / rg["t"],
                                    "same_updates": rg["updates"] == r32["updates"],
                                    "time_vs_default": rg["t"] / r32["t"]}
        print(f"whole-step graphs: {rg['t'] / K * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        # the same instances solved one after another in FP64
        tseq, useq = 0.0, 0
        for k in range(n_inst):
            r = run_timed(I.instance(cfg, k), "fp64", W, K)
            r["ctx"].close()
            tseq += r["t"]
            useq += r["updates"]
        out["batched_fp64_one_by_one"] = {"updates_per_s": useq / tseq, "ms_per_step": tseq / K * 1e3,
                                          "fp32_batched_speedup": rate / (useq / tseq)}
        print(f"one by one fp64: {tseq:.3f} s", file=sys.stderr, flush=True)
        c2 = I.config(2)
        out["stromgren64_rr"] = pair_row(c2, W, K, "64^3 Stromgren with RR (262144 particles, 6.6 kpc box, N_ngb=48, "
                                                   "N_TC=N_RC=N_EC=8, 2 bins)")
        rp = run_timed(c2, "fp32", W, K)
        out["stromgren64_rr"]["shell_profile"] = shell_profile_timing(rp["ctx"], c2)
        rp["ctx"].close()
        out["rr_schemes_stromgren64"] = rr_scheme_row(c2, W, K)
        out["clustered256"] = fp32_row(I.config(5), 1, 2, CLUSTERED_LABEL)
        c3 = I.config(3)
        out["shadow128"] = pair_row(c3, args.c3_warmup, args.c3_steps,
                                    "128^3 shadow set-up (2097152 particles, plane front, 3 blackbody bins + RR, "
                                    "N_ngb=48, N_TC=N_RC=N_EC=16, heating and cooling)")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
