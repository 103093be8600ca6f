"""Benchmark of one TRAPHIC RT step with recombination radiation on one MI355X.

Workload: the 64^3-particle HII region with recombination radiation
(262,144 jittered particles in a 6.6 kpc box, n_H = 1e-3, one 5e48 photons/s
source, N_ngb = 48, N_TC = N_RC = N_EC = 8, a source bin and an RR bin,
dt = 0.1 Myr, 500 steps in all).  A step is one RT step: emission, all forward
steps until no packet moves, chemistry, RR emission and the photon ledger.

The FP32-transport run is the headline (forward steps replayed from captured
graphs); a second FP32 run with per-launch HIP events gives the time split and
the roofline of the forward-step kernel; the same steps in FP64 give the
comparison, the packet-update count (work is credited as counted on the FP64
run) and the x_HI reference for the FP32 error.  The batched workload (64
independent HII regions in the same launches) is reported beside it, against the
same instances solved one after another in FP64.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_hop_float_stromgren64_rr_hbm_bytes.md")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("rt_kernels.hpp", "rt_device.hpp"):
        with open(os.path.join(ROOT, "paper_1311_0182_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per forward-step launch from the committed counter summary,
    valid only while the kernel sources are the ones that were measured."""
    import re
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    sha = re.search(r"kernel_sources_sha256:\s*([0-9a-f]+)", txt)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9]+)", txt)
    if not sha or not val or sha.group(1) != kernel_sources_sha():
        return None
    return float(val.group(1))


def cpu_baseline(budget_s):
    """The FP64 oracle (single thread) on the same workload from step 0, for as
    many whole steps as fit in the budget."""
    from oracle import oracle as O
    from paper_1311_0182_amd import inputs as I
    cfg = I.config(2)
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
                sample=f"first {steps} steps of the same 64^3 workload ({upd} packet updates, "
                       f"{dt:.1f} s; neighbour search {t_init:.1f} s not counted)")


def shell_profile_timing(ctx, cfg, reps=50):
    """The intensity-profile diagnostic on the state left by the timed run: wall
    time per call (stream synchronisation, two fills, the kernel and the copy of
    the histogram back included); the kernel's own duration is in the trace."""
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


def batched_runs(K):
    """The batched workload: every instance in the same launches, FP32 and FP64
    transport, against the same instances solved one after another in FP64."""
    import numpy as np
    import torch

    from paper_1311_0182_amd import inputs as I
    from paper_1311_0182_amd import traphic_rt as RT

    cfg = I.config(4)
    steps = min(K, int(cfg["n_steps"]))

    def run(c, precision):
        ctx = RT.Context(c, precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = ctx.state()
        shape = ctx.hop_shape()
        ctx.close()
        return t, st, shape

    t32, s32, shape = run(cfg, "fp32")
    t64, s64, _ = run(cfg, "fp64")
    n_inst = len(cfg["inst_off"]) - 1
    tseq, useq = 0.0, 0
    for k in range(n_inst):
        t, st, _ = run(I.instance(cfg, k), "fp64")
        tseq += t
        useq += int(st["counters"][3])
    print(f"batched: fp32 {t32:.3f} s, fp64 {t64:.3f} s, fp64 one by one {tseq:.3f} s", file=sys.stderr, flush=True)
    work = int(s64["counters"][3])
    led = s32["ledger"]
    E, A, X, R, F = np.moveaxis(led, -1, 0)
    sizes = np.diff(cfg["inst_off"])
    return {
        "workload": f"{n_inst} independent HII regions, {int(sizes.sum())} particles "
                    f"({int(sizes.min())}..{int(sizes.max())} per instance), recombination radiation "
                    f"transported, N_ngb=48, N_TC=N_RC=N_EC=8, steps 0..{steps - 1}",
        "steps": steps,
        "fp32_updates_per_s": work / t32,
        "fp32_ms_per_step": t32 / steps * 1e3,
        "fp64_updates_per_s": work / t64,
        "fp64_ms_per_step": t64 / steps * 1e3,
        "fp64_one_by_one_updates_per_s": useq / tseq,
        "fp64_one_by_one_ms_per_step": tseq / steps * 1e3,
        "speedup_vs_fp64_one_by_one": (work / t32) / (useq / tseq),
        "max_abs_dx_HI_fp32_vs_fp64": float(np.max(np.abs(s32["xHI"] - s64["xHI"]))),
        "ledger_residual_fp32": float(np.max(np.abs(E - A - X - R - F) / np.maximum(E, 1e-300))),
        "hop_shape": shape,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--calib-copy-mb", type=float, default=0.0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU decomposition is designed, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1311_0182_amd import inputs as I
    from paper_1311_0182_amd import traphic_rt as RT

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
    cfg = I.config(2)
    K, W = args.steps, args.warmup

    def run(precision, timing):
        ctx = RT.Context(cfg, precision=precision)
        if W:
            ctx.step(W)
        u0 = int(ctx.state()["counters"][3])
        ctx.set_timing(timing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(K)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = ctx.state()
        tm = ctx.timing() if timing else None
        prof = shell_profile_timing(ctx, cfg) if timing else None
        res = dict(t=t, updates=int(st["counters"][3]) - u0, state=st, timing=tm, shape=ctx.hop_shape(), prof=prof)
        ctx.close()
        return res

    r32 = run("fp32", False)
    print(f"fp32: {K} steps in {r32['t']:.3f} s, {r32['updates']} updates", file=sys.stderr, flush=True)
    r32t = run("fp32", True)
    print(f"fp32 timed: {K} steps in {r32t['t']:.3f} s", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run("fp64", False)
        print(f"fp64: {K} steps in {r64['t']:.3f} s, {r64['updates']} updates", file=sys.stderr, flush=True)
    work = r64["updates"] if r64 else r32["updates"]
    value = work / r32["t"]
    led = r32["state"]["ledger"]
    E, A, X, R, F = np.moveaxis(led, -1, 0)
    resid = float(np.max(np.abs(E - A - X - R - F) / np.maximum(E, 1e-300)))
    tm = r32t["timing"]
    launches = max(tm["hop_launches"], 1)
    avg_ms = tm["hop_ms"] / launches
    bytes_per_launch = tm["hop_bytes_total"] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    G = cfg["params"]["n_rc"] * cfg["params"]["n_freq"]
    n_tiles = -(-int(cfg["pos"].shape[0]) // max(1, 64 // G))  # one wavefront of slots per tile
    out = {
        "metric": "particle-packet updates/s per RT step, FP32-batched vs FP64 at x_HI err<=1e-3",
        "value": value,
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
            "workload": "stromgren64_rr: 262144 particles (64^3 jittered, 6.6 kpc box), recombination "
                        "radiation transported, N_ngb=48, N_TC=N_RC=N_EC=8, 2 bins, dt=0.1 Myr, "
                        f"steps {W}..{W + K - 1} of 500",
            "particles": int(cfg["pos"].shape[0]),
            "slots": int(cfg["pos"].shape[0]) * 16,
            "transport": "fp32 with TwoSum merge sums; chemistry and ledger fp64",
            "hop_shape": r32["shape"],
        },
        "roofline": {
            "kernel": "k_hop<float> (forward step: gather, merge, cone masks)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "avg_launch_ms": avg_ms,
            "launches": int(tm["hop_launches"]),
            "bytes_per_launch": bytes_per_launch,
            "tiles_per_launch": tm["hop_tiles_total"] / launches,
            "tiles": n_tiles,
            "dense_bytes_per_hop": tm["dense_bytes_per_hop"],
        },
        "fp32_vs_fp64": None,
        "ledger_residual_fp32": resid,
        "time_split_ms": {k: tm[k] for k in ("hop_ms", "vip_ms", "chem_ms", "emit_ms", "ledger_ms")},
        "ms_per_step_timed_run": r32t["t"] / K * 1e3,
        "shell_profile": r32t["prof"],
    }
    if r64:
        dx = float(np.max(np.abs(r32["state"]["xHI"] - r64["state"]["xHI"])))
        out["fp32_vs_fp64"] = {
            "fp64_updates_per_s": r64["updates"] / r64["t"],
            "fp64_ms_per_step": r64["t"] / K * 1e3,
            "speedup": r64["t"] / r32["t"],
            "max_abs_dx_HI": dx,
            "fp32_updates": r32["updates"],
            "fp64_updates": r64["updates"],
        }
    if not args.no_batched:
        out["batched"] = batched_runs(K)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
