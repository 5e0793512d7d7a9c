"""Benchmark: Mcell-updates/s of the fused finite-volume step on one MI355X.

Workload (default): the Cartesian Gaussian-pulse case, 4096 x 4096 cells,
dx = 1e-4 m, water (c0 1500 m/s, rho0 1000 kg/m^3, beta 3.5, delta
4.3e-6 m^2/s), 2 MPa pulse with sigma = 20 cells at a seed-chosen centre
plus 0.5% white noise (seed 2), zero-order-extrapolation sides, CFL 0.9.
A step is one accepted time step of the whole method (x1 sweep, x2 sweep,
source, CFL control) over the grid.

Prints ONE JSON line.  The headline is the FP64 path (the paper's
arithmetic: all its simulations run in double precision).  Beside it: the
FP32 path on the same workload with its error against FP64, the batched form
(64 uneven simulations, one graph-replayed launch per step) against 64
sequential launches, the axisymmetric focused-source configs (8192 x 2048
FP32; 16384 x 8192 in FP32 and FP16 storage), the 3-D step, the
roofline of the step kernels and the FP64 CPU oracle timed on a bounded
sample on the host (one thread and every core of the process's CPU share).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"f64": 48, "f32": 24, "f32_f16store": 12, "f32_bf16store": 12}

# Counter figures of the step kernels on this workload (4096 x 4096), from
# rocprofv3 --pmc runs of this script: HBM bytes per launch from FETCH_SIZE,
# then WRITE_SIZE, each scaled by what the same counter reads for a plain
# device copy (fetch x1.988, write x1.000), and VALU lane-ops per
# cell-update from SQ_INSTS_VALU x 64 / cells, and SIMD issue cycles per
# cell-update from SQ_ACTIVE_INST_VALU (quad-cycles, summed over waves) x 4 /
# cells, which also counts the extra cycles of transcendental instructions
# (an FP64 reciprocal estimate holds the SIMD 4 quad-cycles, FP32 2)
# (profiles/k_step_*.md).  Each
# entry is valid only for the kernel sources, launch configuration (the
# runtime sets the row segments) and build flags whose SHA-256 it records:
# after any change they report null until profiled again.
PMC_SOURCES = ("csrc/fvna_device.hpp", "csrc/fvna_step.hpp", "csrc/fvna_runtime.hip", "build.py")
_PROFILED = {
    "csrc/fvna_device.hpp": "e8a79044eebcf6e19e0827735f2385e5190242fcd93d8f0951e51202d2ddb50c",
    "csrc/fvna_step.hpp": "a9e84437ccfeefe0500bc34f950718571f6c39e84c9e7b8d6134cc1fc4995563",
    "csrc/fvna_runtime.hip": "0d2f8bb9b9116e5a8e1603e80e57027609bc6f354015411944941212688ed2a5",
    "build.py": "02eda4061ab4ab18fbd0c2e868524ec4e9acf39f5fa26d0513e48c2fca74259e",
}
PMC = {
    # profiles/k_step_f64_gaussian4096.md
    "k_step<double,double,0>": {"nx": 4096, "ny": 4096, "fetch_bytes": 4.1953e+08, "write_bytes": 4.0525e+08,
                                "valu_lane_ops_per_cell": 399.6, "valu_issue_cycles_per_cell": 26.49,
                                "sources": _PROFILED},
    # profiles/k_step_f32_gaussian4096.md
    "k_step<float,float,0>": {"nx": 4096, "ny": 4096, "fetch_bytes": 2.1497e+08, "write_bytes": 2.0450e+08,
                              "valu_lane_ops_per_cell": 300.8, "valu_issue_cycles_per_cell": 19.75,
                              "sources": _PROFILED},
}


def _sources_digest():
    import hashlib
    out = {}
    for rel in PMC_SOURCES:
        with open(os.path.join(ROOT, "paper_1311_3004_amd", rel), "rb") as f:
            out[rel] = hashlib.sha256(f.read()).hexdigest()
    return out


def pmc_entry(kernel, nx, ny):
    e = PMC.get(kernel)
    if e is None or (nx, ny) != (e["nx"], e["ny"]) or e["sources"] != _sources_digest():
        return None
    return e


# Vector-ALU rate of the chip counted as the profile counts SQ_INSTS_VALU:
# one wave64 instruction per CU per cycle = 256 CUs x 64 lanes x 2.4 GHz.
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# SIMD cycles available per second: 1024 SIMDs at the 2.4 GHz peak clock.
SIMD_CYCLES_PER_S = 1024 * 2.4e9


def measured_valu(kernel, nx, ny, kernel_s):
    """VALU lane-ops per cell-update of the profiled kernel and the rate they
    run at in the live launch, against the chip's non-packed vector rate; None
    if the kernel sources or grid differ from the profiled ones."""
    e = pmc_entry(kernel, nx, ny)
    if e is None:
        return None
    ops = e["valu_lane_ops_per_cell"]
    rate = ops * nx * ny / kernel_s
    cyc = e["valu_issue_cycles_per_cell"]
    return {"lane_ops_per_cell": ops, "achieved": round(rate / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
            "unit": "T lane-ops/s", "frac": round(rate / VALU_PEAK_LANE_OPS, 4),
            # fraction of the launch the SIMDs spend issuing vector instructions
            # (transcendental cycles included), at the 2.4 GHz peak clock
            "issue_cycles_per_cell": cyc, "issue_frac": round(cyc * nx * ny / kernel_s / SIMD_CYCLES_PER_S, 4)}


def measured_traffic(kernel, nx, ny):
    """PMC HBM bytes per launch if the kernel sources and grid are the profiled ones."""
    e = pmc_entry(kernel, nx, ny)
    return None if e is None else e["fetch_bytes"] + e["write_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_run(sim, steps, warmup):
    """Warm up, then time exactly `steps` accepted steps with HIP events on the
    library's stream (and the host clock around it)."""
    import torch
    sim.fvna_step(warmup)
    sim.fvna_sync()
    st0 = sim.fvna_get_stats()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(sim.stream)
    sim.fvna_step(steps)
    sim.fvna_sync()                 # completes any attempts owed after rejections
    e1.record(sim.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = sim.fvna_get_stats()
    accepted = st1["steps"] - st0["steps"]
    return {"wall_s": t1 - t0, "event_s": e0.elapsed_time(e1) / 1e3, "accepted": accepted,
            "rejected": st1["rejected"] - st0["rejected"], "nu_mean": st1["nu_mean"],
            "nu_std": st1["nu_std"], "t": st1["t"]}


def kernel_roofline(sim, precision, cells, reps=20):
    ms = sim.fvna_time_step_kernel(reps)
    achieved = BYTES_PER_CELL[precision] * cells / (ms * 1e-3) / 1e9
    return ms, achieved


def other_configs(fvna, inputs, steps):
    """Throughput of the step on the axisymmetric focused-source configs: the
    8192 x 2048 FP32 grid and the 16384 x 8192 grid in FP32 and FP16 storage
    (quiescent start, source ramping up; the cost of a step does not depend on
    the field).  FP16 storage halves the bytes but not the time: the kernel is
    bound by its vector instructions, not by HBM.  BF16 storage is left out:
    its 8-bit significand does not resolve the focused field (focal harmonics
    off by 13-270%, the shock front by 4 cells at 8192 x 2048 and 191 at
    16384 x 8192 against the FP64 run)."""
    out = {}
    runs = [("hifu-axisym 8192x2048", inputs.c3_hifu_fp32(), ("f32",))]
    runs.append(("hifu-mixed 16384x8192", inputs.c5_hifu_mixed(), ("f32", "f32_f16store")))
    for name, w, precs in runs:
        med, src = w["medium"], w["source"]
        cells = w["nx"] * w["ny"]
        for prec in precs:
            over = {}
            if "store" in prec:
                over["store_scale"] = (64 * src["p_surface"] / (med["rho0"] * med["c0"] ** 2),) * 3
            s = fvna.sim_from_workload(w, precision=prec, **over)
            r = timed_run(s, steps, 10)
            ms_k, gbs = kernel_roofline(s, prec, cells, reps=5)
            v = cells * r["accepted"] / r["event_s"] / 1e6
            log(f"[bench] {name} {prec}: {v:.1f} Mcell/s, kernel {ms_k:.3f} ms = {gbs:.0f} GB/s")
            out[f"{name} {prec}"] = {"value": round(v, 1), "unit": "Mcell-updates/s", "steps": steps,
                                     "kernel_ms": round(ms_k, 4), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                     "tile_rows": s.fvna_get_tile_rows()}
            if prec == "f32_f16store":
                out[f"{name} {prec}"]["note"] = ("half the bytes of FP32 storage, not faster: the step "
                                                 "kernel is bound by vector instructions")
            s.fvna_destroy()
        del w
    return out


def three_d(n=256, steps=200, precision="f32"):
    """The 3-D step (fused x1-x2 sweep, x3 sweep, source and a device-side
    controller, replayed from a HIP graph) on an n^3 Gaussian pulse (sigma 8
    cells, 2 MPa, 0.5% noise, seed 5), extrapolating sides, in FP32 or FP64:
    whole steps per second (host clock around fvna3_step, which waits once at
    its end) and the mean duration of the three kernels of one step (HIP
    events) against 32 B (FP32) or 64 B (FP64) per cell-update (read and
    write of four fields)."""
    import time
    import numpy as np
    from paper_1311_3004_amd import fvna3d as f3
    from paper_1311_3004_amd.inputs import WATER
    med = dict(WATER)
    rng = np.random.default_rng(5)
    c = (np.arange(n) + 0.5 - n / 2) ** 2
    a = 2e6 / (med["rho0"] * med["c0"] ** 2)
    R = a * np.exp(-(c[:, None, None] + c[None, :, None] + c[None, None, :]) / (2 * 8.0 ** 2))
    R += 0.005 * a * rng.uniform(-1, 1, R.shape)
    Z = np.zeros_like(R)
    s = f3.Sim3(f3.make_params(n, n, n, 1e-4, med, precision=precision))
    s.fvna3_set_state(R * med["rho0"], Z, Z, Z)
    del R, Z
    s.fvna3_step(3)
    t0 = time.perf_counter()
    s.fvna3_step(steps)
    wall = time.perf_counter() - t0
    ms = s.fvna3_time_step_kernels(10)
    cells = n ** 3
    bpc = 32 if precision == "f32" else 64
    gbs = bpc * cells / (ms * 1e-3) / 1e9
    s.fvna3_destroy()
    log(f"[bench] 3-D {n}^3 {precision}: {cells * steps / wall / 1e6:.1f} Mcell/s, step kernels {ms:.3f} ms = {gbs:.0f} GB/s")
    return {"workload": f"gaussian-pulse {n}^3 {precision}", "value": round(cells * steps / wall / 1e6, 1),
            "unit": "Mcell-updates/s", "steps": steps, "step_kernels_ms": round(ms, 4),
            "kernel_rate": round(cells / (ms * 1e-3) / 1e6, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_cell_update": bpc}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Threads the oracle may use: the process's CPU share (OMP_NUM_THREADS
    when set, else the CPUs this process may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(w, steps, threads):
    """FP64 oracle on the host: `steps` steps of the same workload, full grid,
    on `threads` threads (OpenMP over rows; bitwise identical results)."""
    import oracle
    med = w["medium"]
    p = oracle.make_params_si(w["nx"], w["ny"], w["dx"], med["c0"], med["rho0"], med["beta"],
                              med["delta"], bc=w["bc"])
    rp, mx, my = w["state"]
    R, M, N = rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"])
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        _, _, _, info = oracle.run(p, R, M, N, steps)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    assert info["status"] == 0
    return w["nx"] * w["ny"] * steps / dt / 1e6, dt


def step_leg(fvna, w, precision, steps, warmup, tile_rows=0):
    """One precision on the main workload: throughput, live kernel time, state."""
    cells = w["nx"] * w["ny"]
    s = fvna.sim_from_workload(w, precision=precision, tile_rows=tile_rows)
    r = timed_run(s, steps, warmup)
    v = cells * r["accepted"] / r["event_s"] / 1e6
    ms_k, gbs = kernel_roofline(s, precision, cells)
    R = s.fvna_get_state()[0]
    tr = s.fvna_get_tile_rows()
    s.fvna_destroy()
    kernel = {"f64": "k_step<double,double,0>", "f32": "k_step<float,float,0>"}[precision]
    log(f"[bench] {precision}: {v:.1f} Mcell/s, {r['event_s'] * 1e3 / steps:.3f} ms/step, "
        f"step kernel {ms_k:.4f} ms = {gbs:.0f} GB/s algorithmic")
    return {"value": v, "run": r, "kernel_ms": ms_k, "gbs": gbs, "R": R, "tile_rows": tr, "kernel": kernel}


def roofline_of(leg, precision, nx, ny):
    cells = nx * ny
    k = leg["kernel"]
    return {"bound": "hbm", "achieved": round(leg["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(leg["gbs"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(k, nx, ny),
            "kernel": k, "kernel_ms": round(leg["kernel_ms"], 4),
            "bytes_per_launch": BYTES_PER_CELL[precision] * cells,
            "valu": measured_valu(k, nx, ny, leg["kernel_ms"] * 1e-3)}


def batched_leg(fvna, inputs, nb):
    """64 uneven simulations in one batch against 64 sequential contexts:
    throughput of each and bitwise equality of every member's final state.
    The batch's segment heights come from fvna_batch_autotune (timed on the
    batch before the timed region); the kernel is also timed at the fixed
    default height for comparison."""
    import torch
    sims = inputs.c4_batch()
    plist = [fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], precision="f32")
             for x in sims]
    B = fvna.Batch(plist)
    for k, x in enumerate(sims):
        B.fvna_batch_set_state(k, *x["state"])
    B.fvna_batch_time_step_kernel(2)                # warm-up
    ms_default = B.fvna_batch_time_step_kernel(5)
    tuned = B.fvna_batch_autotune()
    classes = {}
    for x, tr in zip(sims, tuned):
        c = 1 << (int(x["ny"]).bit_length() - 1)
        classes.setdefault(f"ny {c}..{2 * c - 1}", set()).add(tr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.fvna_batch_step(nb)
    B.fvna_batch_sync()
    e1.record(B.stream)
    torch.cuda.synchronize()
    tb = e0.elapsed_time(e1) / 1e3
    bcells = sum(x["nx"] * x["ny"] for x in sims)
    vb = bcells * nb / tb / 1e6
    msb = B.fvna_batch_time_step_kernel(5)
    gbsb = 24 * bcells / (msb * 1e-3) / 1e9
    tseq = 0.0
    same = 0
    for k, x in enumerate(sims):
        s = fvna.Sim(plist[k])
        s.fvna_set_state(*x["state"])
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(s.stream)
        s.fvna_step(nb)
        s.fvna_sync()
        a1.record(s.stream)
        torch.cuda.synchronize()
        tseq += a0.elapsed_time(a1) / 1e3
        same += all(np.array_equal(u, v) for u, v in zip(s.fvna_get_state(), B.fvna_batch_get_state(k)))
        s.fvna_destroy()
    vseq = bcells * nb / tseq / 1e6
    log(f"[bench] batched: {vb:.1f} Mcell/s (kernel {gbsb:.0f} GB/s, {ms_default:.4f} ms at the default "
        f"height) vs sequential {vseq:.1f}; bitwise equal {same}/{len(sims)}")
    B.fvna_batch_destroy()
    return {"value": round(vb, 1), "unit": "Mcell-updates/s", "sims": len(sims), "cells": bcells, "steps": nb,
            "sequential_value": round(vseq, 1), "speedup_vs_sequential": round(vb / vseq, 3),
            "kernel_ms": round(msb, 4), "kernel_ms_default_tile_rows": round(ms_default, 4),
            "tile_rows_by_class": {k: sorted(v) for k, v in sorted(classes.items())},
            "hbm_frac": round(gbsb / HBM_PEAK_GBS, 4), "bitwise_equal_members": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 leg of the main workload")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the axisymmetric configs")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D leg")
    ap.add_argument("--fp32-only", action="store_true",
                    help="run only the FP32 leg of the main workload (for its profiles)")
    ap.add_argument("--other-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps on one thread")
    ap.add_argument("--cpu-steps-all", type=int, default=8, help="oracle steps on every core of the share")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (a large domain would "
              "shard as slabs along x1 with a 3-cell halo exchange and one max-reduction of the "
              "wave speed per step).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_3004_amd import fvna, inputs

    torch.cuda.set_device(0)
    w = inputs.c2_pulse_fp32(args.nx, args.ny)
    nx, ny = w["nx"], w["ny"]
    workload = f"gaussian-pulse {nx}x{ny}"
    log(f"[bench] workload {workload}, {args.steps} steps (+{args.warmup} warm-up)")

    extra = {}
    if args.fp32_only:
        l32 = step_leg(fvna, w, "f32", args.steps, args.warmup)
        head, head_prec = l32, "f32"
    else:
        # ---- headline: FP64, the paper's arithmetic ----
        l64 = step_leg(fvna, w, "f64", args.steps, args.warmup)
        head, head_prec = l64, "f64"
        # ---- FP32 on the same workload, and its error against FP64 ----
        if not args.no_fp32:
            l32 = step_leg(fvna, w, "f32", args.steps, args.warmup)
            R32, R64 = l32["R"], l64["R"]
            err = float(np.max(np.abs(R32 - R64)) / np.max(np.abs(R64)))
            l2 = float(np.sqrt(np.mean((R32 - R64) ** 2)) / np.sqrt(np.mean(R64 ** 2)))
            log(f"[bench] fp32 max|dp|/p_peak vs fp64 = {err:.2e}")
            extra["fp32"] = {"value": round(l32["value"], 1), "unit": "Mcell-updates/s",
                             "ms_per_step": round(l32["run"]["event_s"] * 1e3 / args.steps, 4),
                             "tile_rows": l32["tile_rows"], "roofline": roofline_of(l32, "f32", nx, ny),
                             "error_vs_fp64": {"max_abs_dp_over_p_peak": err, "rel_l2": l2,
                                               "steps": args.warmup + args.steps,
                                               "time_rel_diff": abs(l32["run"]["t"] - l64["run"]["t"]) /
                                               l64["run"]["t"]},
                             "over_fp64": round(l32["value"] / l64["value"], 3)}
    r = head["run"]

    if not args.fp32_only and not args.no_batch:
        extra["batched"] = batched_leg(fvna, inputs, args.batch_steps)
    if not args.fp32_only and not args.no_other:
        extra["other_configs"] = other_configs(fvna, inputs, args.other_steps)
    if not args.fp32_only and not args.no_3d:
        extra["three_d"] = three_d()
        extra["three_d_f64"] = three_d(precision="f64")

    out = {
        "metric": "Mcell-updates/s and % HBM roofline, FP32/batched vs FP64 at stated error",
        "value": round(head["value"], 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["event_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_prec,
        "data": "synthetic",
        "config": {"workload": workload, "precision": head_prec, "nx": nx, "ny": ny, "dx_m": w["dx"],
                   "steps": args.steps, "boundaries": "zero-order extrapolation", "seed": 2,
                   "cfl_target": 0.9, "tile_rows": head["tile_rows"]},
        "roofline": roofline_of(head, head_prec, nx, ny),
        "wall_s": round(r["wall_s"], 4),
        "nu_mean": r["nu_mean"], "nu_std": r["nu_std"], "rejected": r["rejected"],
    }
    out.update(extra)
    if not args.no_cpu and not args.fp32_only:
        nt = cpu_threads()
        v1, t1 = cpu_baseline(w, args.cpu_steps, 1)
        vn, tn = cpu_baseline(w, args.cpu_steps_all, nt)
        log(f"[bench] oracle on host: {v1:.2f} Mcell/s on 1 thread ({t1:.1f} s), "
            f"{vn:.2f} Mcell/s on {nt} threads ({tn:.1f} s)")
        out["cpu_baseline"] = {"value": round(vn, 3), "unit": "Mcell-updates/s", "cores": nt, "kind": "oracle",
                               "sample": f"{args.cpu_steps_all} steps of the same workload on the full "
                                         f"{nx}x{ny} grid, FP64, {nt} threads (OpenMP over rows)",
                               "single_thread": {"value": round(v1, 3), "steps": args.cpu_steps},
                               "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * (1 << 30)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
