"""Benchmark: Mcell-updates/s of the fused finite-volume step on one MI355X.

Workload (default): the FP32 Cartesian Gaussian-pulse case, 4096 x 4096
cells, dx = 1e-4 m, water (c0 1500 m/s, rho0 1000 kg/m^3, beta 3.5,
delta 4.3e-6 m^2/s), 2 MPa pulse with sigma = 20 cells at a seed-chosen
centre plus 0.5% white noise (seed 2), zero-order-extrapolation sides, CFL
0.9, 2000 steps.  A step is one accepted time step of the whole method
(x1 sweep, x2 sweep, source, CFL control) over the grid.

Prints ONE JSON line.  Besides the headline FP32 figure it carries the FP64
path on the same workload, the FP32 error against it, the batched form (64
uneven simulations in one graph-replayed launch per step) against 64
sequential launches, the throughput of the axisymmetric focused-source
configs (8192 x 2048 FP32; 16384 x 8192 in FP32, FP16 and BF16 storage), the
roofline of the step kernel and the FP64 CPU oracle timed on a bounded sample
on the host.
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

# HBM bytes per launch of the FP32 step kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE), each scaled by what the
# same counter reads for a plain 1 GiB device copy (fetch x2.000, write x1.000);
# profiles/k_step_f32_gaussian4096.md.  Valid only for the kernel sources and
# build flags whose SHA-256 is recorded here: anything else reports null.
PMC_TRAFFIC = {
    "bytes_per_launch": 216.1e6 + 204.4e6,
    "fetch_bytes": 216.1e6, "write_bytes": 204.4e6,
    "valu_lane_ops_per_cell": 308.0,
    "nx": 4096, "ny": 4096,
    "sources": {
        "fvna_device.hpp": "36224bdec71b2149af2a36c7e561432dc6c8d97c03d0f968f7e439323ef7115c",
        "fvna_runtime.hip": "81331248debaae07efbe8311f94b596b7ab0a8c598f93549c7c276d4e917e5ec",
        "build.py": "1709860880cb190303f24f18d1fde1d9184d0402975a6b07f4af871ebecdc2f1",
    },
}


# Vector-ALU rate of the chip counted as the profile counts SQ_INSTS_VALU:
# one wave64 instruction per CU per cycle = 256 CUs x 64 lanes x 2.4 GHz.
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9


def measured_valu(nx, ny, kernel_s):
    """VALU lane-ops per cell-update of the profiled kernel (SQ_INSTS_VALU x 64
    / cells) and the rate they run at in the live launch, against the chip's
    non-packed vector rate; None if the kernel sources or grid differ from the
    profiled ones."""
    if measured_traffic(nx, ny) is None:
        return None
    ops = PMC_TRAFFIC["valu_lane_ops_per_cell"]
    rate = ops * nx * ny / kernel_s
    return {"lane_ops_per_cell": ops, "achieved": round(rate / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
            "unit": "T lane-ops/s", "frac": round(rate / VALU_PEAK_LANE_OPS, 4)}


def measured_traffic(nx, ny):
    """PMC bytes per launch if the kernel sources and grid are the profiled ones."""
    import hashlib
    if (nx, ny) != (PMC_TRAFFIC["nx"], PMC_TRAFFIC["ny"]):
        return None
    for name, digest in PMC_TRAFFIC["sources"].items():
        sub = () if name == "build.py" else ("csrc",)
        path = os.path.join(ROOT, "paper_1311_3004_amd", *sub, name)
        with open(path, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return PMC_TRAFFIC["bytes_per_launch"]


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
    8192 x 2048 FP32 grid and the 16384 x 8192 grid in FP32, FP16 and BF16
    storage (quiescent start, source ramping up; the cost of a step does not
    depend on the field)."""
    out = {}
    runs = [("hifu-axisym 8192x2048", inputs.c3_hifu_fp32(), ("f32",))]
    runs.append(("hifu-mixed 16384x8192", inputs.c5_hifu_mixed(), ("f32", "f32_f16store", "f32_bf16store")))
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
            s.fvna_destroy()
        del w
    return out


def three_d(n=256, steps=20):
    """The 3-D step (first version: one kernel per sweep and one for the
    source, the step decided on the host) on an n^3 FP32 Gaussian pulse
    (sigma 8 cells, 2 MPa, 0.5% noise, seed 5), extrapolating sides: whole
    steps per second (host clock, one synchronisation per step) and the mean
    duration of the four kernels of one step (HIP events) against 32 B per
    cell-update (read and write of four FP32 fields)."""
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
    s = f3.Sim3(f3.make_params(n, n, n, 1e-4, med, precision="f32"))
    s.fvna3_set_state(R * med["rho0"], Z, Z, Z)
    del R, Z
    s.fvna3_step(3)
    t0 = time.perf_counter()
    s.fvna3_step(steps)
    wall = time.perf_counter() - t0
    ms = s.fvna3_time_step_kernels(10)
    cells = n ** 3
    gbs = 32 * cells / (ms * 1e-3) / 1e9
    s.fvna3_destroy()
    log(f"[bench] 3-D {n}^3 fp32: {cells * steps / wall / 1e6:.1f} Mcell/s, step kernels {ms:.3f} ms = {gbs:.0f} GB/s")
    return {"workload": f"gaussian-pulse {n}^3 fp32", "value": round(cells * steps / wall / 1e6, 1),
            "unit": "Mcell-updates/s", "steps": steps, "step_kernels_ms": round(ms, 4),
            "kernel_rate": round(cells / (ms * 1e-3) / 1e6, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_cell_update": 32}


def cpu_baseline(w, steps):
    """FP64 oracle on the host: `steps` steps of the same workload, full grid."""
    import oracle
    med = w["medium"]
    p = oracle.make_params_si(w["nx"], w["ny"], w["dx"], med["c0"], med["rho0"], med["beta"],
                              med["delta"], bc=w["bc"])
    rp, mx, my = w["state"]
    R, M, N = rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"])
    t0 = time.perf_counter()
    _, _, _, info = oracle.run(p, R, M, N, steps)
    dt = time.perf_counter() - t0
    assert info["status"] == 0
    return w["nx"] * w["ny"] * steps / dt / 1e6, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the axisymmetric configs")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D leg")
    ap.add_argument("--other-steps", type=int, default=200)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
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
    cells = w["nx"] * w["ny"]
    med = w["medium"]
    log(f"[bench] workload {w['name']}, {args.steps} steps (+{args.warmup} warm-up)")

    # ---- headline: FP32 ----
    s32 = fvna.sim_from_workload(w, precision="f32")
    if args.autotune:
        log(f"[bench] autotuned tile_rows = {s32.fvna_autotune()}")
        s32.fvna_set_state(*w["state"])
    r32 = timed_run(s32, args.steps, args.warmup)
    v32 = cells * r32["accepted"] / r32["event_s"] / 1e6
    ms_k, gbs = kernel_roofline(s32, "f32", cells)
    log(f"[bench] fp32: {v32:.1f} Mcell/s, {r32['event_s'] * 1e3 / args.steps:.3f} ms/step, "
        f"step kernel {ms_k:.3f} ms = {gbs:.0f} GB/s algorithmic")
    R32 = s32.fvna_get_state()[0]
    tile_rows = s32.fvna_get_tile_rows()
    s32.fvna_destroy()

    extra = {}
    # ---- FP64 path, same workload, and the FP32 error against it ----
    if not args.no_fp64:
        s64 = fvna.sim_from_workload(w, precision="f64", tile_rows=tile_rows)
        r64 = timed_run(s64, args.steps, args.warmup)
        v64 = cells * r64["accepted"] / r64["event_s"] / 1e6
        ms64, gbs64 = kernel_roofline(s64, "f64", cells)
        R64 = s64.fvna_get_state()[0]
        s64.fvna_destroy()
        err = float(np.max(np.abs(R32 - R64)) / np.max(np.abs(R64)))
        l2 = float(np.sqrt(np.mean((R32 - R64) ** 2)) / np.sqrt(np.mean(R64 ** 2)))
        log(f"[bench] fp64: {v64:.1f} Mcell/s, kernel {ms64:.3f} ms = {gbs64:.0f} GB/s; "
            f"fp32 max|dp|/p_peak = {err:.2e}")
        extra["fp64"] = {"value": round(v64, 1), "unit": "Mcell-updates/s",
                         "ms_per_step": round(r64["event_s"] * 1e3 / args.steps, 4),
                         "kernel_ms": round(ms64, 4), "hbm_frac": round(gbs64 / HBM_PEAK_GBS, 4)}
        extra["fp32_error_vs_fp64"] = {"max_abs_dp_over_p_peak": err, "rel_l2": l2,
                                       "steps": args.warmup + args.steps,
                                       "time_rel_diff": abs(r32["t"] - r64["t"]) / r64["t"]}
        extra["fp32_over_fp64"] = round(v32 / v64, 3)

    # ---- batched form: 64 uneven simulations vs 64 sequential runs ----
    if not args.no_batch:
        sims = inputs.c4_batch()
        plist = [fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], precision="f32")
                 for x in sims]
        B = fvna.Batch(plist)
        for k, x in enumerate(sims):
            B.fvna_batch_set_state(k, *x["state"])
        nb = args.batch_steps
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
        # sequential reference: same simulations, one context each, run one after another
        tseq = 0.0
        same = True
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
            if k % 8 == 0:
                same &= all(np.array_equal(u, v) for u, v in zip(s.fvna_get_state(), B.fvna_batch_get_state(k)))
            s.fvna_destroy()
        vseq = bcells * nb / tseq / 1e6
        log(f"[bench] batched: {vb:.1f} Mcell/s (kernel {gbsb:.0f} GB/s) vs sequential {vseq:.1f}; "
            f"bitwise equal (sampled) {same}")
        extra["batched"] = {"value": round(vb, 1), "unit": "Mcell-updates/s", "sims": len(sims),
                            "cells": bcells, "steps": nb, "sequential_value": round(vseq, 1),
                            "speedup_vs_sequential": round(vb / vseq, 3),
                            "hbm_frac": round(gbsb / HBM_PEAK_GBS, 4),
                            "bitwise_equal_sampled": bool(same)}
        B.fvna_batch_destroy()

    if not args.no_other:
        extra["other_configs"] = other_configs(fvna, inputs, args.other_steps)
    if not args.no_3d:
        extra["three_d"] = three_d()

    out = {
        "metric": "Mcell-updates/s and % HBM roofline, FP32/batched vs FP64 at stated error",
        "value": round(v32, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["event_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "nx": w["nx"], "ny": w["ny"], "dx_m": w["dx"],
                   "steps": args.steps, "boundaries": "zero-order extrapolation", "seed": 2,
                   "cfl_target": 0.9, "tile_rows": tile_rows},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(w["nx"], w["ny"]),
                     "kernel": "k_step<float,float,0>", "kernel_ms": round(ms_k, 4),
                     "bytes_per_launch": BYTES_PER_CELL["f32"] * cells,
                     "valu": measured_valu(w["nx"], w["ny"], ms_k * 1e-3)},
        "wall_s": round(r32["wall_s"], 4),
        "nu_mean": r32["nu_mean"], "nu_std": r32["nu_std"], "rejected": r32["rejected"],
    }
    out.update(extra)
    if not args.no_cpu:
        v_cpu, t_cpu = cpu_baseline(w, args.cpu_steps)
        log(f"[bench] oracle on host: {v_cpu:.2f} Mcell/s ({t_cpu:.1f} s)")
        out["cpu_baseline"] = {"value": round(v_cpu, 3), "unit": "Mcell-updates/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{args.cpu_steps} steps of the same workload on the full "
                                         f"{w['nx']}x{w['ny']} grid, FP64, 1 thread"}
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
