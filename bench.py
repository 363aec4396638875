"""Benchmark: zone-updates/s of the split compressible-Euler step on one MI355X.

Default workload: 3D periodic Kelvin-Helmholtz layer, 256^3 zones, gamma 5/3,
seeded (numpy default_rng(1)) u_y noise, FP32 state with FP64 dt (the FP64
path runs on the same grid beside it).  A zone-update is one interior zone
advanced one full step (three sweeps plus the fused CFL reduction).  The
state is resident in HBM before the timed region starts.

Prints ONE JSON line (rank 0).  Fields beyond the driver's contract:
  roofline      dominant sweep kernel of the FP32 step: algorithmic HBM
                bytes per launch (5 words read + 5 written per zone) over
                its mean duration, measured with hipEvents on the stream it
                runs on (hydro_profile_step), against the 8 TB/s HBM peak;
  step_roofline the whole step against the same peak (120 B per FP32
                zone-update);
  fp64          the FP64 path on the same grid and its speedup;
  cpu_baseline  the FP64 CPU oracle timed on the host (OpenMP threads).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec per MI355X (FP32 vs FP64) and % of HBM roofline"
HBM_PEAK_GBS = 8000.0
WORKLOAD = ("3D periodic Kelvin-Helmholtz, 256^3 on the unit cube, gamma 5/3, "
            "rho 2|1, u_x +-0.5, p 2.5, seeded u_y noise 0.01, CFL 0.8")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256, help="grid edge")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--config", default="", help="force a kernel configuration")
    ap.add_argument("--copy-only", action="store_true",
                    help="run a plain device copy of the state size (counter scale)")
    return ap.parse_args()


def timed_steps(grid, steps, warmup, torch):
    for _ in range(warmup):
        grid.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        grid.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def profile(grid, steps, torch):
    tot = [0.0, 0.0, 0.0]
    for _ in range(steps):
        ms = grid.profile_step()
        for a in range(3):
            tot[a] += ms[a]
    return [t / steps for t in tot]


def run_gpu(P, prec, args, torch, hydro):
    import numpy as np
    dtype = np.float32 if prec == hydro.FP32 else np.float64
    U = torch.from_numpy(np.ascontiguousarray(P.U.astype(dtype))).to("cuda:0")
    flags = hydro.FLAG_NO_TUNE if args.no_tune else 0
    g = hydro.Grid(U, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
    if args.config:
        g.config = args.config
    sec = timed_steps(g, args.steps, args.warmup, torch)
    err = g.error()
    if err != hydro.HYDRO_OK:
        raise RuntimeError("numeric error flag set during the benchmark")
    kms = profile(g, args.profile_steps, torch) if args.profile_steps > 0 else [0, 0, 0]
    cfg = g.config
    g.close()
    del U
    torch.cuda.empty_cache()
    return sec, kms, cfg


def cpu_baseline(P, steps):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=threads)
    U = P.U.copy()
    t0 = time.perf_counter()
    oracle.run(p, U, steps)
    sec = time.perf_counter() - t0
    zones = P.zones
    return {"value": zones * steps / sec, "unit": "zone-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full steps (one per sweep order) of the same "
                      f"{P.shape[2]}x{P.shape[1]}x{P.shape[0]} KH grid in FP64, "
                      f"CFL dt each step, {sec:.1f} s wall"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md)"}))
        sys.exit(2)
    import torch

    if args.copy_only:
        n = args.n ** 3 * 5
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * n * 4, "launches": 10}))
        return

    import hydro_ic as ic
    from paper_1510_05061_amd import hydro

    P = ic.kh(args.n, seed=1)
    zones = P.zones
    sec32, k32, cfg32 = run_gpu(P, hydro.FP32, args, torch, hydro)
    fp64 = None
    if not args.skip_fp64:
        sec64, k64, cfg64 = run_gpu(P, hydro.FP64, args, torch, hydro)
        fp64 = {"value": zones / sec64, "unit": "zone-updates/s",
                "ms_per_step": sec64 * 1e3,
                "step_roofline_frac": zones / sec64 * 240 / (HBM_PEAK_GBS * 1e9),
                "kernel_ms": {"x": k64[0], "y": k64[1], "z": k64[2]},
                "kernel_gbs": {ax: (zones * 80 / (k64[i] * 1e-3) / 1e9 if k64[i] else 0.0)
                               for i, ax in enumerate("xyz")},
                "config": cfg64,
                "fp32_speedup": sec64 / sec32}

    value = zones / sec32
    # dominant kernel: the sweep with the largest mean duration
    dom = max(range(3), key=lambda a: k32[a])
    bytes_launch = zones * 40                      # 5 words read + 5 written, FP32
    achieved = bytes_launch / (k32[dom] * 1e-3) / 1e9 if k32[dom] > 0 else 0.0
    names = {0: "sweep_x_kernel<float>", 1: "sweep_col_kernel<float, y>",
             2: "sweep_col_kernel<float, z>"}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded KH initial state (numpy default_rng(1)), built on the host",
        "config": {"workload": WORKLOAD, "grid": [args.n] * 3, "zones": zones,
                   "state": "FP32 planes, FP64 dt and CFL reduction",
                   "kernels": cfg32},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": names[dom], "mean_ms": k32[dom],
                     "bytes_per_launch": bytes_launch},
        "step_roofline": {"achieved": value * 120 / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": value * 120 / (HBM_PEAK_GBS * 1e9),
                          "bytes_per_zone_update": 120},
        "kernel_ms": {"x": k32[0], "y": k32[1], "z": k32[2]},
        "fp64": fp64,
    }
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
