"""Benchmark: zone-updates/s of the split compressible-Euler step on one MI355X.

Default workload (`--workload kh`): 3D periodic Kelvin-Helmholtz layer,
256^3 zones, gamma 5/3, seeded (numpy default_rng(1)) u_y noise, FP32 state
with FP64 dt; the FP64 path runs on the same grid beside it.  Other
workloads: `rt` (Rayleigh-Taylor 256x256x512, gravity, reflecting z walls),
`turb` (decaying turbulence 768^3), `batch` (4096 uneven periodic KH patches,
one persistent launch per sweep).  A zone-update is one interior zone
advanced one full step (three sweeps plus the fused CFL reduction).  The
state is resident in HBM before the timed region starts; the timed steps are
graph replays bracketed by device synchronisation.

Prints ONE JSON line.  Fields beyond the driver's contract:
  roofline       dominant sweep kernel of the FP32 step: algorithmic HBM
                 bytes per launch (5 words read + 5 written per interior
                 zone) over its mean duration, measured with hipEvent pairs
                 on the stream it runs on (hydro_profile_step), against the
                 8 TB/s HBM peak; `traffic` from rocprofv3 counters when the
                 committed counter summary matches the current kernel source;
  step_roofline  the whole step against the same peak (120 B per FP32
                 zone-update);
  fp64           the FP64 path on the same workload and the FP32 speedup;
  copy_ceiling   a plain device copy of the same bytes, for context;
  cpu_baseline   the FP64 CPU oracle timed on the host (OpenMP threads).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec per MI355X (FP32 vs FP64) and % of HBM roofline"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")

WORKLOADS = {
    "kh": "3D periodic Kelvin-Helmholtz, 256^3 on the unit cube, gamma 5/3, rho 2|1, "
          "u_x +-0.5, p 2.5, seeded u_y noise 0.01, CFL 0.8",
    "rt": "3D Rayleigh-Taylor, 256x256x512 on [0,0.5]^2x[0,1], gamma 1.4, g=-0.1 along z, "
          "rho 2 over 1, hydrostatic p (2.5 at the interface), seeded interface u_z "
          "0.01, reflecting z walls, periodic x/y",
    "turb": "3D decaying turbulence, 768^3 periodic, gamma 5/3, rho=p=1, solenoidal "
            "random-phase velocity in shells k=1..8, E(k)~k^-5/3, rms Mach 0.3",
    "batch": "4096 independent periodic KH patches, edges from {16,32,48,64} (seeded), "
             "4 stored ghost layers, rows padded so each interior row starts on a 128-byte "
             "boundary, gamma 5/3, shear 0.1-1.0, density ratio 1-4; one persistent launch "
             "per sweep, hipGraph step, one global dt",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="kh")
    ap.add_argument("--n", type=int, default=0, help="grid edge (kh, turb)")
    ap.add_argument("--patches", type=int, default=4096)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--config", default="", help="force a kernel configuration")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a plain device copy of the state size")
    return ap.parse_args()


# --------------------------------------------------------------------------
# workloads (host-side initial data)
# --------------------------------------------------------------------------

def make_workload(args):
    import numpy as np
    import hydro_ic as ic
    w = args.workload
    if w == "kh":
        n = args.n or 256
        return {"kind": "grid", "P": ic.kh(n, seed=1), "grid": [n, n, n]}
    if w == "rt":
        return {"kind": "grid", "P": ic.rt(), "grid": [256, 256, 512]}
    if w == "turb":
        n = args.n or 768
        return {"kind": "grid", "P": ic.turbulence(n, dtype=np.float32), "grid": [n, n, n]}
    specs = ic.batch_specs(args.patches, seed=3)
    return {"kind": "batch", "specs": specs, "grid": None}


def interior_zones(W):
    if W["kind"] == "grid":
        return W["P"].zones
    return sum(s.n ** 3 for s in W["specs"])


# --------------------------------------------------------------------------
# GPU runs
# --------------------------------------------------------------------------

def timed_steps(obj, steps, warmup, torch):
    for _ in range(warmup):
        obj.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        obj.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def profile(obj, steps):
    tot = [0.0, 0.0, 0.0]
    for _ in range(steps):
        ms = obj.profile_step()
        for a in range(3):
            tot[a] += ms[a]
    return [t / max(1, steps) for t in tot]


def run_gpu(W, prec, args, torch, hydro):
    import numpy as np
    import hydro_ic as ic
    dtype = np.float32 if prec == hydro.FP32 else np.float64
    flags = hydro.FLAG_NO_TUNE if args.no_tune else 0
    if W["kind"] == "grid":
        P = W["P"]
        U = torch.from_numpy(np.ascontiguousarray(P.U.astype(dtype, copy=False))).to("cuda:0")
        obj = hydro.Grid(U, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
    else:
        # interior rows start on 128-byte boundaries (ghost layers kept)
        pool, patches = ic.batch_pool(W["specs"], ng=4, dtype=dtype, pad_rows=32)
        U = torch.from_numpy(pool).to("cuda:0")
        del pool
        obj = hydro.Batch(U, patches, 5.0 / 3.0, flags=flags)
    if args.config:
        obj.config = args.config
    sec = timed_steps(obj, args.steps, args.warmup, torch)
    if obj.error() != hydro.HYDRO_OK:
        raise RuntimeError("numeric error flag set during the benchmark")
    kms = profile(obj, args.profile_steps)
    cfg = obj.config
    obj.close()
    state_bytes = U.numel() * U.element_size()
    del U
    torch.cuda.empty_cache()
    return sec, kms, cfg, state_bytes


def copy_ceiling(torch, nbytes_state, reps=20):
    """Device-to-device copy of a buffer of the FP32 state size: read + write
    bytes over the mean kernel time (context for the streaming kernels)."""
    words = nbytes_state // 4
    a = torch.ones(words, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * words * 4
    del a, b
    torch.cuda.empty_cache()
    return {"copy_bytes_per_launch": nbytes, "mean_ms": ms,
            "gbs": nbytes / (ms * 1e-3) / 1e9, "launches": reps + 3}


# --------------------------------------------------------------------------
# CPU baseline (the oracle as it stands)
# --------------------------------------------------------------------------

def cpu_baseline(W, steps):
    import numpy as np
    import hydro_ic as ic
    import oracle
    threads = min(16, os.cpu_count() or 1)
    if W["kind"] == "grid":
        P = W["P"]
        p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=threads)
        U = np.ascontiguousarray(P.U, dtype=np.float64)
        t0 = time.perf_counter()
        oracle.run(p, U, steps)
        sec = time.perf_counter() - t0
        zu = P.zones * steps
        sample = (f"{steps} full steps of the same {W['grid'][0]}x{W['grid'][1]}x"
                  f"{W['grid'][2]} grid in FP64, CFL dt each step, {sec:.1f} s wall")
    else:
        specs = W["specs"][:256]
        zu = 0
        sec = 0.0
        for s in specs:
            U = ic.kh_patch(s)
            p = oracle.make_params(U.shape[1:], 1.0 / s.n, 5.0 / 3.0, 0.8, nthreads=threads)
            t0 = time.perf_counter()
            oracle.run(p, U, 1)
            sec += time.perf_counter() - t0
            zu += s.n ** 3
        sample = (f"one step of each of the first {len(specs)} patches of the batch in FP64 "
                  f"(patch by patch), {sec:.1f} s wall")
    return {"value": zu / sec, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "sample": sample}


# --------------------------------------------------------------------------
# counter-based traffic (rocprofv3 --pmc summaries committed under profiles/)
# --------------------------------------------------------------------------

def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1510_05061_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(workload, kernel, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or was taken on different kernel source."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    for e in data.get("entries", []):
        if e.get("workload") == workload and e.get("kernel") == kernel and \
                e.get("precision") == precision:
            return e.get("bytes_per_launch")
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md)"}))
        sys.exit(2)
    import torch

    if args.copy_only:
        n = args.n or 256
        print(json.dumps(copy_ceiling(torch, 5 * n ** 3 * 4)))
        return

    from paper_1510_05061_amd import hydro

    W = make_workload(args)
    zones = interior_zones(W)
    sec32, k32, cfg32, bytes32 = run_gpu(W, hydro.FP32, args, torch, hydro)
    fp64 = None
    if not args.skip_fp64:
        sec64, k64, cfg64, _ = run_gpu(W, hydro.FP64, args, torch, hydro)
        fp64 = {"value": zones / sec64, "unit": "zone-updates/s",
                "ms_per_step": sec64 * 1e3,
                "step_roofline_frac": zones / sec64 * 240 / (HBM_PEAK_GBS * 1e9),
                "kernel_ms": {"x": k64[0], "y": k64[1], "z": k64[2]},
                "kernel_gbs": {ax: (zones * 80 / (k64[i] * 1e-3) / 1e9 if k64[i] else 0.0)
                               for i, ax in enumerate("xyz")},
                "config": cfg64,
                "fp32_speedup": sec64 / sec32}

    value = zones / sec32
    dom = max(range(3), key=lambda a: k32[a])
    bytes_launch = zones * 40                      # 5 words read + 5 written, FP32
    achieved = bytes_launch / (k32[dom] * 1e-3) / 1e9 if k32[dom] > 0 else 0.0
    pers = W["kind"] == "batch"
    names = {0: "sweep_x_kernel<float>", 1: "sweep_col_kernel<float,1>",
             2: "sweep_col_kernel<float,2>"}
    kname = names[dom] + (" (persistent)" if pers else "")
    traffic = counter_traffic(args.workload, names[dom], "fp32")
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
        "data": "synthetic: seeded initial state built on the host (numpy)",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload,
                   "grid": W["grid"], "zones": zones,
                   "state": "FP32 planes, FP64 dt and CFL reduction", "kernels": cfg32},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "mean_ms": k32[dom], "bytes_per_launch": bytes_launch},
        "step_roofline": {"achieved": value * 120 / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": value * 120 / (HBM_PEAK_GBS * 1e9),
                          "bytes_per_zone_update": 120},
        "kernel_ms": {"x": k32[0], "y": k32[1], "z": k32[2]},
        "fp64": fp64,
        "copy_ceiling": copy_ceiling(torch, bytes32),
        "kernel_source": kernel_source_hash(),
    }
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_steps if W["kind"] == "grid" else 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
