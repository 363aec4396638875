"""Benchmark: zone-updates/s of the split compressible-Euler step on one MI355X.

Default workload (`--workload turb`): 3D decaying turbulence, 768^3 zones,
the largest single-GPU grid of the workloads (9.1 GB of FP32 state), gamma
5/3, rho = p = 1, seeded (numpy default_rng(4)) solenoidal velocity in shells
k = 1..8 with E(k) ~ k^-5/3 and rms Mach 0.3; FP32 state with FP64 dt and
totals; the FP64 path runs on the same grid beside it.  Other workloads:
`kh` (Kelvin-Helmholtz 256^3), `rt` (Rayleigh-Taylor 256x256x512, gravity,
reflecting z walls), `batch` (4096 uneven periodic KH patches, one
persistent launch per sweep).  A zone-update is one interior zone advanced
one full step: three sweeps, the fused CFL reduction that sets the next dt
and the fused FP64 conserved totals.  The state is resident in HBM before
the timed region starts; the timed steps are graph replays bracketed by
device synchronisation.

Prints ONE JSON line.  Fields beyond the driver's contract:
  roofline       dominant sweep kernel of the FP32 step: algorithmic HBM
                 bytes per launch (5 words read + 5 written per interior
                 zone) over its mean duration, measured with hipEvent pairs
                 on the stream it runs on (hydro_profile_step), against the
                 8 TB/s HBM peak; `traffic` from rocprofv3 counters when the
                 committed counter summary matches the current kernel source.
                 When the dominant kernel is a fused x+y launch (batch
                 planes or single-grid windows: two sweeps per HBM pass,
                 arithmetic-bound) it is reported as bound "alu":
                 algorithmic flops over its duration against the FP32 vector
                 peak without packed FP32 (78.6 TFLOP/s), and `valu_issue`:
                 its VALU wave instructions per launch from the committed
                 counter summary (SQ_INSTS_VALU) over its duration against
                 the chip's issue rate (one wave64 instruction per SIMD
                 every 4 cycles: 6.144e11/s), the bound that holds it;
  step_roofline  the whole step against the same peak (120 B per FP32
                 zone-update, the three-sweep method's algorithmic bytes);
                 when a step fuses the x and y sweeps it moves 80 B per
                 zone-update, given as hbm_bytes_per_zone_update and
                 hbm_achieved;
  fp64           the FP64 path on the same workload and the FP32 speedup
                 (240 B per FP64 zone-update for the roofline; a step that
                 fuses the x and y sweeps moves 160 B: hbm_bytes_per_zone_update
                 and hbm_achieved in GB/s);
  copy_ceiling   a plain device copy of the same bytes, for context;
  stream_ceiling an in-place read+write pass over the state with no
                 arithmetic (hydro_stream_ceiling): the memory-only ceiling;
  cpu_baseline   the FP64 CPU oracle timed on the host (OpenMP threads) over
                 a bounded sample of the workload;
  per_patch_loop batch only: the same patches stepped one grid at a time
                 (FP32 and FP64), and the batch's speedup over that loop;
  accuracy       fp32_vs_fp64_gpu: per-variable L1 (and max-norm) error of
                 the FP32 path against the FP64 path after the workload's
                 step count, both on the GPU with the same dt sequence;
                 vs_oracle: both GPU paths against the oracle's end state of
                 the CPU sample, replaying the oracle's dt sequence.
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
# MI355X FP32 vector peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops per FMA x 2.4 GHz = 78.6 TFLOP/s.  Packed FP32 doubles it to
# 157.3, but this build turns packed FP32 instructions off, so 78.6 is the
# ceiling its kernels can reach (both are reported).
FP32_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_PACKED_TFLOPS = 157.3
# algorithmic flops of one zone in one sweep: reconstruction, predictor,
# HLLC, update, with each division and square root counted as one
FLOPS_PER_ZONE_SWEEP = 165
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


# steps of the FP32-vs-FP64 side-by-side run per workload (KH and turbulence
# as their workload definitions state; RT and the batch as a matching length)
ACCURACY_STEPS = {"kh": 100, "turb": 50, "rt": 100, "batch": 20}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="turb")
    ap.add_argument("--n", type=int, default=0, help="grid edge (kh, turb)")
    ap.add_argument("--patches", type=int, default=4096)
    ap.add_argument("--pad-rows", type=int, default=32,
                    help="batch: interior rows start on multiples of this many elements "
                         "(0: rows of n + 8 stored back to back)")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU sample (0: about 4e8 zone-updates)")
    ap.add_argument("--skip-accuracy", action="store_true")
    ap.add_argument("--skip-loop", action="store_true",
                    help="batch: skip the per-patch loop baseline")
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="steps of the FP32-vs-FP64 comparison (0: the workload's own)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--config", default="", help="force a kernel configuration")
    ap.add_argument("--skip-diag", action="store_true",
                    help="skip timing the in-situ diagnostics")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a plain device copy of the state size")
    return ap.parse_args()


# --------------------------------------------------------------------------
# workloads (host-side initial data)
# --------------------------------------------------------------------------

def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
        # built in FP64; the FP32 path starts from its round-to-nearest copy
        n = args.n or 768
        return {"kind": "grid", "P": ic.turbulence(n), "grid": [n, n, n]}
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


def build_obj(W, prec, args, torch, hydro, flags=None):
    """The workload's initial state on the GPU in `prec`, wrapped in a Grid or
    Batch.  Returns (obj, state tensor, patch tuples or None)."""
    import numpy as np
    import hydro_ic as ic
    dtype = np.float32 if prec == hydro.FP32 else np.float64
    if flags is None:
        flags = hydro.FLAG_NO_TUNE if args.no_tune else 0
        if W["kind"] == "grid":
            # let the tuner keep the fused x+y step where it is faster
            flags |= hydro.FLAG_FUSE_XY
    if W["kind"] == "grid":
        P = W["P"]
        U = torch.from_numpy(np.ascontiguousarray(P.U.astype(dtype, copy=False))).to("cuda:0")
        obj = hydro.Grid(U, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
        patches = None
    else:
        # interior rows start on 128-byte boundaries (ghost layers kept)
        pool, patches = ic.batch_pool(W["specs"], ng=4, dtype=dtype, pad_rows=args.pad_rows)
        U = torch.from_numpy(pool).to("cuda:0")
        del pool
        obj = hydro.Batch(U, patches, 5.0 / 3.0, flags=flags)
    if args.config:
        obj.config = args.config
    return obj, U, patches


def run_gpu(W, prec, args, torch, hydro):
    log(f"precision {prec}: build and tune")
    obj, U, _ = build_obj(W, prec, args, torch, hydro)
    log(f"precision {prec}: timing with {obj.config}")
    sec = timed_steps(obj, args.steps, args.warmup, torch)
    if obj.error() != hydro.HYDRO_OK:
        raise RuntimeError("numeric error flag set during the benchmark")
    t_end, nsteps = obj.time()
    totals = {"names": ["rho", "mx", "my", "mz", "E", "E+rho*phi"], "values": obj.totals(),
              "after_step": nsteps, "t": t_end,
              "note": "FP64 sums folded into the last sweep of the last timed step"}
    kms = profile(obj, args.profile_steps)
    cfg = obj.config
    state_bytes = U.numel() * U.element_size()
    sms = obj.stream_ceiling(10)
    stream = {"bytes_per_pass": 2 * state_bytes, "mean_ms": sms,
              "gbs": 2 * state_bytes / (sms * 1e-3) / 1e9}
    diag = None
    if prec == hydro.FP32 and not args.skip_diag:
        log("in-situ diagnostics on the evolved state")
        diag = diag_timing(obj, W, args.workload, torch, hydro)
        if W["kind"] != "batch":
            log("reactive source on the evolved state")
            diag["burn"] = burn_timing(obj, W, torch, hydro)
            if args.workload == "kh":
                log("two-level AMR step on the evolved state")
                fl = hydro.FLAG_NO_TUNE if args.no_tune else 0
                diag["amr_level"] = amr_level_timing(U, W, torch, hydro, fl)
                # the fewest ghost layers the step needs (2): smaller fine boxes
                diag["amr_level_g2"] = amr_level_timing(U, W, torch, hydro, fl, g=2)
        else:
            log("AMR operators on the pool")
            diag["amr"] = amr_timing(obj, W, torch, hydro)
    obj.close()
    del U
    torch.cuda.empty_cache()
    return sec, kms, cfg, state_bytes, stream, diag, totals


# FP64 vector peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA
# x 2.4 GHz (one FP64 FMA per lane per cycle)
FP64_VECTOR_PEAK_TFLOPS = 78.6
BURN_SPECIES, BURN_SUBSTEPS = 13, 64


def burn_flops_per_zone(M, nsub):
    """Algorithmic flops of one zone's reactive-source step (a division, exp
    or reciprocal counted as one): temperature 10; per link (-Ta/T, exp, A*,
    h*, 1+, reciprocal) 6; per substep 1 + 3 per later species (fma + mul);
    energy 4 M + 3."""
    return 10 + 6 * (M - 1) + nsub * (1 + 3 * (M - 1)) + 4 * M + 3


def burn_timing(obj, W, torch, hydro, reps=5):
    """Mean device time of the reactive-source step (a 13-species chain,
    64 backward-Euler substeps, every zone starting as species 0) on the
    evolved FP32 state: arithmetic-bound, so reported against the FP64
    vector peak, with the HBM bytes (state and composition read, composition
    and energy written) for context."""
    import numpy as np
    M, n = BURN_SPECIES, BURN_SUBSTEPS
    rng = np.random.default_rng(13)
    A = 10.0 ** rng.uniform(-1, 6, M - 1)
    Ta = rng.uniform(0.0, 3.0, M - 1)
    q = rng.uniform(0.01, 0.1, M - 1)
    X = torch.zeros((M,) + tuple(obj.state.shape[1:]), dtype=obj.state.dtype, device="cuda:0")
    X[0] = 1.0
    dt = 1e-3
    obj.burn(X, A, Ta, q, dt, n)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        obj.burn(X, A, Ta, q, dt, n)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    zones = interior_zones(W)
    flops = burn_flops_per_zone(M, n) * zones
    tf = flops / (ms * 1e-3) / 1e12
    nbytes = zones * 4 * ((5 + M) + (M + 1))
    return {"nspec": M, "nsub": n, "mean_ms": ms, "bound": "alu",
            "flops_per_zone": burn_flops_per_zone(M, n), "achieved": tf,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "bytes": nbytes,
            "gbs": nbytes / (ms * 1e-3) / 1e9,
            "mass_sum_max_err": float((X.double().sum(dim=0) - 1.0).abs().max().item())}


def amr_timing(obj, W, torch, hydro, reps=5):
    """Mean device time of the AMR operators on the batch pool (FP32), run
    after the timed steps: a stored-ghost fill of every patch (ghost shells
    read from and written to the interior edges: 2 x 20 B per ghost cell),
    and restriction and interior prolongation over links pairing each 32^3
    patch with a distinct 64^3 patch at coarse offset (8, 8, 8) (restriction:
    the fine interior read, the 16^3 covered coarse cells written;
    prolongation: the fine interior written, the parents read)."""
    specs = W["specs"]
    ng = 4
    ghost = sum((s.n + 2 * ng) ** 3 - s.n ** 3 for s in specs)
    fine = [i for i, s in enumerate(specs) if s.n == 32]
    coarse = [i for i, s in enumerate(specs) if s.n == 64]
    links = [(f, c, 8, 8, 8) for f, c in zip(fine, coarse)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    def entry(ms, nbytes):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"mean_ms": ms, "bytes": nbytes, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}

    out = {"fill_ghosts": entry(timed(obj.fill_ghosts), ghost * 20 * 2),
           "links": len(links)}
    if links:
        nf = len(links) * 32 ** 3
        out["restrict"] = entry(timed(lambda: obj.restrict(links)), nf * 20 + nf // 8 * 20)
        out["prolong"] = entry(timed(lambda: obj.prolong(links)), nf * 20 + nf // 8 * 20)
    return out


AMR_FINE_N, AMR_FINE_G = 32, 4   # fine interior cells per axis, ghost layers


def amr_level_timing(U, W, torch, hydro, flags, reps=5, g=AMR_FINE_G):
    """Mean device time of one subcycled two-level step (hydro_amr_step,
    FP32) on the evolved single grid: a coarse batch holding a copy of the
    grid, and fine patches of 32^3 cells (g ghost layers: 4 as the batched
    patches store, stored 40^3; 2 is the least the step needs) on a
    lattice of 16^3-coarse-cell blocks two coarse cells apart covering both
    shear layers (y = 1/4 and 3/4), filled by copying each coarse cell into
    its 8 children.  Reported: the step's time, the composite zone-updates
    per second (coarse cells plus two updates of every fine interior cell),
    and the time of the same sweeps as plain batch steps (one coarse step of
    dt, two fine steps of dt/2 over the stored boxes), so the difference is
    the cost of the registers, ghosts, restriction and refluxing."""
    nz, ny, nx = U.shape[1:]
    P = W["P"]
    n = AMR_FINE_N
    m, h = n // 2, g // 2
    lo = h + 2                                  # ceil(g/2) + 1 coarse cells of margin
    xs = list(range(lo, nx - lo - m + 1, m + 2))
    zs = list(range(lo, nz - lo - m + 1, m + 2))
    ys = [ny // 4 - m // 2, 3 * ny // 4 - m // 2]
    offs = [(x, y, z) for z in zs for y in ys for x in xs]
    Cp = U.reshape(-1).clone()
    coarse = hydro.Batch(Cp, [(0, nx, ny, nz, 0) + tuple(P.dx)], P.gamma, P.cfl, P.bc,
                         flags=flags)
    box = n + 2 * g
    per = 5 * box ** 3
    fpool = torch.empty(per * len(offs), dtype=U.dtype, device=U.device)
    for i, (x, y, z) in enumerate(offs):
        sub = U[:, z - h:z + m + h, y - h:y + m + h, x - h:x + m + h]
        up = sub.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3)
        fpool[i * per:(i + 1) * per] = up.reshape(-1)
    fine = hydro.Batch(fpool, [(i * per, box, box, box, 0) + tuple(d / 2 for d in P.dx)
                               for i in range(len(offs))], P.gamma, P.cfl,
                       (hydro.OUTFLOW,) * 6, flags=flags)
    links = [(i, 0) + o for i, o in enumerate(offs)]
    lv = hydro.AmrLevels(coarse, fine, links, g)
    dt = 0.5 * lv.cfl_dt()                     # a dozen steps at a fixed dt

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    ms = timed(lambda: lv.step(dt))
    if coarse.error() != hydro.HYDRO_OK or fine.error() != hydro.HYDRO_OK:
        raise RuntimeError("numeric error flag set in the AMR level step")
    plain = timed(lambda: (coarse.step(dt), fine.step(0.5 * dt), fine.step(0.5 * dt)))
    zc = nx * ny * nz
    zf = len(offs) * n ** 3
    out = {"patches": len(offs), "fine_n": n, "ghosts": g, "mean_ms": ms,
           "coarse_config": coarse.config, "fine_config": fine.config,
           "coarse_zones": zc, "fine_zones": zf,
           "composite_zone_updates_per_s": (zc + 2 * zf) / (ms * 1e-3),
           "plain_steps_ms": plain, "overhead_frac": ms / plain - 1.0}
    coarse.close()
    fine.close()
    del lv, Cp, fpool
    torch.cuda.empty_cache()
    return out


# slab-profile axis and density pair of each single-grid workload: the
# layer's normal (KH: y, RT: z) and its two densities; turbulence has no
# layer (x, and densities around its uniform rho = 1)
DIAG_PROFILE = {"kh": (1, 1.0, 2.0), "rt": (2, 1.0, 2.0), "turb": (0, 0.9, 1.1)}


def diag_timing(obj, W, name, torch, hydro, reps=10):
    """Mean device time (hipEvents on the context's stream, `reps` calls) of
    the in-situ diagnostics on the workload's evolved FP32 state: a Mach
    number PDF (1000 bins; it reads all five planes) and, for a single grid,
    the slab profiles along the layer normal with its mixing width and
    mixedness (20 B read per interior zone each), and the x kinetic-energy
    spectrum (16 B per zone: density and momentum)."""
    zones = interior_zones(W)
    nbytes = zones * 20

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    def entry(ms):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"mean_ms": ms, "bytes": nbytes, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}

    counts = torch.empty(1002, dtype=torch.int64, device="cuda:0")
    res = {"pdf_mach": entry(timed(lambda: obj.pdf(hydro.Q_MACH, 0.0, 2.0, 1000, out=counts)))}
    c = counts.cpu()
    res["pdf_mach"]["mean_mach"] = float(((torch.arange(1000, dtype=torch.float64) + 0.5)
                                          * 0.002 * c[1:1001].double()).sum() / max(1, int(c.sum())))
    if W["kind"] != "batch":
        axis, lo, hi = DIAG_PROFILE[name]
        buf = obj.profile(axis, lo, hi)
        e = entry(timed(lambda: obj.profile(axis, lo, hi, out=buf)))
        h = buf.cpu().numpy()
        e.update({"axis": axis, "rho_lo": lo, "rho_hi": hi, "slabs": (len(h) - 2) // 5,
                  "mixing_width": float(h[-2]), "mixedness": float(h[-1])})
        res["profile"] = e
        nx = W["grid"][0]
        m = nx
        for f in (2, 3):
            while m % f == 0:
                m //= f
        if m == 1 and 2 <= nx <= 1024:
            spec = obj.spectrum()
            es = entry(timed(lambda: obj.spectrum(out=spec)))
            es["bytes"] = zones * 16          # rho and the momentum: 4 planes
            es["gbs"] = es["bytes"] / (es["mean_ms"] * 1e-3) / 1e9
            es["frac"] = es["gbs"] / HBM_PEAK_GBS
            E = spec.cpu().numpy()
            es.update({"kmax": len(E) - 1, "total": float(E.sum()),
                       "E_k1_to_16": [float(v) for v in E[1:17]]})
            res["spectrum_x"] = es
        if all(_fft_len_ok(n) for n in W["grid"]):
            res["spectrum_shell"] = shell_spectrum_timing(obj, W, zones, timed, torch)
    return res


def _fft_len_ok(n):
    m = n
    for f in (2, 3):
        while m % f == 0:
            m //= f
    return m == 1 and 1 <= n <= 1024


def shell_spectrum_timing(obj, W, zones, timed, torch):
    """The shell kinetic-energy spectrum (hydro_diag_spectrum3d): four
    passes, whose algorithmic HBM bytes are the state's density and momentum
    (4 words per zone), the three half spectra (nx/2 + 1 complex FP64 values
    per x-line and component) written, read and written, and read, and
    their power (one FP64 value per half-spectrum point) written and read."""
    nx, ny, nz = W["grid"]
    nbytes, nb = obj.spectrum3d_workspace()
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    out = torch.empty(nb, dtype=torch.float64, device="cuda:0")
    ms = timed(lambda: obj.spectrum3d(out=out, work=work))
    esz = obj.state.element_size()
    half = (nx // 2 + 1) * ny * nz
    alg = zones * 4 * esz + half * (3 * 16 * 4 + 8 * 2)
    gbs = alg / (ms * 1e-3) / 1e9
    E = out.cpu().numpy()
    del work
    return {"mean_ms": ms, "bytes": alg, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "workspace_bytes": nbytes, "shells": nb, "total": float(E.sum()),
            "E_K1_to_16": [float(v) for v in E[1:17]]}


def per_patch_loop(W, prec, npatch, steps, torch, hydro):
    """The batch's first `npatch` patches stepped one by one, each as its own
    grid (hydro_step, one graph launch per patch per step): the baseline that
    the single persistent launch per sweep replaces.  Returns zone-updates/s."""
    import numpy as np
    import hydro_ic as ic
    dtype = np.float32 if prec == hydro.FP32 else np.float64
    grids, zones = [], 0
    for s in W["specs"][:npatch]:
        U = torch.from_numpy(ic.kh_patch(s).astype(dtype)).to("cuda:0")
        grids.append(hydro.Grid(U, 1.0 / s.n, 5.0 / 3.0, flags=hydro.FLAG_NO_TUNE))
        zones += s.n ** 3
    for g in grids:          # warm-up step (first-step CFL, graph upload)
        g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for g in grids:
            g.step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for g in grids:
        g.close()
    del grids
    torch.cuda.empty_cache()
    return zones / sec


# --------------------------------------------------------------------------
# accuracy: L1 errors of a result against a reference of the same workload
# --------------------------------------------------------------------------

VARS = ("rho", "mx", "my", "mz", "E")


def interiors(U, patches):
    """(5, nz, ny, nx) interior views of a grid state or of every patch of a
    pool (ghost layers and row padding excluded)."""
    if patches is None:
        yield U
        return
    for o, nx, ny, nz, ng, _, _, _, rp, sp, pp, io in patches:
        yield U.as_strided((5, nz, ny, nx), (pp, sp, rp, 1), o + io)


class L1:
    """Accumulates sum |q - q_ref| and sum |q_ref| per conserved variable, plus
    the momentum vector measure (component differences summed over the three
    axes over sum |m|_1, meaningful where one component is nearly zero) and
    the max-norm relative error."""

    def __init__(self, torch):
        self.t = torch
        self.num = torch.zeros(5, dtype=torch.float64, device="cuda:0")
        self.den = torch.zeros(5, dtype=torch.float64, device="cuda:0")
        self.dmax = torch.zeros(5, dtype=torch.float64, device="cuda:0")
        self.rmax = torch.zeros(5, dtype=torch.float64, device="cuda:0")

    def add(self, got, ref):
        for v in range(5):
            d = (got[v].to(self.t.float64) - ref[v]).abs_()
            self.num[v] += d.sum()
            self.dmax[v] = self.t.maximum(self.dmax[v], d.max())
            del d
            a = ref[v].abs()
            self.den[v] += a.sum()
            self.rmax[v] = self.t.maximum(self.rmax[v], a.max())
            del a

    def result(self):
        num = self.num.cpu().tolist()
        den = self.den.cpu().tolist()
        dmax = self.dmax.cpu().tolist()
        rmax = self.rmax.cpu().tolist()
        out = {"l1": {VARS[v]: num[v] / max(den[v], 1e-300) for v in range(5)},
               "max_rel": {VARS[v]: dmax[v] / max(rmax[v], 1e-300) for v in range(5)}}
        out["l1"]["m"] = sum(num[1:4]) / max(sum(den[1:4]), 1e-300)
        return out


def replay(W, prec, dts, args, torch, hydro):
    """The workload stepped in `prec` with the given dt sequence (Strang
    parity from step 0).  Returns (state tensor, patches)."""
    obj, U, patches = build_obj(W, prec, args, torch, hydro, flags=hydro.FLAG_NO_TUNE)
    for dt in dts:
        obj.step(dt)
    torch.cuda.synchronize()
    if obj.error() != hydro.HYDRO_OK:
        raise RuntimeError("numeric error flag set during a replay")
    obj.close()
    return U, patches


def side_by_side(W, steps, args, torch, hydro):
    """FP32 against FP64 on the GPU: the FP64 path takes `steps` CFL steps
    (dt from hydro_cfl_dt before each), the FP32 path replays the same dt
    sequence, and the per-variable L1 error of FP32 against FP64 is
    reported."""
    log(f"FP32 vs FP64 side by side, {steps} steps")
    obj, U64, patches = build_obj(W, hydro.FP64, args, torch, hydro,
                                  flags=hydro.FLAG_NO_TUNE)
    dts = []
    for _ in range(steps):
        dt = obj.cfl_dt()
        obj.step(dt)
        dts.append(dt)
    torch.cuda.synchronize()
    obj.close()
    U32, _ = replay(W, hydro.FP32, dts, args, torch, hydro)
    acc = L1(torch)
    for a, b in zip(interiors(U32, patches), interiors(U64, patches)):
        acc.add(a, b)
    out = {"steps": steps, "t": float(sum(dts)), "dt": "CFL of the FP64 path, replayed "
           "in FP32", **acc.result()}
    del U32, U64
    torch.cuda.empty_cache()
    return out


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

def default_cpu_steps(W):
    """Oracle steps of the CPU sample: about 4e8 zone-updates (10-20 s on 16
    host threads), at least one step."""
    if W["kind"] != "grid":
        return 1
    return max(1, min(24, int(4e8 // W["P"].zones)))


ORACLE_1T_ZONES = 4 * 1024 * 1024   # bounded single-thread sample (a few seconds)


def oracle_single_thread(W):
    """The same oracle on one host thread over about 4 M zones of the
    workload: a z-slab of the grid's initial state (its own boundary
    conditions) for one CFL pass and one step, or one step of the leading
    patches of the batch."""
    import numpy as np
    import hydro_ic as ic
    import oracle
    zu, sec = 0, 0.0
    if W["kind"] == "grid":
        P = W["P"]
        nz, ny, nx = P.shape
        depth = max(2, min(nz, ORACLE_1T_ZONES // (ny * nx)))
        U = np.ascontiguousarray(P.U[:, :depth], dtype=np.float64)
        p = oracle.make_params((depth, ny, nx), P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=1)
        t0 = time.perf_counter()
        oracle.step(p, U, oracle.cfl_dt(p, U), 0)
        sec = time.perf_counter() - t0
        zu = depth * ny * nx
        sample = f"one CFL pass and step of a {depth}x{ny}x{nx} z-slab of the grid, 1 thread"
    else:
        n = 0
        for s in W["specs"]:
            if zu >= ORACLE_1T_ZONES:
                break
            p = oracle.make_params((s.n,) * 3, 1.0 / s.n, 5.0 / 3.0, 0.8, nthreads=1)
            U = ic.kh_patch(s)
            t0 = time.perf_counter()
            oracle.step(p, U, oracle.cfl_dt(p, U), 0)
            sec += time.perf_counter() - t0
            zu += s.n ** 3
            n += 1
        sample = f"one CFL pass and step of each of the first {n} patches, 1 thread"
    return {"value": zu / sec, "unit": "zone-updates/s", "cores": 1, "sample": sample}


def host_cpu():
    """nproc and the CPU model of the host the oracle ran on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(W, steps, args, torch, hydro):
    """The FP64 oracle timed on the host over a bounded sample of the
    workload.  Its end state is also the reference of the `vs_oracle`
    accuracy figures: the GPU paths replay the oracle's dt sequence from the
    same initial state and their interiors are compared with it."""
    import numpy as np
    import hydro_ic as ic
    import oracle
    threads = min(16, os.cpu_count() or 1)
    log(f"oracle on {threads} host threads, {steps} step(s)")
    acc32, acc64 = L1(torch), L1(torch)
    if W["kind"] == "grid":
        P = W["P"]
        p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=threads)
        U = np.array(P.U, dtype=np.float64, order="C", copy=True)  # P.U stays the input
        dts = []
        t0 = time.perf_counter()
        for k in range(steps):
            dt = oracle.cfl_dt(p, U)
            oracle.step(p, U, dt, k)
            dts.append(dt)
        sec = time.perf_counter() - t0
        zu = P.zones * steps
        sample = (f"{steps} full steps of the same {W['grid'][0]}x{W['grid'][1]}x"
                  f"{W['grid'][2]} grid in FP64, CFL dt each step, {sec:.1f} s wall")
        ref = torch.from_numpy(U).to("cuda:0")
        del U
        for prec, acc in ((hydro.FP32, acc32), (hydro.FP64, acc64)):
            G, _ = replay(W, prec, dts, args, torch, hydro)
            acc.add(G, ref)
            del G
            torch.cuda.empty_cache()
        del ref
    else:
        specs = W["specs"]
        dx = [1.0 / s.n for s in specs]
        params = [oracle.make_params((s.n,) * 3, d, 5.0 / 3.0, 0.8, nthreads=threads)
                  for s, d in zip(specs, dx)]
        sec = 0.0
        dt = float("inf")
        for s, p in zip(specs, params):       # one global dt, as the batch uses
            U = ic.kh_patch(s)
            t0 = time.perf_counter()
            dt = min(dt, oracle.cfl_dt(p, U))
            sec += time.perf_counter() - t0
        dts = [dt]
        G32, patches = replay(W, hydro.FP32, dts, args, torch, hydro)
        G64, _ = replay(W, hydro.FP64, dts, args, torch, hydro)
        views = zip(interiors(G32, patches), interiors(G64, patches))
        zu = 0
        for s, p, (v32, v64) in zip(specs, params, views):
            U = ic.kh_patch(s)
            t0 = time.perf_counter()
            oracle.step(p, U, dt, 0)
            sec += time.perf_counter() - t0
            zu += s.n ** 3
            ref = torch.from_numpy(U).to("cuda:0")
            acc32.add(v32, ref)
            acc64.add(v64, ref)
        del G32, G64
        torch.cuda.empty_cache()
        sample = (f"one step of all {len(specs)} patches of the batch in FP64 (patch by "
                  f"patch) at one dt, the smallest oracle CFL dt over the patches; CFL "
                  f"pass and step timed, {sec:.1f} s wall")
    base = {"value": zu / sec, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "sample": sample, "single_thread": oracle_single_thread(W), "host": host_cpu()}
    vs = {"steps": len(dts), "t": float(sum(dts)),
          "dt": "the oracle's CFL dt sequence, replayed by both GPU paths",
          "fp32": acc32.result(), "fp64": acc64.result()}
    return base, vs


# --------------------------------------------------------------------------
# counter-based traffic (rocprofv3 --pmc summaries committed under profiles/)
# --------------------------------------------------------------------------

SWEEP_SOURCES = ("euler.hpp", "kernels.hip", "layout.hpp")   # the sweep kernels' code


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1510_05061_amd", "csrc")
    for f in SWEEP_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def counter_entry(workload, kernel, precision):
    """The committed counter summary's entry for `kernel`, or None when it is
    missing or was taken on different kernel source."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    for e in data.get("entries", []):
        if e.get("workload") == workload and e.get("kernel") == kernel and \
                e.get("precision") == precision:
            return e
    return None


def counter_traffic(workload, kernel, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None (see counter_entry)."""
    e = counter_entry(workload, kernel, precision)
    return e.get("bytes_per_launch") if e else None


# VALU issue rate of MI355X: each of the 4 SIMDs of a CU starts one wave64
# instruction every 4 cycles (16 lanes per cycle), so 256 CUs at 2.4 GHz
# issue 256 x 2.4e9 = 6.144e11 wave instructions per second
VALU_WAVE_ISSUE_PER_S = 256 * 2.4e9


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the path would shard as z-slabs, one per GPU, with a 2-cell halo "
                                   "exchange before each z sweep and a max all-reduce of the CFL rate)"}))
        sys.exit(2)
    import torch

    if args.copy_only:
        n = args.n or 256
        print(json.dumps(copy_ceiling(torch, 5 * n ** 3 * 4)))
        return

    from paper_1510_05061_amd import hydro

    W = make_workload(args)
    zones = interior_zones(W)
    sec32, k32, cfg32, bytes32, stream32, diag32, tot32 = run_gpu(W, hydro.FP32, args, torch,
                                                                  hydro)
    fp64 = None
    if not args.skip_fp64:
        sec64, k64, cfg64, _, stream64, _, tot64 = run_gpu(W, hydro.FP64, args, torch, hydro)
        fp64 = {"value": zones / sec64, "unit": "zone-updates/s",
                "ms_per_step": sec64 * 1e3,
                "step_roofline_frac": zones / sec64 * 240 / (HBM_PEAK_GBS * 1e9),
                "hbm_bytes_per_zone_update": 160 if "f=1" in cfg64 else 240,
                "hbm_achieved": zones / sec64 * (160 if "f=1" in cfg64 else 240) / 1e9,
                "kernel_ms": {"x": k64[0], "y": k64[1], "z": k64[2]},
                "kernel_gbs": {ax: (zones * 80 / (k64[i] * 1e-3) / 1e9 if k64[i] else 0.0)
                               for i, ax in enumerate("xyz")},
                "config": cfg64,
                "stream_ceiling": stream64,
                "totals": tot64,
                "fp32_speedup": sec64 / sec32}

    value = zones / sec32
    dom = max(range(3), key=lambda a: k32[a])
    bytes_launch = zones * 40                      # 5 words read + 5 written, FP32
    achieved = bytes_launch / (k32[dom] * 1e-3) / 1e9 if k32[dom] > 0 else 0.0
    pers = W["kind"] == "batch"
    fused = "f=1" in cfg32
    xpart = cfg32.split(";")[0]                      # x:v=V,b=B[,m=1[,g=G]]
    xv = xpart.split("v=")[1].split(",")[0]
    names = {0: (f"sweep_xm_kernel<float,{xv}>" if "m=1" in xpart
                 else f"sweep_x_kernel<float,{xv}>"),
             1: "sweep_col_kernel<float,1>", 2: "sweep_col_kernel<float,2>"}
    if fused and pers:   # one launch does the x and y sweeps of every patch z-plane
        names[0] = "sweep_plane_kernel<float> (x and y sweeps fused)"
    elif fused:          # one launch does the x and y sweeps, 64 x 64 windows per z-plane
        names[0] = "sweep_window_kernel<float> (x and y sweeps fused)"
    kname = names[dom] + (" (persistent)" if pers else "")
    hbm_per_zu = 80 if fused else 120
    traffic = counter_traffic(args.workload, names[dom].split(" (")[0], "fp32")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
            "mean_ms": k32[dom], "bytes_per_launch": bytes_launch}
    if fused and dom == 0:
        # the fused launch does two sweeps per HBM pass and is bound by its
        # arithmetic: algorithmic flops (FLOPS_PER_ZONE_SWEEP per zone per
        # sweep) over its duration against the FP32 vector peak
        flops = 2 * FLOPS_PER_ZONE_SWEEP * zones
        tf = flops / (k32[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tf / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                "kernel": kname, "mean_ms": k32[dom], "flops_per_launch": flops,
                "flops_per_zone_sweep": FLOPS_PER_ZONE_SWEEP, "hbm_bytes_per_launch": bytes_launch,
                "hbm_gbs": achieved, "peak_packed": FP32_VECTOR_PEAK_PACKED_TFLOPS}
        # what binds it: its counted VALU instructions (SQ_INSTS_VALU from the
        # committed counter summary) over its duration against the issue rate
        e = counter_entry(args.workload, names[dom].split(" (")[0], "fp32")
        if e and e.get("valu_wave_insts_per_launch"):
            wi = e["valu_wave_insts_per_launch"]
            roof["valu_issue"] = {"wave_insts_per_launch": wi,
                                  "achieved_per_s": wi / (k32[dom] * 1e-3),
                                  "peak_per_s": VALU_WAVE_ISSUE_PER_S,
                                  "frac": wi / (k32[dom] * 1e-3) / VALU_WAVE_ISSUE_PER_S}
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
                   "state": "FP32 planes; FP64 dt, CFL reduction and conserved totals",
                   "kernels": cfg32},
        "totals": tot32,
        "roofline": roof,
        "step_roofline": {"achieved": value * 120 / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": value * 120 / (HBM_PEAK_GBS * 1e9),
                          "bytes_per_zone_update": 120,
                          "hbm_bytes_per_zone_update": hbm_per_zu,
                          "hbm_achieved": value * hbm_per_zu / 1e9},
        "kernel_ms": {"x": k32[0], "y": k32[1], "z": k32[2]},
        "fp64": fp64,
        "copy_ceiling": copy_ceiling(torch, bytes32),
        "stream_ceiling": stream32,
        "kernel_source": kernel_source_hash(),
        "diagnostics": diag32,
    }
    if W["kind"] == "batch" and not args.skip_loop:
        npl = min(len(W["specs"]), 1024)
        log(f"per-patch loop over {npl} patches")
        l32 = per_patch_loop(W, hydro.FP32, npl, 5, torch, hydro)
        l64 = per_patch_loop(W, hydro.FP64, npl, 5, torch, hydro)
        out["per_patch_loop"] = {
            "sample": f"the first {npl} patches, each its own grid stepped by hydro_step "
                      "(one graph launch per patch per step), 5 timed steps",
            "fp32": l32, "fp64": l64, "unit": "zone-updates/s",
            "batch_fp32_over_loop_fp32": value / l32,
            "batch_fp32_over_loop_fp64": value / l64}
    acc = {}
    if not args.skip_accuracy:
        steps = args.accuracy_steps or ACCURACY_STEPS[args.workload]
        acc["fp32_vs_fp64_gpu"] = side_by_side(W, steps, args, torch, hydro)
    if not args.skip_cpu:
        steps = args.cpu_steps or default_cpu_steps(W)
        out["cpu_baseline"], acc["vs_oracle"] = cpu_baseline(W, steps, args, torch, hydro)
    out["accuracy"] = acc or None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
