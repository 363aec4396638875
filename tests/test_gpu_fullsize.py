"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (autotuned kernels, graph-replayed steps).

KH 256^3 is checked whole against the oracle; RT 256x256x512, turbulence
768^3 and the 4096-patch batch are checked on sampled blocks or patches that
the oracle computes on its own (a block's centre is exact when the block
carries 2 extra cells on every side), plus properties that hold at any size.
"""
import math

import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import (grid_scale, host, l1_fp32_errors, max_fp32_errors, oracle_box_step, params_of,
                      rel_err, say, sub_box, sub_box_dev, torch)
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

THREADS = 16


def _grid(P, prec, U=None):
    t = torch()
    dt = np.float64 if prec == hydro.FP64 else np.float32
    src = P.U if U is None else U
    dev = t.from_numpy(np.ascontiguousarray(src.astype(dt, copy=False))).to("cuda:0")
    return hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav), dev


def test_kh256_fp64_two_steps_match_oracle():
    say("kh256 fp64 full")
    P = ic.kh(256, seed=1)
    p = params_of(P, nthreads=THREADS)
    g, dev = _grid(P, hydro.FP64)
    state = P.U.copy()
    for step in range(2):
        dt = oracle.cfl_dt(p, state)
        if step == 0:
            assert abs(g.cfl_dt() - dt) <= 1e-14 * dt
        g.step(dt)
        oracle.step(p, state, dt, step)
        err = rel_err(host(dev), state)
        say(f"  step {step} rel err {max(err):.2e}")
        assert max(err) <= 1e-12, err
        dev.copy_(torch().from_numpy(state).to("cuda:0"))
        g.state_changed()
    g.close()


def test_kh256_fp32_step_l1():
    say("kh256 fp32 full")
    P = ic.kh(256, seed=1)
    U32 = P.U.astype(np.float32)
    U64 = U32.astype(np.float64)
    p = params_of(P, nthreads=THREADS)
    dt = oracle.cfl_dt(p, U64)
    g, dev = _grid(P, hydro.FP32, U=U32)
    g.step(dt)
    oracle.step(p, U64, dt, 0)
    out = host(dev)
    e = l1_fp32_errors(out, U64)
    mx = max_fp32_errors(out, U64)
    say(f"  L1 (rho, m, E) {e} max {mx}")
    assert max(e) <= 2e-6
    assert max(mx) <= 1e-5
    g.close()


def test_rt_full_sampled_blocks_and_invariants():
    say("rt full")
    P = ic.rt()                       # 256 x 256 x 512, reflecting z walls
    prec = hydro.FP64
    g, dev = _grid(P, prec)
    p = params_of(P, nthreads=THREADS)
    dt = oracle.cfl_dt(p, P.U)
    assert abs(g.cfl_dt() - dt) <= 1e-14 * dt
    t0 = np.array(g.totals())
    ref_tot = oracle.totals(p, P.U)
    assert np.all(np.abs(t0 - ref_tot) <= 1e-13 * np.abs(ref_tot) + 1e-13)
    g.step(dt)
    out = host(dev)
    scale = grid_scale(out)
    # interior blocks (away from the z walls: the box wraps periodically)
    rng = np.random.default_rng(0)
    m = 12
    for _ in range(6):
        corner = (int(rng.integers(4, 512 - m - 4)), int(rng.integers(0, 256)),
                  int(rng.integers(0, 256)))
        want = oracle_box_step(P.U, corner, m, P, dt, 0)
        got = sub_box(out, *corner, m)
        err = rel_err(got, want, scale)
        assert max(err) <= 1e-12, (corner, err)
    # blocks touching the walls: run the oracle on a full-height column
    for x0, y0 in ((5, 7), (200, 100)):
        col = np.ascontiguousarray(
            P.U[:, :, (np.arange(y0 - 2, y0 + 14) % 256)[:, None],
                (np.arange(x0 - 2, x0 + 14) % 256)[None, :]])
        q = oracle.make_params(col.shape[1:], P.dx, P.gamma, P.cfl,
                               (1, 1, 1, 1, ic.REFLECT, ic.REFLECT), P.grav)
        oracle.step(q, col, dt, 0)
        want = col[:, :, 2:-2, 2:-2]
        got = np.ascontiguousarray(
            out[:, :, (np.arange(y0, y0 + 12) % 256)[:, None],
                (np.arange(x0, x0 + 12) % 256)[None, :]])
        err = rel_err(got, want, scale)
        assert max(err) <= 1e-12, ((x0, y0), err)
    # mass, transverse momenta and E + rho*phi are conserved by the step
    t1 = np.array(g.totals())
    for v in (0, 1, 2, 5):
        assert abs(t1[v] - t0[v]) <= 1e-13 * max(1.0, abs(t0[v])), (v, t0, t1)
    g.close()


def test_rt_full_fp32_sampled_blocks_and_walls():
    """The RT workload as bench.py runs it (FP32 state, reflecting z walls,
    gravity, autotuned kernels, graph step), one step from the FP32-rounded
    initial state against the oracle on sampled interior blocks and on
    full-height columns through both walls.  rho and E: L1 per block within
    the one-step bound 2e-6 and per cell within 1e-5 of the grid's largest
    value.  The layer starts near rest (|m| <= 0.02), and the rounding of
    its momentum comes from the momentum flux rho u^2 + p ~ p; so momentum
    is measured per cell against the acoustic scale max(rho) max(c) (also
    1e-5), not against its own tiny magnitude."""
    say("rt full fp32")
    P = ic.rt()
    U32 = P.U.astype(np.float32)
    U64 = U32.astype(np.float64)
    p = params_of(P, nthreads=THREADS)
    dt = oracle.cfl_dt(p, U64)
    g, dev = _grid(P, hydro.FP32, U=U32)
    say(f"  config {g.config}")
    g.step(dt)
    out = host(dev)
    rho_max = float(np.abs(U64[0]).max())
    E_max = float(np.abs(U64[4]).max())
    pr = (P.gamma - 1.0) * (U64[4] - 0.5 * (U64[1] ** 2 + U64[2] ** 2 + U64[3] ** 2) / U64[0])
    m_acoustic = rho_max * float(np.sqrt(P.gamma * pr / U64[0]).max())
    del pr

    def check(got, want, where):
        e = l1_fp32_errors(got, want)
        assert e[0] <= 2e-6 and e[2] <= 2e-6, (where, e)
        mx = (np.abs(got[0] - want[0]).max() / rho_max,
              np.abs(got[1:4] - want[1:4]).max() / m_acoustic,
              np.abs(got[4] - want[4]).max() / E_max)
        assert max(mx) <= 1e-5, (where, mx)

    rng = np.random.default_rng(3)
    m = 12
    for _ in range(6):
        corner = (int(rng.integers(4, 512 - m - 4)), int(rng.integers(0, 256)),
                  int(rng.integers(0, 256)))
        want = oracle_box_step(U64, corner, m, P, dt, 0)
        check(sub_box(out, *corner, m), want, corner)
    for x0, y0 in ((9, 250), (131, 60)):
        col = np.ascontiguousarray(
            U64[:, :, (np.arange(y0 - 2, y0 + 14) % 256)[:, None],
                (np.arange(x0 - 2, x0 + 14) % 256)[None, :]])
        q = oracle.make_params(col.shape[1:], P.dx, P.gamma, P.cfl,
                               (1, 1, 1, 1, ic.REFLECT, ic.REFLECT), P.grav)
        oracle.step(q, col, dt, 0)
        want = col[:, :, 2:-2, 2:-2]
        got = np.ascontiguousarray(
            out[:, :, (np.arange(y0, y0 + 12) % 256)[:, None],
                (np.arange(x0, x0 + 12) % 256)[None, :]])
        check(got, want, (x0, y0))
        # the wall rows themselves (first and last two z layers)
        for zs in (slice(0, 2), slice(-2, None)):
            check(got[:, zs], want[:, zs], ((x0, y0), zs))
    assert g.error() == hydro.HYDRO_OK
    g.close()


@pytest.fixture(scope="module")
def turb768():
    """The 768^3 turbulence initial state in FP64 (18 GB on the host), built
    once for the tests of both precisions."""
    say("building the 768^3 turbulence state")
    P = ic.turbulence(768)
    yield P
    del P


def _turb_blocks(P, U_in, dev, dt, corners, m, nsteps):
    """Oracle steps of (m + 4 nsteps)^3 boxes of U_in around each sampled
    corner (the centre m^3 is exact after nsteps steps) beside the same
    blocks gathered from the device state."""
    g = 2 * nsteps
    for corner in corners:
        block_in = sub_box(U_in, corner[0] - g, corner[1] - g, corner[2] - g, m + 2 * g)
        block_in = block_in.astype(np.float64)
        q = oracle.make_params(block_in.shape[1:], P.dx, P.gamma, P.cfl, (1,) * 6)
        for s in range(nsteps):
            oracle.step(q, block_in, dt, s)
        want = block_in[:, g:-g, g:-g, g:-g]
        got = sub_box_dev(dev, *corner, m).cpu().numpy().astype(np.float64)
        yield corner, got, want


def test_turbulence768_fp32_sampled_blocks(turb768):
    """Two steps (both Strang orders; the second ends with the x sweep, which
    folds the CFL maximum) at one dt from the oracle; 12^3 blocks checked
    against the oracle run on a (12+8)^3 box of the input (the centre is
    exact after two steps)."""
    say("turbulence 768 fp32")
    P = turb768
    U32 = P.U.astype(np.float32)
    p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=THREADS)
    dt = oracle.cfl_dt(p, U32.astype(np.float64))
    g, dev = _grid(P, hydro.FP32, U=U32)
    say(f"  config {g.config}")
    g.step(dt)
    g.step(dt)
    torch().cuda.synchronize()
    rng = np.random.default_rng(1)
    corners = [tuple(int(v) for v in rng.integers(0, 768, size=3)) for _ in range(8)]
    for corner, got, want in _turb_blocks(P, U32, dev, dt, corners, 12, 2):
        e = l1_fp32_errors(got, want)
        assert max(e) <= 4e-6, (corner, e)
    assert g.error() == hydro.HYDRO_OK
    g.close()
    del dev, U32
    torch().cuda.empty_cache()


def test_turbulence768_fp64_tuned_fused_and_wide_x_lane_runs(turb768):
    """The FP64 path at 768^3 in the autotuned configuration bench.py times
    (the fused x+y step allowed), the fused step forced (64 x 32 windows) and
    separate sweeps with x lane runs of 4 cells over three waves per pencil
    (x:v=4,b=192): two steps at the oracle's dt, sampled 12^3 blocks against
    the oracle to 1e-12 of the grid's scale, and the configurations bit for
    bit equal on the sampled blocks."""
    P = turb768
    p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=THREADS)
    dt = oracle.cfl_dt(p, P.U)
    scale = grid_scale(P.U)
    t = torch()
    src = t.from_numpy(P.U).to("cuda:0")
    rng = np.random.default_rng(5)
    corners = [tuple(int(v) for v in rng.integers(0, 768, size=3)) for _ in range(6)]
    first = None
    for flags, cfg in ((hydro.FLAG_FUSE_XY, None),
                       (hydro.FLAG_NO_TUNE | hydro.FLAG_FUSE_XY,
                        "x:v=4,b=192;y:q=256,s=1;z:q=256,s=1;p:f=1;w:v=2,b=256"),
                       (0, "x:v=4,b=192")):
        dev = src.clone()
        g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
        if cfg:
            g.config = cfg
        say(f"turbulence 768 fp64 {g.config}")
        assert abs(g.cfl_dt() - dt) <= 1e-14 * dt
        g.step(dt)
        g.step(dt)
        t.cuda.synchronize()
        blocks = []
        for corner, got, want in _turb_blocks(P, P.U, dev, dt, corners, 12, 2):
            err = rel_err(got, want, scale)
            assert max(err) <= 1e-12, (g.config, corner, err)
            blocks.append(got)
        if first is None:
            first = blocks
        else:
            for a, b in zip(first, blocks):
                np.testing.assert_array_equal(a, b)
        assert g.error() == hydro.HYDRO_OK
        g.close()
        del dev
        t.cuda.empty_cache()
    del src
    t.cuda.empty_cache()




def test_turbulence768_fp32_fused_step(turb768):
    """The benchmark's FP32 launch configuration: the fused x+y step (64 x 64
    windows written to the second buffer, the z march writing back) in the
    configuration its tuner keeps, two steps (both Strang orders) at the
    oracle's dt.  The whole state equals the separate sweeps' bit for bit
    (compared on the device), and sampled 12^3 blocks match the oracle."""
    P = turb768
    U32 = P.U.astype(np.float32)
    p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, nthreads=THREADS)
    dt = oracle.cfl_dt(p, U32.astype(np.float64))
    t = torch()
    src = t.from_numpy(U32).to("cuda:0")
    out = []
    for flags, cfg in ((hydro.FLAG_NO_TUNE | hydro.FLAG_FUSE_XY,
                        "x:v=4,b=256,m=1;y:q=256,s=2;z:q=128,s=4;p:f=1;w:v=2,b=512"),
                       (hydro.FLAG_NO_TUNE, "x:v=4,b=256,m=1;y:q=256,s=2;z:q=128,s=4")):
        dev = src.clone()
        g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
        g.config = cfg
        say(f"turbulence 768 fp32 {g.config}")
        g.step(dt)
        g.step(dt)
        t.cuda.synchronize()
        assert g.error() == hydro.HYDRO_OK
        out.append((dev, g.totals()))
        g.close()
    assert bool(t.equal(out[0][0], out[1][0]))
    for v in range(6):
        assert abs(out[0][1][v] - out[1][1][v]) <= 1e-12 * max(1.0, abs(out[1][1][v]))
    rng = np.random.default_rng(7)
    corners = [tuple(int(v) for v in rng.integers(0, 768, size=3)) for _ in range(4)]
    for corner, got, want in _turb_blocks(P, U32, out[0][0], dt, corners, 12, 2):
        e = l1_fp32_errors(got, want)
        assert max(e) <= 4e-6, (corner, e)
    del out, src
    t.cuda.empty_cache()

@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
def test_turbulence768_shell_spectrum(turb768, prec):
    """The shell spectrum at full size: the initial data's closed form
    (rho = 1, every shell K = 1..8 holding vrms^2 K^(-5/3) / sum_K' K'^(-5/3)
    of <|v|^2>, nothing elsewhere) and Parseval against <|u|^2> / 2 reduced
    by torch from the device state."""
    P = turb768
    t = torch()
    dt = np.float64 if prec == hydro.FP64 else np.float32
    dev = t.from_numpy(P.U.astype(dt, copy=False)).to("cuda:0")
    g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=hydro.FLAG_NO_TUNE)
    say(f"turbulence 768 shell spectrum prec={prec}")
    E = g.spectrum3d().cpu().numpy()
    assert E.shape == (666,)
    r = dev[0].double()
    half_u2 = 0.5 * sum(((dev[c].double() / r) ** 2).mean() for c in (1, 2, 3)).item()
    del r
    np.testing.assert_allclose(E.sum(), half_u2, rtol=1e-12 if prec == hydro.FP64 else 1e-10)
    vrms2 = 0.3 * 0.3 * (5.0 / 3.0)
    K = np.arange(1, 9)
    want = 0.5 * vrms2 * K ** (-5.0 / 3.0) / np.sum(K ** (-5.0 / 3.0))
    np.testing.assert_allclose(E[1:9], want, rtol=1e-10 if prec == hydro.FP64 else 1e-6)
    rest = np.concatenate([E[:1], E[9:]])
    assert rest.max() < (1e-20 if prec == hydro.FP64 else 1e-12) * E.sum()
    g.close()
    del dev
    t.cuda.empty_cache()

def test_batch4096_fp32_sampled_patches():
    say("batch 4096 fp32")
    specs = ic.batch_specs(4096, seed=3)
    pool, patches = ic.batch_pool(specs, ng=4, dtype=np.float32, pad_rows=32)
    t = torch()
    dev = t.from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, 5.0 / 3.0)
    # one global dt: the smallest oracle CFL dt over the patches
    dt = math.inf
    for pch in patches:
        ng = pch[4]
        u = np.ascontiguousarray(ic.patch_view(pool, pch)[:, ng:-ng, ng:-ng, ng:-ng],
                                 dtype=np.float64)
        prm = oracle.make_params(u.shape[1:], pch[5], 5.0 / 3.0, 0.8, nthreads=THREADS)
        dt = min(dt, oracle.cfl_dt(prm, u))
    assert abs(b.cfl_dt() - dt) <= 1e-6 * dt   # FP32 state: speeds in FP32
    b.step(dt)
    out = dev.cpu().numpy()
    rng = np.random.default_rng(2)
    for i in rng.choice(len(patches), size=24, replace=False):
        pch = patches[int(i)]
        ng = pch[4]
        full_in = ic.patch_view(pool, pch)
        interior = np.ascontiguousarray(full_in[:, ng:-ng, ng:-ng, ng:-ng]).astype(np.float64)
        prm = oracle.make_params(interior.shape[1:], pch[5], 5.0 / 3.0, 0.8)
        oracle.step(prm, interior, dt, 0)
        got = ic.patch_view(out, pch)[:, ng:-ng, ng:-ng, ng:-ng]
        e = l1_fp32_errors(got.astype(np.float64), interior)
        assert max(e) <= 2e-6, (int(i), e)
        # ghosts untouched
        mask = np.ones(full_in.shape[1:], bool)
        mask[ng:-ng, ng:-ng, ng:-ng] = False
        np.testing.assert_array_equal(ic.patch_view(out, pch)[:, mask], full_in[:, mask])
    assert b.error() == hydro.HYDRO_OK
    b.close()


def test_fp32_trajectory_within_sensitivity_bound():
    """KH 64^3, 100 steps of fixed dt: the FP32 GPU run stays within 10 S_N +
    1e-5 of the FP64 oracle, where S_N is the L1 gap between two FP64 oracle
    runs started from the exact and from the FP32-rounded initial state (the
    flow's own sensitivity to a rounding-size perturbation)."""
    say("fp32 trajectory")
    P = ic.kh(64, seed=1)
    p = params_of(P, nthreads=THREADS)
    dt = 0.5 * oracle.cfl_dt(p, P.U)
    steps = 100
    exact = P.U.copy()
    rounded = P.U.astype(np.float32).astype(np.float64)
    pert = rounded.copy()
    for s in range(steps):
        oracle.step(p, exact, dt, s)
        oracle.step(p, pert, dt, s)
    S_N = l1_fp32_errors(pert, exact)
    g, dev = _grid(P, hydro.FP32, U=rounded.astype(np.float32))
    for _ in range(steps):
        g.step(dt)
    e = l1_fp32_errors(host(dev), exact)
    say(f"  S_N {S_N}  FP32 {e}")
    for a, s in zip(e, S_N):
        assert a <= 10 * s + 1e-5
    g.close()
