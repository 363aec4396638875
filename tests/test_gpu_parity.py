"""GPU parity of libhydro against the FP64 CPU oracle, through the C ABI.

FP64: every sweep and every step matches the oracle to 1e-12 relative
(max |gpu - oracle| / max |oracle| per conserved variable) from the same
input state; dt to 1e-14.  Shapes span several workgroup tiles and ragged
tails (x widths not a multiple of 64, column lengths not a multiple of the
segment length).  FP32: relative L1 error of each conserved quantity within
2e-6 of the FP64 oracle after one step from an FP32-representable state,
about 34 units of FP32 round-off (one rounding of the stored state plus three
sweeps of flux differences), and a per-cell (max-norm) error within 1e-5 of
the variable's largest magnitude: each cell's update is a Lipschitz function
(limiter and Riemann solver are continuous) of about 20 inputs that carry
FP32 rounding, so a single cell may collect a few times the L1 average, and
1e-5 (about 170 units of round-off) leaves that margin while a wrong
boundary row or gravity sign, at O(dt g) or O(1) relative, still fails it.
"""
import math

import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import (gpu_grid, host, l1_err, l1_fp32_errors, max_fp32_errors, params_of,
                      rel_err, say, to_device)
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

P_, O_, R_ = ic.PERIODIC, ic.OUTFLOW, ic.REFLECT

# (name, shape (nz, ny, nx), bc, grav)
CASES = [
    ("periodic", (20, 70, 36), (P_,) * 6, (0.0, 0.0, 0.0)),
    ("outflow", (18, 33, 44), (O_,) * 6, (0.0, 0.0, 0.0)),
    ("reflect_g", (66, 12, 20), (R_,) * 6, (0.05, -0.1, 0.2)),
    ("mixed_g", (40, 18, 130), (P_, P_, O_, O_, R_, R_), (0.0, 0.0, -0.3)),
]


def _problem(shape, bc, grav, seed):
    return ic.smooth_random(shape, seed=seed, bc=bc, grav=grav)


@pytest.mark.parametrize("name,shape,bc,grav", CASES)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_single_sweep_fp64(name, shape, bc, grav, axis):
    say(f"sweep fp64 {name} {shape} axis {axis}")
    P = _problem(shape, bc, grav, seed=100 + axis)
    p = params_of(P)
    dt = 0.5 * oracle.cfl_dt(p, P.U)
    g, dev = gpu_grid(P)
    g.sweep(axis, dt)
    ref = P.U.copy()
    oracle.sweep(p, ref, dt, axis)
    err = rel_err(host(dev), ref)
    assert max(err) <= 1e-12, err
    g.close()


@pytest.mark.parametrize("name,shape,bc,grav", CASES)
def test_steps_fp64_from_identical_states(name, shape, bc, grav):
    say(f"steps fp64 {name} {shape}")
    P = _problem(shape, bc, grav, seed=7)
    p = params_of(P)
    g, dev = gpu_grid(P)
    state = P.U.copy()
    for step in range(4):
        dt = oracle.cfl_dt(p, state)
        dev.copy_(to_device(state, hydro.FP64))
        g.state_changed()
        g.set_time(0.0, step)
        g.step(dt)
        ref = state.copy()
        oracle.step(p, ref, dt, step)
        err = rel_err(host(dev), ref)
        assert max(err) <= 1e-12, (step, err)
        state = ref
    assert g.error() == hydro.HYDRO_OK
    g.close()


@pytest.mark.parametrize("name,shape,bc,grav", CASES)
def test_cfl_dt_fp64(name, shape, bc, grav):
    say(f"cfl fp64 {name}")
    P = _problem(shape, bc, grav, seed=3)
    g, dev = gpu_grid(P)
    dt_gpu = g.cfl_dt()
    dt_ref = oracle.cfl_dt(params_of(P), P.U)
    assert abs(dt_gpu - dt_ref) <= 1e-14 * dt_ref
    g.close()


def test_folded_dt_equals_standalone_reduction():
    say("folded dt")
    P = _problem((16, 20, 24), (P_,) * 6, (0, 0, 0), seed=4)
    g, dev = gpu_grid(P)
    g.step(1e-3)                   # the last sweep folds the CFL of the new state
    t0, _ = g.time()
    g.step()                       # advances by the folded dt
    t1, _ = g.time()
    folded = t1 - t0
    # recompute: redo the first step on a fresh grid and reduce its state
    h, dev2 = gpu_grid(P)
    h.step(1e-3)
    fresh = h.cfl_dt()
    assert abs(folded - fresh) <= 1e-15 * fresh
    g.close()
    h.close()


def test_totals_fp64():
    say("totals fp64")
    P = _problem((17, 23, 29), (P_, P_, P_, P_, R_, R_), (0.0, 0.0, -0.2), seed=5)
    g, dev = gpu_grid(P)
    got = np.array(g.totals())
    want = oracle.totals(params_of(P), P.U)
    vol = np.prod(P.dx)
    for v in range(6):
        src = P.U[min(v, 4)]
        scale = np.abs(src).sum() * vol
        assert abs(got[v] - want[v]) <= 1e-14 * scale, (v, got, want)
    # deterministic: bitwise equal on repeat
    assert list(got) == g.totals()
    g.close()


def test_uniform_state_unchanged_bitwise():
    for prec in (hydro.FP32, hydro.FP64):
        for bc in (P_, O_, R_):
            say(f"uniform prec {prec} bc {bc}")
            P = ic.uniform((9, 70, 68), bc=(bc,) * 6)
            g, dev = gpu_grid(P, prec=prec)
            before = host(dev)
            for _ in range(4):
                g.step(1e-3)
            np.testing.assert_array_equal(host(dev), before)
            g.close()
    P = ic.uniform((9, 70, 68), v=(0.3, -0.7, 1.9))
    g, dev = gpu_grid(P)
    before = host(dev)
    for _ in range(4):
        g.step(1e-3)
    np.testing.assert_array_equal(host(dev), before)
    g.close()


def test_stationary_contact_bitwise():
    say("stationary contact")
    P = ic.stationary_contact(256)
    g, dev = gpu_grid(P)
    before = host(dev)
    for _ in range(20):
        g.step()
    np.testing.assert_array_equal(host(dev), before)
    g.close()


def _gpu_sod(n=1024, axis=0, transverse=1, prec=hydro.FP64):
    P = ic.sod(n, axis=axis, transverse=transverse)
    g, dev = gpu_grid(P, prec=prec)
    g.set_t_end(P.t_end)
    steps = 0
    while True:
        t, s = g.time()
        if t >= P.t_end:
            break
        for _ in range(64):
            g.step()
        steps += 64
        assert steps < 5000
    t, s = g.time()
    out = host(dev)
    g.close()
    return P, out, t


def test_sod_fp64_matches_oracle_run_and_exact_solution():
    say("sod fp64")
    P, out, t = _gpu_sod()
    assert t == pytest.approx(0.2, abs=1e-15)
    ref = P.U.copy()
    tt, steps, _ = oracle.run(params_of(P), ref, 10 ** 6, t_end=0.2)
    err = rel_err(out, ref)
    assert max(err) <= 1e-10, err
    dx = 1.0 / 1024
    assert abs(out[0].sum() * dx - 0.5625) <= 1e-14
    assert abs(out[4].sum() * dx - 1.375) <= 1e-14
    from oracle.exact_riemann import ExactRiemann, RiemannState
    e = ExactRiemann(RiemannState(1, 0, 1), RiemannState(0.125, 0, 0.1), 1.4)
    avg = e.cell_averages(np.linspace(0, 1, 1025), 0.2, 0.5)
    assert np.abs(out[0, 0, 0] - avg[:, 0]).mean() < 1e-3


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sod_embedded_in_3d_is_bitwise(axis):
    say(f"sod embedded axis {axis}")
    n = 512
    P1, out1, t1 = _gpu_sod(n)
    P3, out3, t3 = _gpu_sod(n, axis=axis, transverse=4)
    assert t1 == t3
    line = [slice(None)] * 4
    for a in range(3):
        line[3 - a] = slice(None) if a == axis else 1
    got = out3[tuple(line)]
    np.testing.assert_array_equal(got[0], out1[0, 0, 0])
    np.testing.assert_array_equal(got[1 + axis], out1[1, 0, 0])
    np.testing.assert_array_equal(got[4], out1[4, 0, 0])


def test_fp32_one_step_l1_bound():
    say("fp32 one step")
    P = ic.kh(shape=(40, 64, 72), seed=9)
    U32 = P.U.astype(np.float32).astype(np.float64)   # FP32-representable input
    p = params_of(P)
    for step in (0, 1):
        dt = oracle.cfl_dt(p, U32)
        g, dev = gpu_grid(P, prec=hydro.FP32, U=U32)
        g.set_time(0.0, step)
        g.step(dt)
        ref = U32.copy()
        oracle.step(p, ref, dt, step)
        got = host(dev)
        e = l1_fp32_errors(got, ref)
        mx = max_fp32_errors(got, ref)
        say(f"  step {step} L1 (rho, m, E) {e} per-variable {l1_err(got, ref)} max {mx}")
        # 2e-6 is about 34 units of FP32 round-off (2^-24): one rounding of
        # the stored state plus three sweeps of flux differences, each a
        # chain of ~20 rounded operations scaled by dt/dx |F| <~ |U|
        assert max(e) <= 2e-6, e
        assert max(mx) <= 1e-5, mx
        g.close()


@pytest.mark.parametrize("name,shape,bc,grav", CASES)
def test_fp32_one_step_every_boundary_and_gravity(name, shape, bc, grav):
    # reflecting walls, outflow ends and gravity in FP32 against the FP64
    # oracle, both Strang orders, the L1 and the per-cell bounds above
    P = _problem(shape, bc, grav, seed=31)
    U32 = P.U.astype(np.float32).astype(np.float64)
    p = params_of(P)
    for step in (0, 1):
        say(f"fp32 step {name} {shape} parity {step}")
        dt = oracle.cfl_dt(p, U32)
        g, dev = gpu_grid(P, prec=hydro.FP32, U=U32)
        g.set_time(0.0, step)
        g.step(dt)
        ref = U32.copy()
        oracle.step(p, ref, dt, step)
        got = host(dev)
        e = l1_fp32_errors(got, ref)
        mx = max_fp32_errors(got, ref)
        say(f"  L1 (rho, m, E) {e} max {mx}")
        assert max(e) <= 2e-6, e
        assert max(mx) <= 1e-5, mx
        g.close()


# x pencils longer than 64 lanes of 4 cells: lane runs spread over several
# waves of a workgroup that trade edge values through LDS
WIDE = [
    ("periodic", (4, 5, 768), (P_,) * 6, (0.0, 0.0, 0.0),
     ["x:v=4,b=192", "x:v=4,b=384", "x:v=1,b=64,m=1"]),
    ("outflow", (3, 6, 384), (O_, O_, P_, P_, P_, P_), (0.0, 0.0, 0.0),
     ["x:v=4,b=128", "x:v=4,b=256", "x:v=4,b=512", "x:v=2,b=64,m=1"]),
    ("reflect_g", (5, 4, 520), (R_, R_, P_, P_, O_, O_), (-0.2, 0.0, 0.1),
     ["x:v=4,b=192", "x:v=4,b=384", "x:v=2,b=128,m=1"]),
]


@pytest.mark.parametrize("name,shape,bc,grav,configs", WIDE)
def test_multiwave_x_lane_runs_fp64(name, shape, bc, grav, configs):
    P = _problem(shape, bc, grav, seed=41)
    p = params_of(P)
    dt = oracle.cfl_dt(p, P.U)
    ref_sweep = P.U.copy()
    oracle.sweep(p, ref_sweep, dt, 0)
    ref_steps = P.U.copy()
    for s in range(2):
        oracle.step(p, ref_steps, dt, s)
    first = None
    for cfg in configs:
        say(f"wide x fp64 {name} {shape} {cfg}")
        g, dev = gpu_grid(P, config=cfg)
        assert g.config.startswith(cfg)
        g.sweep(0, dt)
        err = rel_err(host(dev), ref_sweep)
        assert max(err) <= 1e-12, (cfg, err)
        g.close()
        g, dev = gpu_grid(P, config=cfg)
        g.step(dt)
        g.step(dt)
        out = host(dev)
        err = rel_err(out, ref_steps)
        assert max(err) <= 1e-12, (cfg, err)
        if first is None:
            first = out
        else:
            np.testing.assert_array_equal(out, first)   # every configuration: same bits
        g.close()


def test_error_flag_on_negative_pressure():
    say("error flag")
    P = ic.uniform((8, 8, 64))
    U = P.U.copy()
    U[4, 3, 4, 10] = -1.0
    g, dev = gpu_grid(P, U=U)
    with pytest.raises(hydro.HydroError) as e:
        g.cfl_dt()
    assert e.value.status == hydro.HYDRO_ENUMERIC
    g.clear_error()
    g.step(1e-4)
    assert g.error() == hydro.HYDRO_ENUMERIC
    g.close()


def test_invalid_arguments_raise():
    t = __import__("torch")
    U = t.zeros((5, 4, 4, 4), dtype=t.float64, device="cuda:0")
    with pytest.raises(hydro.HydroError):
        hydro.Grid(U, 0.25, 1.4, cfl=2.0)
    g = hydro.Grid(U + 1.0, 0.25, 1.4, flags=hydro.FLAG_NO_TUNE)
    with pytest.raises(hydro.HydroError):
        g.step(-1.0)
    with pytest.raises(hydro.HydroError):
        g.config = "x:v=3,b=256"
    g.close()
