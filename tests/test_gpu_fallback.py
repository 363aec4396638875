"""GPU parity where the positivity fallback acts: cells whose Hancock face
state has rho <= 0 or p <= 0 are reconstructed with zero slopes.

The supersonic staircases put one such cell in every pencil along the swept
axis (the oracle pins show the sweep is then the first-order upwind scheme);
the two strong rarefactions reach the fallback over a run.  FP64 matches the
oracle to 1e-12 per sweep and per run; FP32, from the same FP32-representable
state, stays within the one-step L1 bound (2e-6) and a per-cell bound.  The
fallback decision itself is taken in each path's own precision; the face
values that trigger it here are -3.5 against a cell value of 10, so both
precisions take the same branch.
"""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import gpu_grid, host, l1_fp32_errors, max_fp32_errors, params_of, rel_err, say
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

KINDS = ["rho_left", "rho_right", "p_left", "p_right"]

# kernel shapes of the swept axis: lane runs (packed and multi-wave), the
# chunked x march, and column marches with one and several segments
X_CONFIGS = {72: ["x:v=1,b=128", "x:v=4,b=64", "x:v=2,b=64,m=1"],
             296: ["x:v=4,b=128", "x:v=1,b=320", "x:v=1,b=128,m=1"]}
COL_CONFIGS = ["y:q=64,s=1;z:q=64,s=1", "y:q=64,s=4;z:q=128,s=3"]


def _staircase(kind, axis, n, grav):
    # a 5 x 5 cross-section (periodic) repeats the pencil, so a packed x wave
    # and a column-march tile hold several copies of it
    return ic.steep_supersonic(kind, n=n, k=n // 2 - 3, axis=axis, transverse=5, grav=grav)


def _configs(axis, n):
    return X_CONFIGS[n] if axis == 0 else COL_CONFIGS


@pytest.mark.parametrize("n", [72, 296])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("kind", KINDS)
def test_fallback_sweep_fp64(kind, axis, n):
    grav = -40.0 if kind.startswith("p") else 0.0
    P = _staircase(kind, axis, n, grav)
    p = params_of(P)
    dt = 0.5 * P.dx[axis] / 20.0
    ref = P.U.copy()
    assert oracle.sweep(p, ref, dt, axis) == int(np.prod(P.shape)) // n
    for cfg in _configs(axis, n):
        say(f"fallback fp64 {kind} axis {axis} n {n} {cfg}")
        g, dev = gpu_grid(P, config=cfg)
        g.sweep(axis, dt)
        err = rel_err(host(dev), ref)
        assert max(err) <= 1e-12, (cfg, err)
        g.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("kind", KINDS)
def test_fallback_sweep_fp32(kind, axis):
    n = 72
    P = _staircase(kind, axis, n, -40.0 if kind.endswith("right") else 0.0)
    U32 = P.U.astype(np.float32).astype(np.float64)
    p = params_of(P)
    dt = 0.5 * P.dx[axis] / 20.0
    ref = U32.copy()
    oracle.sweep(p, ref, dt, axis)
    for cfg in _configs(axis, n):
        say(f"fallback fp32 {kind} axis {axis} {cfg}")
        g, dev = gpu_grid(P, prec=hydro.FP32, U=U32, config=cfg)
        g.sweep(axis, dt)
        got = host(dev)
        e = l1_fp32_errors(got, ref)
        mx = max_fp32_errors(got, ref)
        say(f"  L1 {e} max {mx}")
        assert max(e) <= 2e-6, (cfg, e)
        assert max(mx) <= 1e-5, (cfg, mx)
        g.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_two_rarefactions_run_fp64(axis):
    # the whole run to t = 0.02 with the CFL dt, fallbacks included (the
    # oracle reports them), embedded along each axis of a 3D grid
    P = ic.two_rarefactions(128, axis=axis, transverse=4)
    ref = P.U.copy()
    t, steps, fb = oracle.run(params_of(P), ref, 10 ** 6, t_end=P.t_end)
    assert fb > 0
    say(f"two rarefactions axis {axis}: {steps} steps, {fb} fallbacks")
    g, dev = gpu_grid(P)
    g.set_t_end(P.t_end)
    for _ in range(steps):
        g.step()
    tg, sg = g.time()
    assert tg == pytest.approx(P.t_end, abs=1e-15) and sg == steps
    err = rel_err(host(dev), ref)
    assert max(err) <= 1e-10, err
    assert g.error() == hydro.HYDRO_OK
    g.close()
