"""The chunked x march (one pencil per wave, marched in chunks of 64 lane
runs, the last cell of each chunk finished by the next chunk) against the
FP64 oracle, and bit for bit against the lane-run x sweep.

Pencil lengths are picked so that the march takes several chunks with a
ragged last one (e.g. 200 cells at one cell per lane: chunks of 64, 64, 64
and 8 lanes) and also a single chunk, for every boundary kind, with gravity
along x on the reflecting case.
"""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import gpu_grid, host, params_of, rel_err, say
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

P_, O_, R_ = ic.PERIODIC, ic.OUTFLOW, ic.REFLECT

# (name, shape (nz, ny, nx), bc, grav)
CASES = [
    ("periodic", (6, 5, 200), (P_,) * 6, (0.0, 0.0, 0.0)),
    ("outflow", (5, 7, 136), (O_,) * 6, (0.0, 0.0, 0.0)),
    ("reflect_g", (4, 6, 264), (R_,) * 6, (0.3, -0.1, 0.05)),
]

MARCH = {hydro.FP64: ["x:v=1,b=64,m=1", "x:v=2,b=192,m=1"],
         hydro.FP32: ["x:v=1,b=128,m=1", "x:v=2,b=64,m=1", "x:v=4,b=256,m=1"]}


def lane_run(nx):
    """A lane-run x configuration valid for pencils of nx cells: one cell per
    lane, a workgroup of whole pencils."""
    return f"x:v=1,b={64 * (-(-nx // 64))}"


def _problem(shape, bc, grav, seed):
    return ic.smooth_random(shape, seed=seed, bc=bc, grav=grav)


@pytest.mark.parametrize("name,shape,bc,grav", CASES)
@pytest.mark.parametrize("cfg", MARCH[hydro.FP64])
def test_march_sweep_fp64_matches_oracle(name, shape, bc, grav, cfg):
    say(f"x march sweep fp64 {name} {shape} {cfg}")
    P = _problem(shape, bc, grav, seed=300)
    p = params_of(P)
    dt = 0.5 * oracle.cfl_dt(p, P.U)
    g, dev = gpu_grid(P, config=cfg)
    assert g.config.startswith(cfg)
    g.sweep(0, dt)
    ref = P.U.copy()
    oracle.sweep(p, ref, dt, 0)
    err = rel_err(host(dev), ref)
    assert max(err) <= 1e-12, err
    g.close()


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("name,shape,bc,grav", CASES)
def test_march_steps_equal_lane_run_bitwise(prec, name, shape, bc, grav):
    """Four CFL steps (the odd ones end with the x sweep, which folds the
    CFL maximum, so the held cells' speeds count too)."""
    P = _problem(shape, bc, grav, seed=301)

    def run(cfg):
        g, dev = gpu_grid(P, prec=prec, config=cfg)
        for _ in range(4):
            g.step()
        out, t, e = host(dev), g.time(), g.error()
        g.close()
        return out, t, e

    ref, tref, eref = run(lane_run(shape[2]))
    assert eref == hydro.HYDRO_OK
    for cfg in MARCH[prec]:
        say(f"x march steps {name} {shape} {cfg} prec {prec}")
        out, t, e = run(cfg)
        np.testing.assert_array_equal(out, ref)
        assert t == tref and e == eref


def test_march_flags_a_bad_held_cell():
    """A negative-pressure cell in the last position of the first chunk (the
    cell the next chunk finishes) sets the error flag.  Its neighbours stay
    healthy (the oracle agrees: with a NaN sound speed on one side the Davis
    bounds fall back to the other side's), so only the held cell's own check
    can raise it."""
    say("x march error flag on a held cell")
    P = ic.uniform((2, 3, 200), rho=1.0, p=1.0)
    U = P.U.copy()
    U[4, 1, 1, 63] = -0.5
    out = {}
    for cfg in ("x:v=1,b=64,m=1", lane_run(200)):
        g, dev = gpu_grid(P, config=cfg, U=U)
        g.sweep(0, 1e-6, fold_cfl=True)
        out[cfg] = (host(dev), g.error())
        g.close()
    a, b = out.values()
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1] == hydro.HYDRO_ENUMERIC
