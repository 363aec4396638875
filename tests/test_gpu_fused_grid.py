"""The fused x+y step of a single grid (HYDRO_FLAG_FUSE_XY) against the
separate sweeps, in FP32 (64 x 64 windows) and FP64 (64 x 32 windows).

The windows compute every written cell from the same stencil values with the
same lane-run arithmetic as the separate x and y sweeps, and the z march only
changes where it writes, so a fused step must give the same bits: checked
over several steps (both Strang orders; the CFL dt of each step folded by
each path) for every boundary kind on each axis, gravity along every axis,
ragged window counts, stored ghost layers and both window kernel shapes.
The folded totals follow the windows' partition: checked against the oracle
(as in the totals tests) and bitwise against the replay.  FP64 fused steps
also match the oracle's steps to 1e-12 of the grid's scale.
"""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import gpu_grid, grid_scale, host, params_of, rel_err, say, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

P_, O_, R_ = ic.PERIODIC, ic.OUTFLOW, ic.REFLECT
FUSE = hydro.FLAG_NO_TUNE | hydro.FLAG_FUSE_XY
FP32, FP64 = hydro.FP32, hydro.FP64

CASES = [
    ("periodic", (6, 64, 64), (P_,) * 6, (0.0, 0.0, 0.0), 0),
    ("periodic_ragged", (5, 70, 136), (P_,) * 6, (0.0, 0.0, 0.0), 0),
    ("outflow_x_reflect_y", (4, 130, 66), (O_, O_, R_, R_, P_, P_), (0.0, 0.0, 0.0), 0),
    ("reflect_x_outflow_y_g", (6, 66, 128), (R_, R_, O_, O_, R_, R_), (-0.3, 0.2, -0.1), 2),
    ("mixed_g_ghosts", (7, 124, 64), (P_, P_, R_, R_, O_, O_), (0.0, -0.4, 0.25), 2),
]
# y extents of 32 to 62 cells take FP64 windows (32 rows) but no FP32 ones
CASES64 = CASES + [
    ("fp64_short_y", (5, 40, 66), (P_, P_, O_, O_, R_, R_), (0.1, -0.2, 0.3), 0),
    ("fp64_short_y_periodic", (4, 34, 72), (P_,) * 6, (0.0, 0.0, 0.0), 2),
]
CFGS = {FP32: ["p:f=1;w:v=2,b=512", "p:f=1;w:v=1,b=256"],
        FP64: ["p:f=1;w:v=2,b=256", "p:f=1;w:v=1,b=512"]}


def _grid(P, ng, flags, prec, cfg=None):
    """Grid of P's state in `prec` with ng stored ghost layers of NaN (the
    sweeps never read them); returns the grid and the interior view of its
    state."""
    nz, ny, nx = P.shape
    dt = np.float32 if prec == FP32 else np.float64
    full = np.full((5, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng), np.nan, dtype=dt)
    full[:, ng:ng + nz, ng:ng + ny, ng:ng + nx] = P.U
    dev = torch().from_numpy(full).to("cuda:0")
    g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, ng=ng, flags=flags)
    if cfg:
        g.config = cfg
    return g, dev[:, ng:ng + nz, ng:ng + ny, ng:ng + nx]


def _pair(P, cfg, prec, ng=0):
    """The same state in a fused grid and in a grid of separate sweeps."""
    return _grid(P, ng, FUSE, prec, cfg), _grid(P, ng, hydro.FLAG_NO_TUNE, prec)


def _cases(prec):
    return [(prec, c) for c in (CASES if prec == FP32 else CASES64)]


@pytest.mark.parametrize("prec,case", _cases(FP32) + _cases(FP64))
@pytest.mark.parametrize("k", [0, 1])
def test_fused_step_equals_separate_sweeps_bitwise(prec, case, k):
    name, shape, bc, grav, ng = case
    cfg = CFGS[prec][k]
    P = ic.smooth_random(shape, seed=61, bc=bc, grav=grav)
    (g_f, d_f), (g_s, d_s) = _pair(P, cfg, prec, ng)
    assert "p:f=1" in g_f.config, g_f.config
    for step in range(4):
        say(f"fused {name} prec {prec} {cfg} step {step}")
        g_f.step()
        g_s.step()
        a, b = host(d_f), host(d_s)
        assert np.array_equal(a, b), (name, step, np.abs(a - b).max())
        assert g_f.time() == g_s.time(), (g_f.time(), g_s.time())
    assert g_f.error() == hydro.HYDRO_OK and g_s.error() == hydro.HYDRO_OK
    g_f.close()
    g_s.close()


@pytest.mark.parametrize("prec", [FP32, FP64])
@pytest.mark.parametrize("name,shape,bc,grav,ng", CASES[1:4])
def test_fused_step_totals(prec, name, shape, bc, grav, ng):
    P = ic.smooth_random(shape, seed=62, bc=bc, grav=grav)
    p = params_of(P)
    (g_f, d_f), (g_s, _) = _pair(P, CFGS[prec][0], prec, ng)
    vol = float(np.prod(P.dx))
    for step in range(3):
        say(f"fused totals {name} prec {prec} step {step}")
        g_f.step()
        g_s.step()
        folded = np.array(g_f.totals())
        state = host(d_f).astype(np.float64)
        want = oracle.totals(p, state)
        scale = [float(np.abs(state[v]).sum()) * vol for v in range(5)]
        scale.append(scale[4] + 10.0 * scale[0])
        for v in range(6):
            assert abs(folded[v] - want[v]) <= 1e-13 * scale[v], (name, step, v)
        # the separate path sums another partition: equal to rounding
        other = np.array(g_s.totals())
        assert np.all(np.abs(folded - other) <= 1e-13 * np.array(scale))
        g_f.state_changed()
        assert folded.tolist() == list(g_f.totals()), (name, step)
    g_f.close()
    g_s.close()


@pytest.mark.parametrize("name,shape,bc,grav,ng", [CASES[3], CASES64[-2]])
def test_fused_step_fp64_matches_oracle(name, shape, bc, grav, ng):
    """Three FP64 fused steps (both Strang orders, gravity, walls) against
    the oracle's steps at the oracle's CFL dt, to 1e-12 of the grid's scale."""
    P = ic.smooth_random(shape, seed=65, bc=bc, grav=grav)
    p = params_of(P)
    g, d = _grid(P, ng, FUSE, FP64, CFGS[FP64][0])
    U = P.U.astype(np.float64).copy()
    scale = grid_scale(U)
    for step in range(3):
        say(f"fused fp64 oracle {name} step {step}")
        dt = oracle.cfl_dt(p, U)
        oracle.step(p, U, dt, step)
        g.step(dt)
        err = rel_err(host(d), U, scale)
        assert max(err) <= 1e-12, (name, step, err)
    assert g.error() == hydro.HYDRO_OK
    g.close()


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_fused_step_graph_vs_eager_and_tuned(prec):
    P = ic.kh(shape=(16, 128, 128), seed=63)
    U = P.U.astype(np.float32).astype(np.float64) if prec == FP32 else P.U
    cfg = CFGS[prec][0]
    runs = []
    for flags, c in ((FUSE, cfg),
                     (FUSE | hydro.FLAG_NO_GRAPH, cfg),
                     (hydro.FLAG_FUSE_XY, None),            # tuned: fused or not
                     (hydro.FLAG_NO_TUNE, None)):
        g, d = gpu_grid(P, prec=prec, U=U, flags=flags, config=c)
        say(f"fused kh prec {prec} flags {flags} config {g.config}")
        for _ in range(5):
            g.step()
        runs.append(host(d))
        g.close()
    for r in runs[1:]:
        assert np.array_equal(runs[0], r)


def test_fused_step_config_errors_and_workspace():
    P = ic.smooth_random((4, 64, 64), seed=64)
    g, _ = gpu_grid(P, prec=FP32)          # no FUSE flag: no second buffer
    with pytest.raises(hydro.HydroError) as e:
        g.config = "p:f=1;w:v=2,b=512"
    assert e.value.status == hydro.HYDRO_EINVAL
    g.close()
    g, _ = gpu_grid(P, prec=FP32, flags=FUSE)
    for bad in ("p:f=1;w:v=4,b=512", "p:f=1;w:v=2,b=96"):
        with pytest.raises(hydro.HydroError) as e:
            g.config = bad
        assert e.value.status == hydro.HYDRO_EINVAL
    g.config = "p:f=1;w:v=2,b=256"
    assert "p:f=1;w:v=2,b=256" in g.config
    g.close()
    # a y extent below an FP32 window (64 rows) takes FP64 windows only
    Q = ic.smooth_random((4, 40, 64), seed=66)
    g, _ = gpu_grid(Q, prec=FP32, flags=FUSE)
    with pytest.raises(hydro.HydroError) as e:
        g.config = "p:f=1;w:v=2,b=512"
    assert e.value.status == hydro.HYDRO_EINVAL
    g.close()
    g, _ = gpu_grid(Q, prec=FP64, flags=FUSE)
    g.config = "p:f=1;w:v=2,b=256"
    assert "p:f=1;w:v=2,b=256" in g.config
    g.close()
    # the flag adds the state's size to the workspace where it applies
    for prec, word in ((FP32, 4), (FP64, 8)):
        d = hydro.make_desc((4, 64, 64), (1 / 64,) * 3, 1.4, precision=prec)
        d_f = hydro.make_desc((4, 64, 64), (1 / 64,) * 3, 1.4, precision=prec,
                              flags=hydro.FLAG_FUSE_XY)
        grow = hydro.hydro_workspace_bytes(d_f) - hydro.hydro_workspace_bytes(d)
        assert grow >= 5 * 64 * 64 * 4 * word, (prec, grow)
    d = hydro.make_desc((4, 30, 64), (1 / 64,) * 3, 1.4, precision=FP64)
    d_f = hydro.make_desc((4, 30, 64), (1 / 64,) * 3, 1.4, precision=FP64,
                          flags=hydro.FLAG_FUSE_XY)
    assert hydro.hydro_workspace_bytes(d_f) == hydro.hydro_workspace_bytes(d)  # y < 32
