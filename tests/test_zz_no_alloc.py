"""hydro_step_noalloc against hydro_step: the allocation-free entry point runs
the step of a context made with HYDRO_FLAG_NO_TUNE from the same descriptor,
so the state, the dt taken, the next CFL dt and the folded FP64 totals must
match bit for bit.  Two calls in a row on two grids, the second smaller (the
static scratch keeps the first call's contents), in both precisions, with
an explicit dt and with the CFL dt; and a grid whose totals need more
partial sums than the scratch holds is refused."""
import ctypes

import numpy as np
import pytest

import hydro_ic as ic
from gpu_util import host, say, to_device, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu


def _reference(P, prec, dt, step):
    """The existing path: a context (built-in configuration), set to the step
    counter, one hydro_step; returns state, the dt taken, next dt, totals."""
    dev = to_device(P.U, prec)
    g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=hydro.FLAG_NO_TUNE)
    g.set_time(0.0, step)
    if dt == hydro.DT_CFL:
        dt = g.cfl_dt()
    g.step(dt)
    t, _ = g.time()
    tot = g.totals()
    nxt = g.cfl_dt()
    out = host(dev)
    g.close()
    return out, t, nxt, tot


def _noalloc(P, prec, dt, step):
    t = torch()
    dev = to_device(P.U, prec)
    desc = hydro.make_desc(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav, prec)
    res = t.full((9,), -1.0, dtype=t.float64, device="cuda:0")
    stream = t.cuda.current_stream()
    hydro.hydro_step_noalloc(desc, ctypes.c_void_p(dev.data_ptr()),
                             dev.numel() * dev.element_size(), dt, step,
                             ctypes.c_void_p(stream.cuda_stream),
                             ctypes.c_void_p(res.data_ptr()))
    t.cuda.synchronize()
    return host(dev), res.cpu().numpy()


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("dt", [2e-3, hydro.DT_CFL])
def test_noalloc_step_equals_hydro_step_twice(prec, dt):
    first = ic.smooth_random((24, 40, 72), seed=61, bc=(0, 0, 1, 1, 2, 2),
                             grav=(0.0, 0.0, -0.2))
    second = ic.kh(shape=(12, 20, 36), seed=62)          # smaller, other data
    for P, step in ((first, 0), (second, 1)):
        say(f"noalloc prec {prec} dt {dt} shape {P.shape} step {step}")
        want, t_ref, next_ref, tot_ref = _reference(P, prec, dt, step)
        got, res = _noalloc(P, prec, dt, step)
        np.testing.assert_array_equal(got, want)
        assert res[0] == t_ref                          # the dt taken
        assert res[1] == next_ref                       # the CFL dt of the new state
        assert list(res[2:8]) == list(tot_ref)          # the folded totals
        assert res[8] == 0.0                            # no error bits


def test_noalloc_refuses_grid_beyond_scratch():
    t = torch()
    # 1 x 1536 x 1024 (one z layer, so z is skipped, y sweep last on even
    # steps: 1536 x 1 columns / 64 = 24 partial sums, fine); a 4 x 1536 x 1024
    # grid's z sweep needs 1536 * 1024 / 64 = 24576 > the scratch's partials
    desc = hydro.make_desc((4, 1536, 1024), 1e-3, 1.4, precision=hydro.FP32)
    dev = t.ones((5, 4, 1536, 1024), dtype=t.float32, device="cuda:0")
    with pytest.raises(hydro.HydroError) as e:
        hydro.hydro_step_noalloc(desc, ctypes.c_void_p(dev.data_ptr()),
                                 dev.numel() * 4, 1e-4, 0,
                                 ctypes.c_void_p(t.cuda.current_stream().cuda_stream))
    assert e.value.status == hydro.HYDRO_EINVAL
    assert "static scratch" in str(e.value)
    np.testing.assert_array_equal(dev.cpu().numpy(), 1.0)   # nothing ran
