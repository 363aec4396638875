"""Bitwise invariances of the GPU path: graph replay vs one-by-one launches,
every kernel configuration, repeated runs, checkpoint/resume, and an
autotuner that leaves the state untouched."""
import os

import numpy as np
import pytest

import hydro_ic as ic
from gpu_util import gpu_grid, host, say, to_device
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

CONFIGS = [
    "x:v=1,b=128;y:q=64,s=1;z:q=64,s=1",
    "x:v=2,b=256;y:q=64,s=2;z:q=128,s=2",
    "x:v=4,b=64;y:q=128,s=4;z:q=64,s=4",
    "x:v=4,b=512;y:q=64,s=8;z:q=256,s=2",
    "x:v=1,b=192,m=1;y:q=128,s=2;z:q=128,s=1",   # chunked x march: 72 = 64 + 8 lanes
    "x:v=2,b=64,m=1;y:q=64,s=1;z:q=64,s=1",
]


def _run(P, prec, steps, flags=hydro.FLAG_NO_TUNE, config=None):
    g, dev = gpu_grid(P, prec=prec, flags=flags, config=config)
    for _ in range(steps):
        g.step()
    out = host(dev)
    t = g.time()
    g.close()
    return out, t


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_graph_replay_equals_eager_launches(prec):
    say(f"graph vs eager {prec}")
    P = ic.kh(shape=(40, 64, 72), seed=21)
    a, ta = _run(P, prec, 6)
    b, tb = _run(P, prec, 6, flags=hydro.FLAG_NO_TUNE | hydro.FLAG_NO_GRAPH)
    np.testing.assert_array_equal(a, b)
    assert ta == tb


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_every_kernel_configuration_gives_the_same_bits(prec):
    P = ic.smooth_random((40, 64, 72), seed=22, bc=(0, 0, 1, 1, 2, 2),
                         grav=(0.0, 0.0, -0.1))
    ref = None
    for cfg in CONFIGS:
        say(f"config {cfg} prec {prec}")
        out, t = _run(P, prec, 4, config=cfg)
        if ref is None:
            ref, tref = out, t
        else:
            np.testing.assert_array_equal(out, ref)
            assert t == tref


def test_run_to_run_bitwise():
    say("run to run")
    P = ic.kh(shape=(32, 48, 64), seed=23)
    a, _ = _run(P, hydro.FP32, 5)
    b, _ = _run(P, hydro.FP32, 5)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_resume_from_checkpoint_is_bitwise(prec):
    say(f"resume {prec}")
    P = ic.rt(nx=32, ny=32, nz=64, seed=24)
    full, tfull = _run(P, prec, 6)
    g, dev = gpu_grid(P, prec=prec)
    for _ in range(3):
        g.step()
    t, s = g.time()
    ckpt = host(dev)
    g.close()
    h, dev2 = gpu_grid(P, prec=prec, U=ckpt)
    h.set_time(t, s)
    for _ in range(3):
        h.step()
    np.testing.assert_array_equal(host(dev2), full)
    assert h.time() == tfull
    h.close()


def test_autotuner_leaves_state_unchanged_and_caches(tmp_path):
    say("autotune")
    os.environ["HYDRO_TUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        P = ic.kh(shape=(48, 64, 80), seed=25)
        before = P.U.astype(np.float32)
        g, dev = gpu_grid(P, prec=hydro.FP32, flags=0)
        np.testing.assert_array_equal(host(dev), before.astype(np.float64))
        cfg = g.config
        assert (tmp_path / "tune.json").exists()
        g.close()
        h, _ = gpu_grid(P, prec=hydro.FP32, flags=0)
        assert h.config == cfg
        h.close()
    finally:
        del os.environ["HYDRO_TUNE_CACHE"]


def test_time_sweeps_leaves_state_unchanged():
    say("time sweeps")
    P = ic.kh(shape=(32, 48, 64), seed=26)
    g, dev = gpu_grid(P, prec=hydro.FP64)
    before = host(dev)
    ms = g.time_sweeps(3)
    assert all(m > 0 for m in ms)
    np.testing.assert_array_equal(host(dev), before)
    assert g.stream_ceiling(2) > 0
    np.testing.assert_array_equal(host(dev), before)
    # stepping afterwards matches a fresh grid
    g.step(1e-4)
    h, dev2 = gpu_grid(P, prec=hydro.FP64)
    h.step(1e-4)
    np.testing.assert_array_equal(host(dev), host(dev2))
    g.close()
    h.close()
