"""Batched patches: one persistent launch per sweep over a patch list must
give, patch by patch, the bits of the single-grid path, parity with the
oracle, the global dt as the minimum over patches, and untouched stored
ghost layers; with a dt per patch (HYDRO_BATCH_PER_PATCH_DT) every patch
takes the steps and reaches the times of its own single-grid run."""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import host, rel_err, say, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def _batch(count, prec, seed=3, ng=4, flags=hydro.FLAG_NO_TUNE, pad_rows=0):
    specs = ic.batch_specs(count, seed=seed)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = ic.batch_pool(specs, ng=ng, dtype=dt, pad_rows=pad_rows)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, GAMMA, flags=flags)
    return b, dev, pool, patches


def _single(pool, patch, prec):
    view = np.array(ic.patch_view(pool, patch), order="C")  # a writable copy
    dev = torch().from_numpy(view).to("cuda:0")
    d = patch[5]
    g = hydro.Grid(dev, (d, d, d), GAMMA, ng=patch[4], flags=hydro.FLAG_NO_TUNE)
    return g, dev


@pytest.mark.parametrize("pad_rows", [0, 32])
@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_batch_equals_single_grids_bitwise(prec, pad_rows):
    say(f"batch vs single {prec} pad {pad_rows}")
    b, dev, pool, patches = _batch(12, prec, pad_rows=pad_rows)
    dts = [1.3e-3, 1.1e-3, 0.9e-3]
    for dt in dts:
        b.step(dt)
    out = host(dev)
    for i, p in enumerate(patches):
        g, sd = _single(pool, p, prec)
        for dt in dts:
            g.step(dt)
        np.testing.assert_array_equal(ic.patch_view(out, p), host(sd))
        g.close()
    b.close()


def test_batch_dt_is_min_over_patches():
    say("batch dt")
    b, dev, pool, patches = _batch(10, hydro.FP64, pad_rows=32)
    dt = b.cfl_dt()
    singles = []
    for p in patches:
        g, _ = _single(pool, p, hydro.FP64)
        singles.append(g.cfl_dt())
        g.close()
    assert dt == min(singles)
    b.close()


@pytest.mark.parametrize("pad_rows", [0, 32])
def test_batch_fp64_matches_oracle_and_keeps_ghosts(pad_rows):
    say(f"batch oracle pad {pad_rows}")
    b, dev, pool, patches = _batch(8, hydro.FP64, pad_rows=pad_rows)
    # one global dt: the smallest oracle CFL dt over the patches
    interiors, params = [], []
    for p in patches:
        ng = p[4]
        interiors.append(np.ascontiguousarray(ic.patch_view(pool, p)[:, ng:-ng, ng:-ng, ng:-ng]))
        params.append(oracle.make_params(interiors[-1].shape[1:], p[5], GAMMA, 0.8))
    dt = min(oracle.cfl_dt(prm, u) for prm, u in zip(params, interiors))
    assert abs(b.cfl_dt() - dt) <= 1e-14 * dt
    b.step(dt)
    out = host(dev)
    for p, interior, prm in zip(patches, interiors, params):
        ng = p[4]
        full = ic.patch_view(pool, p)
        ref = interior.copy()
        oracle.step(prm, ref, dt, 0)
        got_full = ic.patch_view(out, p)
        err = rel_err(got_full[:, ng:-ng, ng:-ng, ng:-ng], ref)
        assert max(err) <= 1e-12, err
        mask = np.ones(full.shape[1:], bool)
        mask[ng:-ng, ng:-ng, ng:-ng] = False
        np.testing.assert_array_equal(got_full[:, mask], full[:, mask])
    # padding outside every patch block is untouched too
    touched = np.zeros(pool.size, bool)
    for p in patches:
        o = p[0]
        touched[o:o + 5 * (p[10] if len(p) > 10 and p[10] else (p[1] + 2 * p[4]) ** 3)] = True
    np.testing.assert_array_equal(out[~touched], pool[~touched])
    b.close()


def test_batch_graph_equals_eager_and_totals():
    say("batch graph/totals")
    a, deva, pool, patches = _batch(9, hydro.FP32, seed=5, pad_rows=32)
    e, deve, _, _ = _batch(9, hydro.FP32, seed=5, pad_rows=32,
                          flags=hydro.FLAG_NO_TUNE | hydro.FLAG_NO_GRAPH)
    for _ in range(3):
        a.step()
        e.step()
    np.testing.assert_array_equal(host(deva), host(deve))
    tot = np.array(a.totals())
    out = host(deva)
    want = np.zeros(6)
    for p in patches:
        ng = p[4]
        v = ic.patch_view(out, p)[:, ng:-ng, ng:-ng, ng:-ng]
        vol = p[5] ** 3
        want[:5] += v.reshape(5, -1).sum(axis=1) * vol
    want[5] = want[4]
    np.testing.assert_allclose(tot, want, rtol=1e-12, atol=1e-12)
    a.close()
    e.close()


def test_cached_autotune_config_runs_the_whole_batch(tmp_path):
    """A second context on the same batch shape takes its kernel
    configuration from the autotune cache; its steps must still cover every
    patch (same bits as a context with the built-in configuration)."""
    import os
    say("batch cached config")
    os.environ["HYDRO_TUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        outs = []
        for flags in (0, 0, hydro.FLAG_NO_TUNE):
            b, dev, pool, patches = _batch(40, hydro.FP32, seed=7, pad_rows=32, flags=flags)
            for _ in range(2):
                b.step(1e-3)
            outs.append((host(dev), b.config))
            b.close()
        assert (tmp_path / "tune.json").exists()
        assert outs[0][1] == outs[1][1]
        np.testing.assert_array_equal(outs[0][0], outs[2][0])
        np.testing.assert_array_equal(outs[1][0], outs[2][0])
    finally:
        del os.environ["HYDRO_TUNE_CACHE"]


def _mixed_speed_batch(count, prec, flags):
    """A batch whose patches differ in signal speed (shear and density
    ratio from the seeded specs): with a dt per patch each takes its own."""
    return _batch(count, prec, seed=11, pad_rows=32, flags=flags)


@pytest.mark.parametrize("prec,cfg", [(hydro.FP64, ""), (hydro.FP32, ""),
                                      (hydro.FP32, "p:f=1;w:v=4,b=256")])
def test_per_patch_dt_equals_single_grids_bitwise(prec, cfg):
    say(f"per-patch dt {prec} {cfg}")
    b, dev, pool, patches = _mixed_speed_batch(
        10, prec, hydro.FLAG_NO_TUNE | hydro.BATCH_PER_PATCH_DT)
    if cfg:
        b.config = cfg
    steps = 5
    dt_min = b.cfl_dt()
    for _ in range(steps):
        b.step()
    out = host(dev)
    tb, dtb = b.times()
    assert b.time()[0] == min(tb)
    for i, p in enumerate(patches):
        g, sd = _single(pool, p, prec)
        for _ in range(steps):
            g.step()
        np.testing.assert_array_equal(ic.patch_view(out, p), host(sd))
        t, s = g.time()
        assert tb[i] == t and s == steps
        assert dtb[i] == g.cfl_dt()          # the next dt of the patch
        g.close()
    assert len(set(tb)) == len(tb)           # every patch at its own time
    assert min(dtb) >= 0 and dt_min > 0
    assert b.error() == hydro.HYDRO_OK
    b.close()


def test_per_patch_dt_fp64_matches_oracle_runs():
    say("per-patch dt vs oracle")
    b, dev, pool, patches = _mixed_speed_batch(
        6, hydro.FP64, hydro.FLAG_NO_TUNE | hydro.BATCH_PER_PATCH_DT)
    steps = 3
    for _ in range(steps):
        b.step()
    out = host(dev)
    tb, _ = b.times()
    for i, p in enumerate(patches):
        ng = p[4]
        u = np.ascontiguousarray(ic.patch_view(pool, p)[:, ng:-ng, ng:-ng, ng:-ng])
        prm = oracle.make_params(u.shape[1:], p[5], GAMMA, 0.8)
        t, s, _ = oracle.run(prm, u, steps)
        got = ic.patch_view(out, p)[:, ng:-ng, ng:-ng, ng:-ng]
        err = rel_err(got, u)
        assert max(err) <= 1e-12, (i, err)
        assert abs(tb[i] - t) <= 1e-14 * t
    b.close()


def test_per_patch_dt_lands_every_patch_on_t_end():
    say("per-patch dt t_end")
    b, dev, pool, patches = _mixed_speed_batch(
        8, hydro.FP64, hydro.FLAG_NO_TUNE | hydro.BATCH_PER_PATCH_DT)
    t_end = 3.5 * b.cfl_dt()     # about four steps for the patch with the smallest dt
    b.set_t_end(t_end)
    steps = 0
    while b.time()[0] < t_end:
        b.step()
        steps += 1
        assert steps <= 50
    tb, dtb = b.times()
    assert all(t == t_end for t in tb) and all(d == 0.0 for d in dtb)
    out = host(dev)
    for p in patches[:3]:
        g, sd = _single(pool, p, hydro.FP64)
        g.set_t_end(t_end)
        for _ in range(steps):
            g.step()
        np.testing.assert_array_equal(ic.patch_view(out, p), host(sd))
        g.close()
    b.close()


# --------------------------------------------------- z sweep over x-z planes

ZP_CASES = [
    ((ic.PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((ic.PERIODIC, ic.PERIODIC, ic.OUTFLOW, ic.OUTFLOW, ic.REFLECT, ic.REFLECT), (0.0, 0.0, -0.7)),
    ((ic.OUTFLOW,) * 4 + (ic.OUTFLOW, ic.REFLECT), (0.2, 0.0, 0.4)),
]


@pytest.mark.parametrize("v,block", [(1, 256), (2, 512), (4, 256)])
@pytest.mark.parametrize("bc,grav", ZP_CASES)
@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_zplane_z_sweep_equals_column_march_bitwise(prec, bc, grav, v, block):
    # the z sweep as lane runs over x-z planes in LDS gives the bits of the
    # z march, for every boundary kind at the z ends and gravity along z,
    # over both Strang orders with the CFL dt; FP64 patches up to 32 cells
    # along z fit the LDS share
    say(f"zplane prec {prec} bc {bc} grav {grav} v {v} b {block}")
    sizes = (16, 32) if prec == hydro.FP64 else (16, 32, 48, 64)
    specs = ic.batch_specs(10, seed=8, sizes=sizes)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = ic.batch_pool(specs, ng=4, dtype=dt, pad_rows=32)
    runs = []
    for cfg in (f"p:z=1;u:v={v},b={block}", "p:z=0"):
        dev = torch().from_numpy(pool.copy()).to("cuda:0")
        b = hydro.Batch(dev, patches, GAMMA, 0.8, bc, grav, flags=hydro.FLAG_NO_TUNE)
        b.config = cfg
        assert ("z=1" in b.config) == cfg.startswith("p:z=1"), b.config
        for _ in range(4):
            b.step()
        assert b.error() == hydro.HYDRO_OK
        runs.append((host(dev), b.time(), b.totals()))
        b.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
    scale = np.abs(runs[1][2]).max() + 1.0
    assert np.all(np.abs(np.array(runs[0][2]) - np.array(runs[1][2])) <= 1e-13 * scale)


def test_zplane_rejected_where_a_plane_does_not_fit():
    # FP64 x-z planes of 48 or 64 cells along z exceed a workgroup's LDS share
    specs = ic.batch_specs(6, seed=9, sizes=(48, 64))
    pool, patches = ic.batch_pool(specs, ng=4, dtype=np.float64, pad_rows=32)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, GAMMA, flags=hydro.FLAG_NO_TUNE)
    with pytest.raises(hydro.HydroError) as e:
        b.config = "p:z=1;u:v=2,b=512"
    assert e.value.status == hydro.HYDRO_EINVAL
    b.close()
