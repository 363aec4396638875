"""Batched patches: one persistent launch per sweep over a patch list must
give, patch by patch, the bits of the single-grid path, parity with the
oracle, the global dt as the minimum over patches, and untouched stored
ghost layers."""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import host, rel_err, say, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def _batch(count, prec, seed=3, ng=4, flags=hydro.FLAG_NO_TUNE):
    specs = ic.batch_specs(count, seed=seed)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = ic.batch_pool(specs, ng=ng, dtype=dt)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, GAMMA, flags=flags)
    return b, dev, pool, patches


def _single(pool, patch, prec):
    view = ic.patch_view(pool, patch).copy()
    dev = torch().from_numpy(view).to("cuda:0")
    d = patch[5]
    g = hydro.Grid(dev, (d, d, d), GAMMA, ng=patch[4], flags=hydro.FLAG_NO_TUNE)
    return g, dev


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_batch_equals_single_grids_bitwise(prec):
    say(f"batch vs single {prec}")
    b, dev, pool, patches = _batch(12, prec)
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
    b, dev, pool, patches = _batch(10, hydro.FP64)
    dt = b.cfl_dt()
    singles = []
    for p in patches:
        g, _ = _single(pool, p, hydro.FP64)
        singles.append(g.cfl_dt())
        g.close()
    assert dt == min(singles)
    b.close()


def test_batch_fp64_matches_oracle_and_keeps_ghosts():
    say("batch oracle")
    b, dev, pool, patches = _batch(8, hydro.FP64)
    dt = b.cfl_dt()
    b.step(dt)
    out = host(dev)
    for p in patches:
        o, n, _, _, ng = p[:5]
        full = ic.patch_view(pool, p)
        interior = np.ascontiguousarray(full[:, ng:-ng, ng:-ng, ng:-ng])
        prm = oracle.make_params(interior.shape[1:], p[5], GAMMA, 0.8)
        ref = interior.copy()
        oracle.step(prm, ref, dt, 0)
        got_full = ic.patch_view(out, p)
        err = rel_err(got_full[:, ng:-ng, ng:-ng, ng:-ng], ref)
        assert max(err) <= 1e-12, err
        mask = np.ones(full.shape[1:], bool)
        mask[ng:-ng, ng:-ng, ng:-ng] = False
        np.testing.assert_array_equal(got_full[:, mask], full[:, mask])
    b.close()


def test_batch_graph_equals_eager_and_totals():
    say("batch graph/totals")
    a, deva, pool, patches = _batch(9, hydro.FP32, seed=5)
    e, deve, _, _ = _batch(9, hydro.FP32, seed=5,
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
