"""Fused x and y sweeps of the batched path: each patch z-plane is held in
LDS while both sweeps run on it, one launch per step for the two.  Results
must be bit for bit those of the separate sweeps, in both Strang orders (x
then y on even steps, y then x on odd ones, where the fused launch is the
last of the step and folds the CFL maximum), for every plane configuration,
boundary kind and gravity; and match the oracle patch by patch."""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import host, rel_err, say, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0
P_, O_, R_ = ic.PERIODIC, ic.OUTFLOW, ic.REFLECT

UNFUSED = "x:v=4,b=512;y:q=64,s=4;z:q=64,s=4;p:g=512,d=1,f=0"


def fused(v, b):
    return f"x:v=4,b=512;y:q=64,s=4;z:q=64,s=4;p:g=512,d=1,f=1;w:v={v},b={b}"


def _pool(prec, count=10, seed=7):
    # a plane must fit in 80 KiB of LDS: FP32 up to 64^2, FP64 up to 32^2
    sizes = (16, 32, 48, 64) if prec == hydro.FP32 else (16, 32)
    specs = ic.batch_specs(count, seed=seed, sizes=sizes)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    return ic.batch_pool(specs, ng=4, dtype=dt, pad_rows=32)


def _run(pool, patches, cfg, dts, bc=(P_,) * 6, grav=(0.0, 0.0, 0.0)):
    dev = torch().from_numpy(pool.copy()).to("cuda:0")
    b = hydro.Batch(dev, patches, GAMMA, bc=bc, grav=grav, flags=hydro.FLAG_NO_TUNE)
    b.config = cfg
    got_cfg = b.config
    for dt in dts:
        b.step(dt)
    out, t, err = host(dev), b.time(), b.error()
    b.close()
    return out, t, err, got_cfg


# explicit dts for two steps of each parity, then two CFL steps (dt from the
# folded maximum of the previous step)
DTS = [1.1e-3, 0.9e-3, 1.0e-3, 0.8e-3, hydro.DT_CFL, hydro.DT_CFL]


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
@pytest.mark.parametrize("v,b", [(4, 512), (2, 256), (1, 512)])
def test_fused_equals_separate_sweeps_bitwise(prec, v, b):
    say(f"fused vs separate {prec} v={v} b={b}")
    pool, patches = _pool(prec)
    ref, tref, eref, _ = _run(pool, patches, UNFUSED, DTS)
    out, t, e, cfg = _run(pool, patches, fused(v, b), DTS)
    assert "f=1" in cfg and f"w:v={v},b={b}" in cfg, cfg
    np.testing.assert_array_equal(out, ref)
    assert t == tref and e == eref == hydro.HYDRO_OK


@pytest.mark.parametrize("bc,grav", [
    ((R_, R_, O_, O_, P_, P_), (0.3, -0.2, 0.05)),
    ((O_, O_, R_, R_, R_, R_), (0.0, 0.4, -0.1)),
])
def test_fused_boundaries_and_gravity_bitwise(bc, grav):
    say(f"fused bc {bc} grav {grav}")
    pool, patches = _pool(hydro.FP32, count=6, seed=8)
    ref, tref, _, _ = _run(pool, patches, UNFUSED, DTS, bc=bc, grav=grav)
    out, t, _, _ = _run(pool, patches, fused(4, 512), DTS, bc=bc, grav=grav)
    np.testing.assert_array_equal(out, ref)
    assert t == tref


def test_fused_fp64_matches_oracle():
    """Two steps (x-first, then y-first fused launches) at one oracle dt."""
    say("fused fp64 vs oracle")
    pool, patches = _pool(hydro.FP64, count=6, seed=9)
    interiors, params = [], []
    for p in patches:
        ng = p[4]
        interiors.append(np.ascontiguousarray(ic.patch_view(pool, p)[:, ng:-ng, ng:-ng, ng:-ng]))
        params.append(oracle.make_params(interiors[-1].shape[1:], p[5], GAMMA, 0.8))
    dt = min(oracle.cfl_dt(prm, u) for prm, u in zip(params, interiors))
    out, _, err, cfg = _run(pool, patches, fused(2, 512), [dt, dt])
    assert "f=1" in cfg and err == hydro.HYDRO_OK
    for p, u, prm in zip(patches, interiors, params):
        ng = p[4]
        ref = u.copy()
        oracle.step(prm, ref, dt, 0)
        oracle.step(prm, ref, dt, 1)
        e = rel_err(ic.patch_view(out, p)[:, ng:-ng, ng:-ng, ng:-ng], ref)
        assert max(e) <= 1e-12, e
        # ghost layers untouched
        mask = np.ones(ic.patch_view(pool, p).shape[1:], bool)
        mask[ng:-ng, ng:-ng, ng:-ng] = False
        np.testing.assert_array_equal(ic.patch_view(out, p)[:, mask],
                                      ic.patch_view(pool, p)[:, mask])


def test_fused_rejected_when_a_plane_does_not_fit():
    """48^2 FP64 planes need 90 KiB of LDS: the fused launch is refused."""
    specs = ic.batch_specs(4, seed=3, sizes=(48,))
    pool, patches = ic.batch_pool(specs, ng=4, dtype=np.float64, pad_rows=32)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, GAMMA, flags=hydro.FLAG_NO_TUNE)
    with pytest.raises(hydro.HydroError):
        b.config = fused(2, 512)
    assert "f=1" not in b.config
    b.close()
