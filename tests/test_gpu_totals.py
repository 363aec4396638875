"""FP64 conserved totals folded into the last sweep of every step.

After each step the totals of the new state (rho, mx, my, mz, E and
E + rho phi, times the cell volume) are already on the device: the last
sweep sums them per workgroup or work item and the step's final kernel adds
the partials in a fixed order.  Checked here:
  * against the oracle's compensated sum of the same (GPU) state, within
    1e-14 of the sum of |q| (FP64 summation of ~1e5..1e6 terms in a fixed
    tree: a relative error of a few 1e-16 of that sum);
  * bitwise against hydro_totals on the same state after the library is
    told the state changed (it then replays the last sweep with dt = 0 and
    no stores, the same partition of the sums);
  * bitwise run to run, for every boundary kind, gravity, both Strang
    orders, both precisions, a one-dimensional grid, and batches (separate
    and fused plane sweeps).
"""
import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import gpu_grid, host, params_of, say, torch
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

P_, O_, R_ = ic.PERIODIC, ic.OUTFLOW, ic.REFLECT

CASES = [
    ("periodic", (20, 70, 36), (P_,) * 6, (0.0, 0.0, 0.0)),
    ("outflow", (18, 33, 44), (O_,) * 6, (0.0, 0.0, 0.0)),
    ("reflect_g", (66, 12, 20), (R_,) * 6, (0.05, -0.1, 0.2)),
    ("mixed_g", (40, 18, 130), (P_, P_, O_, O_, R_, R_), (0.0, 0.0, -0.3)),
    ("line_x", (1, 1, 300), (O_, O_, P_, P_, P_, P_), (0.0, 0.0, 0.0)),
]


def _scale(U, dx, grav):
    """sum |q| dV per total (the sixth: |E| + |rho phi|)."""
    vol = float(np.prod(dx))
    s = [float(np.abs(U[v]).sum()) * vol for v in range(5)]
    nz, ny, nx = U.shape[1:]
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dx[2], (np.arange(ny) + 0.5) * dx[1],
                          (np.arange(nx) + 0.5) * dx[0], indexing="ij")
    phi = -(grav[0] * x + grav[1] * y + grav[2] * z)
    s.append(s[4] + float(np.abs(U[0] * phi).sum()) * vol)
    return np.array(s)


def _check(got, want, scale, where):
    for v in range(6):
        assert abs(got[v] - want[v]) <= 1e-14 * scale[v], (where, v, got[v], want[v])


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("name,shape,bc,grav", CASES)
def test_folded_totals_match_oracle_and_replay(name, shape, bc, grav, prec):
    P = ic.smooth_random(shape, seed=51, bc=bc, grav=grav)
    p = params_of(P)
    g, dev = gpu_grid(P, prec=prec)
    # before any step: the replayed sums of the current state
    t0 = np.array(g.totals())
    _check(t0, oracle.totals(p, host(dev)), _scale(host(dev), P.dx, grav), (name, "start"))
    for step in range(4):
        say(f"totals {name} prec {prec} step {step}")
        g.step()
        folded = np.array(g.totals())
        state = host(dev)
        _check(folded, oracle.totals(p, state), _scale(state, P.dx, grav), (name, step))
        g.state_changed()
        replay = g.totals()
        assert folded.tolist() == list(replay), (name, step, folded, replay)
    assert g.error() == hydro.HYDRO_OK
    g.close()


def test_folded_totals_run_to_run_and_graph_vs_eager():
    P = ic.kh(shape=(40, 64, 72), seed=52)
    seqs = []
    for flags in (hydro.FLAG_NO_TUNE, hydro.FLAG_NO_TUNE, hydro.FLAG_NO_TUNE | hydro.FLAG_NO_GRAPH):
        g, dev = gpu_grid(P, prec=hydro.FP32, flags=flags)
        seq = []
        for _ in range(5):
            g.step()
            seq.append(g.totals())
        seqs.append(seq)
        g.close()
    assert seqs[0] == seqs[1] == seqs[2]


@pytest.mark.parametrize("cfg", ["x:v=4,b=256;y:q=64,s=1;z:q=64,s=2",
                                 "x:v=1,b=128,m=1;y:q=128,s=2;z:q=128,s=4",
                                 "x:v=2,b=128;y:q=64,s=4;z:q=256,s=1"])
def test_folded_totals_in_every_kernel_shape(cfg):
    # lane runs and the x march (odd steps end with x), column marches of
    # one and several segments (even steps end with z)
    P = ic.smooth_random((30, 40, 136), seed=53, bc=(P_, P_, O_, O_, R_, R_),
                         grav=(0.0, 0.0, -0.2))
    p = params_of(P)
    g, dev = gpu_grid(P, config=cfg)
    for step in range(2):
        say(f"totals {cfg} step {step}")
        g.step()
        folded = np.array(g.totals())
        state = host(dev)
        _check(folded, oracle.totals(p, state), _scale(state, P.dx, P.grav), (cfg, step))
        g.state_changed()
        assert folded.tolist() == list(g.totals())
    g.close()


def _batch(prec, cfg, count=24, seed=3):
    specs = ic.batch_specs(count, seed=seed)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = ic.batch_pool(specs, ng=4, dtype=dt, pad_rows=32)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, 5.0 / 3.0, flags=hydro.FLAG_NO_TUNE)
    if cfg:
        b.config = cfg
    return b, dev, patches


@pytest.mark.parametrize("prec,cfg", [(hydro.FP64, ""), (hydro.FP32, ""),
                                      (hydro.FP32, "p:f=1;w:v=4,b=256"),
                                      (hydro.FP32, "p:d=0,f=1;w:v=2,b=512")])
def test_batch_folded_totals(prec, cfg):
    b, dev, patches = _batch(prec, cfg)
    say(f"batch totals prec {prec} config {b.config}")
    for step in range(3):
        b.step()
        folded = np.array(b.totals())
        out = host(dev)
        want = np.zeros(6)
        scale = np.zeros(6)
        for pch in patches:
            ng = pch[4]
            u = np.ascontiguousarray(ic.patch_view(out, pch)[:, ng:-ng, ng:-ng, ng:-ng])
            prm = oracle.make_params(u.shape[1:], pch[5], 5.0 / 3.0, 0.8)
            want += oracle.totals(prm, u)
            scale += _scale(u, (pch[5],) * 3, (0.0, 0.0, 0.0))
        _check(folded, want, scale, (cfg, step))
        b.state_changed()
        assert folded.tolist() == list(b.totals())
    b.close()
