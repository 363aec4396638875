"""The subcycled two-level step (hydro_amr_step) on the GPU against the
oracle's level_step: a periodic coarse grid with two fine patches of uneven
shapes, two steps (both sweep orders), FP64 to 1e-12 and FP32 to an L1
bound, with and without refluxing; the composite totals conserved on the
GPU; and the argument errors, all raised on the host before any launch."""
import ctypes

import numpy as np
import pytest

import hydro_ic as ic
import oracle
from gpu_util import l1_fp32_errors, say, torch
from oracle import amr
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

G = 4
GAMMA = 1.4
SHAPE = (14, 16, 18)                      # coarse (nz, ny, nx)
DX = (1 / 18, 1 / 16, 1 / 14)
# fine interior extents (nx, ny, nz) and the coarse cell of fine cell (0,0,0)
FINE = [((10, 8, 6), (3, 4, 3)), ((6, 8, 8), (11, 7, 6))]


def inputs(seed):
    C = ic.smooth_random(SHAPE, seed, gamma=GAMMA, mach=0.3).U
    fines = []
    for i, (n, _) in enumerate(FINE):
        shp = (n[2] + 2 * G, n[1] + 2 * G, n[0] + 2 * G)
        fines.append(ic.smooth_random(shp, seed + 10 + i, gamma=GAMMA, mach=0.3).U)
    return C, fines


def device_levels(C, fines, prec, bc_fine=(hydro.OUTFLOW,) * 6, grav=(0.0, 0.0, 0.0)):
    dt = np.float64 if prec == hydro.FP64 else np.float32
    tc = torch().from_numpy(C.reshape(-1).astype(dt)).to("cuda:0")
    coarse = hydro.Batch(tc, [(0, SHAPE[2], SHAPE[1], SHAPE[0], 0) + DX], GAMMA, grav=grav,
                         flags=hydro.FLAG_NO_TUNE)
    offs, flat = [], []
    off = 0
    for F in fines:
        offs.append(off)
        flat.append(F.reshape(-1))
        off += F.size
        pad = (-off) % 64
        flat.append(np.zeros(pad))
        off += pad
    tf = torch().from_numpy(np.concatenate(flat).astype(dt)).to("cuda:0")
    patches = []
    for o, F in zip(offs, fines):
        nz, ny, nx = F.shape[1:]
        patches.append((o, nx, ny, nz, 0, DX[0] / 2, DX[1] / 2, DX[2] / 2))
    fine = hydro.Batch(tf, patches, GAMMA, bc=bc_fine, grav=grav, flags=hydro.FLAG_NO_TUNE)
    links = [(i, 0) + tuple(o) for i, (_, o) in enumerate(FINE)]
    return coarse, fine, tc, tf, offs, links


def read(tc, tf, offs, fines):
    C = tc.double().cpu().numpy().reshape((5,) + SHAPE)
    f = tf.double().cpu().numpy()
    return C, [f[o:o + F.size].reshape(F.shape) for o, F in zip(offs, fines)]


def step_dt(C, fines):
    pc = oracle.make_params(SHAPE, DX, GAMMA)
    dtf = min(oracle.cfl_dt(oracle.make_params(F.shape[1:], tuple(h / 2 for h in DX), GAMMA), F)
              for F in fines)
    return 0.5 * min(oracle.cfl_dt(pc, C), 2 * dtf)


def max_rel(got, want):
    return max(float(np.abs(got[v] - want[v]).max() / max(np.abs(want[v]).max(), 1e-300))
               for v in range(5))


def composite(C, fines):
    cov = np.zeros(SHAPE, bool)
    tot = np.zeros(5)
    for F, (n, o) in zip(fines, FINE):
        cov[o[2]:o[2] + n[2] // 2, o[1]:o[1] + n[1] // 2, o[0]:o[0] + n[0] // 2] = True
        tot += F[:, G:-G, G:-G, G:-G].sum(axis=(1, 2, 3)) / 8
    return (tot + C[:, ~cov].sum(axis=1)) * np.prod(DX)


@pytest.mark.parametrize("reflux", [True, False])
@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
def test_two_steps_match_the_oracle(prec, reflux):
    say(f"amr step prec={prec} reflux={reflux}")
    C, fines = inputs(21)
    if prec == hydro.FP32:
        C = C.astype(np.float32).astype(np.float64)
        fines = [F.astype(np.float32).astype(np.float64) for F in fines]
    coarse, fine, tc, tf, offs, links = device_levels(C, fines, prec)
    lv = hydro.AmrLevels(coarse, fine, links, G)
    Cw, fw = C, fines
    offsets = [o for _, o in FINE]
    for s in range(2):
        dt = step_dt(Cw, fw)
        Cw, fw = amr.level_step(Cw, fw, offsets, G, dt, GAMMA, DX, step_c=s, step_f=2 * s,
                                reflux=reflux)
        lv.step(dt, reflux=reflux)
        Cg, fg = read(tc, tf, offs, fines)
        if prec == hydro.FP64:
            e = [max_rel(Cg, Cw)] + [max_rel(a, b) for a, b in zip(fg, fw)]
            say(f"  step {s} max rel {e}")
            assert max(e) <= 1e-12, e
        else:
            e = [l1_fp32_errors(Cg, Cw)] + [l1_fp32_errors(a[:, G:-G, G:-G, G:-G],
                                                           b[:, G:-G, G:-G, G:-G])
                                            for a, b in zip(fg, fw)]
            say(f"  step {s} L1 {e}")
            # one step (each starts from the GPU state) on two levels: a few
            # FP32 roundings per sweep, like the single-grid bound of 2e-6
            assert max(max(x) for x in e) <= 4e-6, e
        Cw, fw = Cg, fg          # the next step starts from the GPU state
    assert coarse.time()[1] == 2 and fine.time()[1] == 4
    coarse.close()
    fine.close()


def test_gravity_matches_the_oracle():
    # gravity enters the registers' face states (half kick) and the sweeps'
    # momentum and energy sources; both levels share it
    say("amr step with gravity")
    grav = (0.1, -0.2, -0.5)
    C, fines = inputs(24)
    coarse, fine, tc, tf, offs, links = device_levels(C, fines, hydro.FP64, grav=grav)
    lv = hydro.AmrLevels(coarse, fine, links, G)
    offsets = [o for _, o in FINE]
    Cw, fw = C, fines
    for s in range(2):
        dt = step_dt(Cw, fw)
        if s == 0:
            # the case exercises gravity: without it the first step differs
            plain, _ = amr.level_step(C, fines, offsets, G, dt, GAMMA, DX)
        Cw, fw = amr.level_step(Cw, fw, offsets, G, dt, GAMMA, DX, grav=grav,
                                step_c=s, step_f=2 * s)
        if s == 0:
            assert max_rel(plain, Cw) > 1e-6
        lv.step(dt)
        Cg, fg = read(tc, tf, offs, fines)
        e = [max_rel(Cg, Cw)] + [max_rel(a, b) for a, b in zip(fg, fw)]
        say(f"  step {s} max rel {e}")
        assert max(e) <= 1e-12, e
        Cw, fw = Cg, fg
    coarse.close()
    fine.close()


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
def test_composite_totals_are_conserved_on_the_gpu(prec):
    say(f"amr step conservation prec={prec}")
    C, fines = inputs(22)
    if prec == hydro.FP32:
        C = C.astype(np.float32).astype(np.float64)
        fines = [F.astype(np.float32).astype(np.float64) for F in fines]
    coarse, fine, tc, tf, offs, links = device_levels(C, fines, prec)
    lv = hydro.AmrLevels(coarse, fine, links, G)
    before = composite(C, fines)
    scale = np.abs(C).sum(axis=(1, 2, 3)) * np.prod(DX)
    for s in range(3):
        lv.step(step_dt(*read(tc, tf, offs, fines)))
    Cg, fg = read(tc, tf, offs, fines)
    after = composite(Cg, fg)
    tot = np.asarray(coarse.totals()[:5])
    err = np.abs(after - before) / scale
    say(f"  conservation {err}")
    # FP64: round-off; FP32: every update of a cell is rounded to FP32,
    # random-signed errors of 2^-24 relative that largely cancel in the
    # totals (measured about 2e-9)
    bound = 1e-13 if prec == hydro.FP64 else 1e-7
    assert err.max() < bound, err
    np.testing.assert_allclose(tot, after, rtol=bound, atol=bound * scale.max())
    coarse.close()
    fine.close()


def test_argument_errors():
    say("amr step errors")
    C, fines = inputs(23)
    coarse, fine, tc, tf, offs, links = device_levels(C, fines, hydro.FP64)
    lib = hydro.lib()
    nbytes = hydro.hydro_amr_step_workspace_bytes(coarse.ctx, fine.ctx, G)
    ws = torch().empty(nbytes, dtype=torch().uint8, device="cuda:0")
    wp = ctypes.c_void_p(ws.data_ptr())

    def call(lk, g=G, dt=1e-3, flags=0, c=coarse.ctx, f=fine.ctx, nb=nbytes):
        arr = hydro.make_links(lk)
        return lib.hydro_amr_step(c, f, arr, len(lk), g, dt, flags, wp, nb)

    E = hydro.HYDRO_EINVAL
    assert call(links, g=1) == E                                   # too few ghosts
    assert call([links[0]]) == E                                   # a fine patch unlinked
    assert call([links[0], links[0]]) == E                         # linked twice
    assert call([(0, 0, 2, 4, 3), links[1]]) == E                  # too close to the edge
    assert call([links[0], (1, 0, 8, 4, 3)]) == E                  # touching patch 0
    assert call([links[0], (1, 1, 11, 7, 6)]) == E                 # no such coarse patch
    assert call(links, dt=0.0) == E
    assert call(links, flags=4) == E
    assert call(links, nb=nbytes - 8) == E
    assert call(links, f=coarse.ctx) == E                          # one context twice
    # fine cells not half as wide
    tf2 = tf.clone()
    wrong = [(o, F.shape[3], F.shape[2], F.shape[1], 0, DX[0], DX[1] / 2, DX[2] / 2)
             for o, F in zip(offs, fines)]
    fine2 = hydro.Batch(tf2, wrong, GAMMA, flags=hydro.FLAG_NO_TUNE)
    assert call(links, f=fine2.ctx) == E
    fine2.close()
    coarse.close()
    fine.close()


def test_many_small_patches_match_the_oracle():
    # 144 one-coarse-cell patches: more links than one kernel's arguments
    # hold, so the device link table is written in several chunks
    say("amr step 144 small patches")
    shape = (16, 16, 16)
    dx = (1 / 16,) * 3
    g = 2
    offs = [(x, y, z) for z in range(2, 14, 3) for y in range(2, 14, 2)
            for x in range(2, 14, 2)]
    assert len(offs) == 144
    C = ic.smooth_random(shape, 31, gamma=GAMMA, mach=0.3).U
    fines = [ic.smooth_random((6, 6, 6), 100 + i, gamma=GAMMA, mach=0.3).U
             for i in range(len(offs))]
    tc = torch().from_numpy(C.reshape(-1).copy()).to("cuda:0")
    coarse = hydro.Batch(tc, [(0, 16, 16, 16, 0) + dx], GAMMA, flags=hydro.FLAG_NO_TUNE)
    per = 5 * 6 ** 3
    tf = torch().from_numpy(np.concatenate([F.reshape(-1) for F in fines])).to("cuda:0")
    fine = hydro.Batch(tf, [(i * per, 6, 6, 6, 0) + tuple(h / 2 for h in dx)
                            for i in range(len(offs))], GAMMA,
                       bc=(hydro.OUTFLOW,) * 6, flags=hydro.FLAG_NO_TUNE)
    links = [(i, 0) + o for i, o in enumerate(offs)]
    lv = hydro.AmrLevels(coarse, fine, links, g)
    dtf = min(oracle.cfl_dt(oracle.make_params((6, 6, 6), tuple(h / 2 for h in dx), GAMMA), F)
              for F in fines)
    dt = 0.5 * min(oracle.cfl_dt(oracle.make_params(shape, dx, GAMMA), C), 2 * dtf)
    Cw, fw = amr.level_step(C, fines, offs, g, dt, GAMMA, dx)
    lv.step(dt)
    Cg = tc.cpu().numpy().reshape((5,) + shape)
    fg = tf.cpu().numpy()
    e = [max_rel(Cg, Cw)] + [max_rel(fg[i * per:(i + 1) * per].reshape(5, 6, 6, 6), fw[i])
                             for i in range(len(offs))]
    say(f"  max rel {max(e)}")
    assert max(e) <= 1e-12
    coarse.close()
    fine.close()


def test_two_ghost_layers_large_patch_matches_the_oracle():
    """A fine patch of 28 x 24 x 20 cells with 2 ghost layers: its ghost
    prolongation walks only the parents with a ghost child (37.5 % of the
    box), from the start-of-step cells and from cells interpolated in time.
    Two steps (both sweep orders) against the oracle to 1e-12 (FP64)."""
    say("amr step large patch, 2 ghost layers")
    shape = (20, 20, 24)                  # coarse (nz, ny, nx)
    dx = (1 / 24, 1 / 20, 1 / 20)
    g, n, off = 2, (28, 24, 20), (4, 4, 4)
    fdx = tuple(h / 2 for h in dx)
    C = ic.smooth_random(shape, 41, gamma=GAMMA, mach=0.3).U
    F = ic.smooth_random((n[2] + 2 * g, n[1] + 2 * g, n[0] + 2 * g), 42, gamma=GAMMA,
                         mach=0.3).U
    tc = torch().from_numpy(C.reshape(-1).copy()).to("cuda:0")
    coarse = hydro.Batch(tc, [(0, shape[2], shape[1], shape[0], 0) + dx], GAMMA,
                         flags=hydro.FLAG_NO_TUNE)
    tf = torch().from_numpy(F.reshape(-1).copy()).to("cuda:0")
    fine = hydro.Batch(tf, [(0, n[0] + 2 * g, n[1] + 2 * g, n[2] + 2 * g, 0) + fdx], GAMMA,
                       bc=(hydro.OUTFLOW,) * 6, flags=hydro.FLAG_NO_TUNE)
    lv = hydro.AmrLevels(coarse, fine, [(0, 0) + off], g)
    Cw, Fw = C, F
    for s in range(2):
        dtf = oracle.cfl_dt(oracle.make_params(Fw.shape[1:], fdx, GAMMA), Fw)
        dt = 0.5 * min(oracle.cfl_dt(oracle.make_params(shape, dx, GAMMA), Cw), 2 * dtf)
        Cw, fw = amr.level_step(Cw, [Fw], [off], g, dt, GAMMA, dx, step_c=s, step_f=2 * s)
        Fw = fw[0]
        lv.step(dt)
        Cg = tc.cpu().numpy().reshape((5,) + shape)
        Fg = tf.cpu().numpy().reshape(F.shape)
        e = [max_rel(Cg, Cw), max_rel(Fg, Fw)]
        say(f"  step {s} max rel {e}")
        assert max(e) <= 1e-12, e
        Cw, Fw = Cg, Fg          # the next step starts from the GPU state
    coarse.close()
    fine.close()


def test_fp32_ten_steps_stay_within_the_l1_bound():
    # an FP32 trajectory of ten steps against the FP64 oracle's, both from
    # the same FP32-representable state with the oracle's dt sequence: the
    # error is FP32 round-off accumulated over the steps
    say("amr step fp32 ten steps")
    C, fines = inputs(25)
    C = C.astype(np.float32).astype(np.float64)
    fines = [F.astype(np.float32).astype(np.float64) for F in fines]
    coarse, fine, tc, tf, offs, links = device_levels(C, fines, hydro.FP32)
    lv = hydro.AmrLevels(coarse, fine, links, G)
    offsets = [o for _, o in FINE]
    Cw, fw = C, fines
    for s in range(10):
        dt = step_dt(Cw, fw)
        Cw, fw = amr.level_step(Cw, fw, offsets, G, dt, GAMMA, DX, step_c=s, step_f=2 * s)
        lv.step(dt)
    Cg, fg = read(tc, tf, offs, fines)
    e = [l1_fp32_errors(Cg, Cw)] + [l1_fp32_errors(a[:, G:-G, G:-G, G:-G],
                                                   b[:, G:-G, G:-G, G:-G])
                                    for a, b in zip(fg, fw)]
    say(f"  ten-step L1 (rho, m, E) per level {e}")
    assert max(max(x) for x in e) <= 2e-5, e
    coarse.close()
    fine.close()


def test_two_coarse_patches_one_with_stored_ghosts():
    # links point at two coarse patches of one batch; the second keeps 2
    # stored ghost layers (its interior sits at an offset in the pool).  The
    # patches are independent, so the oracle steps each with its own fine
    # patches.
    say("amr step two coarse patches")
    shapes = [(14, 16, 18), (12, 12, 16)]          # (nz, ny, nx)
    ngs = [0, 2]
    dxs = [(1 / 18, 1 / 16, 1 / 14), (1 / 16, 1 / 12, 1 / 12)]
    fine_of = [[((10, 8, 6), (3, 4, 3)), ((6, 8, 8), (11, 7, 6))], [((8, 6, 6), (4, 3, 3))]]
    Cs = [ic.smooth_random(s, 41 + i, gamma=GAMMA, mach=0.3).U for i, s in enumerate(shapes)]
    fines = []
    for c, fl in enumerate(fine_of):
        for i, (n, _) in enumerate(fl):
            shp = (n[2] + 2 * G, n[1] + 2 * G, n[0] + 2 * G)
            fines.append(ic.smooth_random(shp, 60 + 10 * c + i, gamma=GAMMA, mach=0.3).U)
    # coarse pool: patch 0 packed, patch 1 with its stored ghosts (NaN)
    parts, cpatches, off = [], [], 0
    for C, ng, dx in zip(Cs, ngs, dxs):
        S = np.full((5,) + tuple(s + 2 * ng for s in C.shape[1:]), np.nan)
        S[:, ng:S.shape[1] - ng, ng:S.shape[2] - ng, ng:S.shape[3] - ng] = C
        parts.append(S.reshape(-1))
        nz, ny, nx = C.shape[1:]
        cpatches.append((off, nx, ny, nz, ng) + dx)
        off += S.size
        pad = (-off) % 64
        parts.append(np.zeros(pad))
        off += pad
    tc = torch().from_numpy(np.concatenate(parts)).to("cuda:0")
    coarse = hydro.Batch(tc, cpatches, GAMMA, flags=hydro.FLAG_NO_TUNE)
    fparts, fpatches, foffs, off = [], [], [], 0
    k = 0
    for c, fl in enumerate(fine_of):
        for (n, o) in fl:
            F = fines[k]
            foffs.append(off)
            fparts.append(F.reshape(-1))
            nz, ny, nx = F.shape[1:]
            fpatches.append((off, nx, ny, nz, 0) + tuple(h / 2 for h in dxs[c]))
            off += F.size
            pad = (-off) % 64
            fparts.append(np.zeros(pad))
            off += pad
            k += 1
    tf = torch().from_numpy(np.concatenate(fparts)).to("cuda:0")
    fine = hydro.Batch(tf, fpatches, GAMMA, bc=(hydro.OUTFLOW,) * 6, flags=hydro.FLAG_NO_TUNE)
    links, k = [], 0
    for c, fl in enumerate(fine_of):
        for (_, o) in fl:
            links.append((k, c) + tuple(o))
            k += 1
    lv = hydro.AmrLevels(coarse, fine, links, G)
    dt = 1e30
    k = 0
    for c, fl in enumerate(fine_of):
        pc = oracle.make_params(shapes[c], dxs[c], GAMMA)
        dt = min(dt, oracle.cfl_dt(pc, Cs[c]))
        for _ in fl:
            pf = oracle.make_params(fines[k].shape[1:], tuple(h / 2 for h in dxs[c]), GAMMA)
            dt = min(dt, 2 * oracle.cfl_dt(pf, fines[k]))
            k += 1
    # the library's level dt (hydro_amr_cfl_dt) is the same minimum
    level_dt = lv.cfl_dt()
    assert abs(level_dt - dt) <= 1e-14 * dt, (level_dt, dt)
    dt *= 0.5
    lv.step(dt)
    got_pool = tc.cpu().numpy()
    got_f = tf.cpu().numpy()
    k = 0
    for c, fl in enumerate(fine_of):
        want_c, want_f = amr.level_step(Cs[c], fines[k:k + len(fl)], [o for _, o in fl], G, dt,
                                        GAMMA, dxs[c])
        o0, nx, ny, nz, ng = cpatches[c][:5]
        S = got_pool[o0:o0 + 5 * (nz + 2 * ng) * (ny + 2 * ng) * (nx + 2 * ng)].reshape(
            5, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng)
        got_c = S[:, ng:ng + nz, ng:ng + ny, ng:ng + nx]
        e = [max_rel(got_c, want_c)]
        if ng:
            assert np.all(np.isnan(S[:, :ng])), "stored coarse ghosts were written"
        for i, W in enumerate(want_f):
            F = got_f[foffs[k + i]:foffs[k + i] + W.size].reshape(W.shape)
            e.append(max_rel(F, W))
        say(f"  coarse patch {c}: max rel {e}")
        assert max(e) <= 1e-12, e
        k += len(fl)
    coarse.close()
    fine.close()
