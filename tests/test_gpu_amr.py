"""AMR operators on the GPU against the oracle, bit for bit: stored-ghost
fills of grids (ghost depths beyond an axis length, every boundary kind) and
of batches (padded and unpadded rows), restriction and prolongation (the
fine interior or only its ghost shell) between patches of one batch, FP32
and FP64; the prolong-then-restrict round trip; and the argument errors."""
import ctypes

import numpy as np
import pytest

import hydro_ic as ic
from gpu_util import say, torch
from oracle import amr
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

P, O, R = hydro.PERIODIC, hydro.OUTFLOW, hydro.REFLECT


def rand_interior(shape, seed):
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(5,) + shape)
    U[0] = rng.uniform(0.5, 2.0, shape)
    U[4] = rng.uniform(2.0, 4.0, shape)
    return U


def stored_nan(U, ng):
    S = np.full((5,) + tuple(s + 2 * ng for s in U.shape[1:]), np.nan)
    S[:, ng:S.shape[1] - ng, ng:S.shape[2] - ng, ng:S.shape[3] - ng] = U
    return S


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("ng,bc", [(1, (P,) * 6), (3, (P, P, O, R, R, O)), (5, (R,) * 6),
                                   (4, (O,) * 6)])
def test_grid_fill_ghosts(prec, ng, bc):
    say(f"grid fill prec={prec} ng={ng} bc={bc}")
    shape = (6, 3, 7)                       # (nz, ny, nx): ny = 3 < ng for some cases
    dt = np.float64 if prec == hydro.FP64 else np.float32
    S = stored_nan(rand_interior(shape, 1).astype(dt).astype(np.float64), ng)
    dev = torch().from_numpy(S.astype(dt)).to("cuda:0")
    g = hydro.Grid(dev, (0.1, 0.2, 0.3), 1.4, bc=bc, ng=ng, flags=hydro.FLAG_NO_TUNE)
    g.fill_ghosts()
    got = dev.double().cpu().numpy()
    np.testing.assert_array_equal(got, amr.fill_ghosts(S, ng, bc))
    g.close()


def make_pool(shapes, ng, dtype, seed, pad_rows=0):
    """A batch pool of patches of the given interior shapes (nz, ny, nx),
    each with ng ghost layers (NaN), laid out back to back."""
    layout, off = [], 0
    for (nz, ny, nx) in shapes:
        if pad_rows:
            A = pad_rows
            rp = -(-(A + nx + ng) // A) * A
            x0 = A - ng
        else:
            rp, x0 = nx + 2 * ng, 0
        sp = rp * (ny + 2 * ng)
        pp = sp * (nz + 2 * ng)
        io = x0 + ng + ng * rp + ng * sp
        layout.append((off, rp, sp, pp, io, x0))
        off += 5 * pp
        off = (off + 63) // 64 * 64
    pool = np.full(off, np.nan)
    patches = []
    for k, ((nz, ny, nx), (o, rp, sp, pp, io, x0)) in enumerate(zip(shapes, layout)):
        view = pool[o:o + 5 * pp].reshape(5, nz + 2 * ng, ny + 2 * ng, rp)
        view[:, ng:ng + nz, ng:ng + ny, x0 + ng:x0 + ng + nx] = rand_interior((nz, ny, nx), seed + k)
        d = 1.0 / nx
        patches.append((o, nx, ny, nz, ng, d, d, d, rp, sp, pp, io))
    return pool.astype(dtype).astype(np.float64), patches


def sview(pool, p):
    return ic.patch_view(pool, p)


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("pad", [0, 32])
def test_batch_fill_ghosts(prec, pad):
    say(f"batch fill prec={prec} pad={pad}")
    dt = np.float64 if prec == hydro.FP64 else np.float32
    bc = (P, P, R, R, O, O)
    pool, patches = make_pool([(8, 6, 10), (4, 4, 4), (6, 12, 8)], 3, dt, 2, pad)
    dev = torch().from_numpy(pool.astype(dt)).to("cuda:0")
    b = hydro.Batch(dev, patches, 1.4, bc=bc, flags=hydro.FLAG_NO_TUNE)
    b.fill_ghosts()
    got = dev.double().cpu().numpy()
    for p in patches:
        np.testing.assert_array_equal(sview(got, p), amr.fill_ghosts(sview(pool, p), 3, bc))
    b.close()


def _amr_batch(prec, seed=3):
    """Coarse patch 0 (12 x 10 x 14 interior, 2 ghosts) and two fine patches
    (ng 2) inside it: patch 1 (8 x 6 x 4 fine cells) at coarse (1, 2, 3),
    patch 2 (4 x 8 x 6) at coarse (8, 1, 5)."""
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = make_pool([(12, 10, 14), (4, 6, 8), (6, 8, 4)], 2, dt, seed)
    links = [(1, 0, 1, 2, 3), (2, 0, 8, 1, 5)]
    dev = torch().from_numpy(pool.astype(dt)).to("cuda:0")
    b = hydro.Batch(dev, patches, 1.4, flags=hydro.FLAG_NO_TUNE)
    return b, dev, pool, patches, links, dt


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
def test_restrict(prec):
    say(f"restrict prec={prec}")
    b, dev, pool, patches, links, dt = _amr_batch(prec)
    b.restrict(links)
    got = dev.double().cpu().numpy()
    C = sview(pool, patches[0])
    for f, c, ox, oy, oz in links:
        C = amr.restrict(sview(pool, patches[f]), 2, C, 2, (ox, oy, oz))
    np.testing.assert_array_equal(sview(got, patches[0]), C.astype(dt).astype(np.float64))
    b.close()


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("ghosts_only", [False, True])
def test_prolong(prec, ghosts_only):
    say(f"prolong prec={prec} ghosts_only={ghosts_only}")
    b, dev, pool, patches, links, dt = _amr_batch(prec, seed=4)
    b.fill_ghosts()                                   # coarse ghosts used by the stencil
    b.prolong(links, ghosts_only=ghosts_only)
    got = dev.double().cpu().numpy()
    C = amr.fill_ghosts(sview(pool, patches[0]), 2, (P,) * 6)
    for f, c, ox, oy, oz in links:
        Ff = amr.fill_ghosts(sview(pool, patches[f]), 2, (P,) * 6)
        want = amr.prolong(C, 2, Ff, 2, (ox, oy, oz), ghosts_only=ghosts_only)
        np.testing.assert_array_equal(sview(got, patches[f]), want.astype(dt).astype(np.float64))
    b.close()


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("ng", [2, 4])
def test_prolong_ghost_shell_of_a_large_patch(prec, ng):
    """Ghost prolongation of a fine patch of 28 x 24 x 20 cells at coarse
    (4, 4, 4) of a 22 x 20 x 18 coarse patch.  With 2 ghost layers the
    parents with a ghost child are 37.5 % of the box of parents, so the
    launch walks only those (a grid layer per variable); with 4 they are
    58 % and it walks the whole box: both bit for bit against the oracle."""
    say(f"prolong large patch prec={prec} ng={ng}")
    dt = np.float64 if prec == hydro.FP64 else np.float32
    pool, patches = make_pool([(18, 20, 22), (20, 24, 28)], ng, dt, 7)
    links = [(1, 0, 4, 4, 4)]
    dev = torch().from_numpy(pool.astype(dt)).to("cuda:0")
    b = hydro.Batch(dev, patches, 1.4, flags=hydro.FLAG_NO_TUNE)
    b.fill_ghosts()                                   # coarse ghosts used by the stencil
    b.prolong(links, ghosts_only=True)
    got = dev.double().cpu().numpy()
    C = amr.fill_ghosts(sview(pool, patches[0]), ng, (P,) * 6)
    Ff = amr.fill_ghosts(sview(pool, patches[1]), ng, (P,) * 6)
    want = amr.prolong(C, ng, Ff, ng, (4, 4, 4), ghosts_only=True)
    np.testing.assert_array_equal(sview(got, patches[1]), want.astype(dt).astype(np.float64))
    b.close()


def test_prolong_then_restrict_returns_the_coarse_cells():
    say("prolong-restrict round trip")
    b, dev, pool, patches, links, dt = _amr_batch(hydro.FP64, seed=5)
    b.fill_ghosts()
    before = sview(dev.cpu().numpy(), patches[0]).copy()
    b.prolong(links)
    b.restrict(links)
    after = sview(dev.cpu().numpy(), patches[0])
    np.testing.assert_allclose(after, before, rtol=1e-15, atol=1e-15)
    b.close()


def test_amr_argument_errors():
    b, dev, pool, patches, links, dt = _amr_batch(hydro.FP64)
    # index out of range, fine == coarse, past the coarse interior (x 11..14
    # of 14 cells), before it
    bad = [[(3, 0, 0, 0, 0)], [(1, 1, 0, 0, 0)], [(1, 0, 11, 0, 0)], [(1, 0, -1, 0, 0)]]
    for lk in bad:
        with pytest.raises(hydro.HydroError) as e:
            b.restrict(lk)
        assert e.value.status == hydro.HYDRO_EINVAL
    # prolongation needs the parents' neighbours inside the coarse stored
    # region (14 interior cells + 2 ghosts along x): the 8-cell fine
    # interior at coarse x = 11 reaches coarse x 15 (the last ghost), its
    # ghost shell one cell further (refused)
    b.prolong([(1, 0, 11, 0, 0)])
    with pytest.raises(hydro.HydroError) as e:
        b.prolong([(1, 0, 11, 0, 0)], ghosts_only=True)
    assert e.value.status == hydro.HYDRO_EINVAL
    b.close()
    g = hydro.Grid(torch().zeros((5, 4, 4, 4), dtype=torch().float64, device="cuda:0") + 1.0,
                   (0.25,) * 3, 1.4, flags=hydro.FLAG_NO_TUNE)
    with pytest.raises(hydro.HydroError) as e:
        hydro.hydro_amr_restrict(g.ctx, [(0, 0, 0, 0, 0)])
    assert e.value.status == hydro.HYDRO_ESTATE
    g.close()
