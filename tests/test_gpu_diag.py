"""In-situ diagnostics on the GPU against the oracle: PDF counts bit for
bit (the bin decision is taken in FP64 with IEEE operations on both sides),
slab profiles and mixing measures within the FP64 summation bound, on
ragged shapes, with stored ghost layers, FP32 and FP64 states, both counter
paths (LDS and global), batches, the full KH grid, and the error paths."""
import ctypes

import numpy as np
import pytest

import hydro_ic as ic
from gpu_util import say, torch
from oracle import diagnostics as D
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu

QUANTS = (hydro.Q_RHO, hydro.Q_PRESSURE, hydro.Q_SPEED, hydro.Q_MACH)
EPS = np.finfo(np.float64).eps


def _state(shape, seed, ng=0, prec=hydro.FP64, special=True):
    """A smooth random state (interior shape (nz, ny, nx)) with ng stored
    ghost layers of junk around it, plus a few special cells: a negative
    pressure (Mach is NaN there) and one cell exactly on a bin edge."""
    P = ic.smooth_random(shape, seed, gamma=1.4, mach=0.8)
    U = P.U.copy()
    if special:
        U[4, 0, 0, 0] = 0.1 * U[0, 0, 0, 0]          # E below ke: p < 0
        U[0, -1, -1, -1] = 1.25                       # on an edge of [0.5, 2.0) / 8 bins
    dt = np.float64 if prec == hydro.FP64 else np.float32
    U = U.astype(dt)
    if ng:
        full = np.full((5,) + tuple(s + 2 * ng for s in shape), np.nan, dtype=dt)
        full[:, ng:-ng, ng:-ng, ng:-ng] = U
    else:
        full = U
    dev = torch().from_numpy(np.ascontiguousarray(full)).to("cuda:0")
    g = hydro.Grid(dev, P.dx, P.gamma, ng=ng, flags=hydro.FLAG_NO_TUNE)
    return g, U.astype(np.float64), P


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
@pytest.mark.parametrize("ng", [0, 3])
def test_pdf_bit_exact(prec, ng):
    shape = (23, 29, 37)
    g, U, P = _state(shape, seed=11, ng=ng, prec=prec)
    for q in QUANTS:
        for nb, lo, hi in ((8, 0.5, 2.0), (1, 0.0, 1.0), (1000, -0.3, 3.1), (9000, 0.0, 2.5)):
            say(f"pdf prec={prec} ng={ng} q={q} nb={nb}")
            got = g.pdf(q, lo, hi, nb).cpu().numpy()
            want = D.pdf(U, P.gamma, q, lo, hi, nb)
            np.testing.assert_array_equal(got, want)
            assert got.sum() == U[0].size
    g.close()


def test_pdf_counts_are_overwritten_and_repeatable():
    g, U, P = _state((16, 16, 16), seed=12)
    out = torch().full((42,), 7, dtype=torch().int64, device="cuda:0")
    a = g.pdf(hydro.Q_MACH, 0.0, 2.0, 40, out=out).cpu().numpy()
    b = g.pdf(hydro.Q_MACH, 0.0, 2.0, 40, out=out).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, D.pdf(U, P.gamma, D.MACH, 0.0, 2.0, 40))
    g.close()


@pytest.mark.parametrize("pad", [0, 32])
def test_batch_pdf_bit_exact(pad):
    specs = ic.batch_specs(24, seed=5, sizes=(16, 32, 48))
    pool, patches = ic.batch_pool(specs, ng=4, dtype=np.float32, pad_rows=pad)
    dev = torch().from_numpy(pool).to("cuda:0")
    b = hydro.Batch(dev, patches, 5.0 / 3.0, flags=hydro.FLAG_NO_TUNE)
    interiors = []
    for p in patches:
        ng = p[4]
        interiors.append(ic.patch_view(pool, p)[:, ng:-ng, ng:-ng, ng:-ng].astype(np.float64))
    for q, lo, hi, nb in ((hydro.Q_RHO, 0.9, 4.1, 64), (hydro.Q_MACH, 0.0, 0.6, 300),
                          (hydro.Q_PRESSURE, 2.49, 2.51, 9000)):
        say(f"batch pdf pad={pad} q={q}")
        got = b.pdf(q, lo, hi, nb).cpu().numpy()
        np.testing.assert_array_equal(got, D.pdf(interiors, 5.0 / 3.0, q, lo, hi, nb))
    out = torch().zeros(5 * 64 + 2, dtype=torch().float64, device="cuda:0")
    with pytest.raises(hydro.HydroError) as e:   # a batch has no slab profiles
        hydro.hydro_diag_profile(b.ctx, 2, 1.0, 2.0, ctypes.c_void_p(out.data_ptr()))
    assert e.value.status == hydro.HYDRO_ESTATE
    b.close()


def _profile_bound(U, gamma, axis, rho_lo, rho_hi):
    """Oracle slab means and a per-field bound on |GPU - oracle|.  Both sides
    compute the same per-cell values (same IEEE operations in the same
    order) and differ only in summation order: each sum of m terms is within
    (m - 1) eps of the sum of magnitudes, so the means differ by at most
    2 m eps times the largest mean magnitude (every field is nonnegative
    here), plus the rounding of the division."""
    m = U[0].size // U.shape[3 - axis]
    ref = D.profile(U, gamma, axis, rho_lo, rho_hi)
    scale = np.abs(ref).max(axis=0)
    return ref, 4.0 * m * EPS * np.maximum(scale, 1e-300)


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("ng", [0, 2])
def test_profile_matches_oracle(prec, axis, ng):
    shape = (19, 26, 33)
    say(f"profile prec={prec} axis={axis} ng={ng}")
    g, U, P = _state(shape, seed=13, ng=ng, prec=prec, special=False)
    rho_lo, rho_hi = 1.0, 1.5
    out = g.profile(axis, rho_lo, rho_hi).cpu().numpy()
    n = U.shape[3 - axis]
    assert out.shape == (5 * n + 2,)
    ref, tol = _profile_bound(U, P.gamma, axis, rho_lo, rho_hi)
    got = out[:5 * n].reshape(n, 5)
    assert np.all(np.abs(got - ref) <= tol), (np.abs(got - ref).max(axis=0), tol)
    # W and Theta are sums over n slab means, each within tol of the oracle's
    W, theta = D.mixing(ref, P.dx[axis])
    np.testing.assert_allclose(out[5 * n], W, rtol=1e-10, atol=4 * n * tol[3])
    np.testing.assert_allclose(out[5 * n + 1], theta, rtol=1e-10, atol=4 * n * tol[3])
    again = g.profile(axis, rho_lo, rho_hi).cpu().numpy()
    np.testing.assert_array_equal(out, again)   # fixed summation order
    g.close()


def test_full_kh_grid_pdf_and_profile():
    """KH 256^3 in FP32 after the initial state: the density PDF and the y
    profile (the layer's mixing width) against the oracle."""
    P = ic.kh(256)
    U32 = P.U.astype(np.float32)
    dev = torch().from_numpy(U32).to("cuda:0")
    g = hydro.Grid(dev, P.dx, P.gamma, flags=hydro.FLAG_NO_TUNE)
    U = U32.astype(np.float64)
    say("kh256 pdf")
    for q, lo, hi, nb in ((hydro.Q_RHO, 0.5, 2.5, 200), (hydro.Q_MACH, 0.0, 0.5, 1000)):
        np.testing.assert_array_equal(g.pdf(q, lo, hi, nb).cpu().numpy(),
                                      D.pdf(U, P.gamma, q, lo, hi, nb))
    say("kh256 profile")
    out = g.profile(1, 1.0, 2.0).cpu().numpy()
    ref, tol = _profile_bound(U, P.gamma, 1, 1.0, 2.0)
    got = out[:5 * 256].reshape(256, 5)
    assert np.all(np.abs(got - ref) <= tol)
    # a sharp layer: f is 0 or 1 in every cell, so the width and mixedness are 0
    assert out[5 * 256] == 0.0 and out[5 * 256 + 1] == 0.0
    g.close()


def test_argument_errors():
    g, U, P = _state((8, 8, 8), seed=14, special=False)
    t = torch()
    counts = t.zeros(12, dtype=t.int64, device="cuda:0")
    ptr = ctypes.c_void_p(counts.data_ptr())
    for args in ((4, 0.0, 1.0, 10), (0, 1.0, 1.0, 10), (0, 0.0, 1.0, 0),
                 (0, float("nan"), 1.0, 10), (0, 0.0, float("inf"), 10)):
        with pytest.raises(hydro.HydroError) as e:
            hydro.hydro_diag_pdf(g.ctx, *args, ptr)
        assert e.value.status == hydro.HYDRO_EINVAL
    out = t.zeros(5 * 8 + 2, dtype=t.float64, device="cuda:0")
    optr = ctypes.c_void_p(out.data_ptr())
    for axis, lo, hi in ((3, 1.0, 2.0), (0, 2.0, 1.0), (1, float("nan"), 2.0)):
        with pytest.raises(hydro.HydroError) as e:
            hydro.hydro_diag_profile(g.ctx, axis, lo, hi, optr)
        assert e.value.status == hydro.HYDRO_EINVAL
    g.close()


# ------------------------------------------------------------ spectrum

def _spec_tol(ref):
    """|GPU - oracle| bound: both transform in FP64 (FFT error within a few
    eps log2 N of the line norm), so every power differs by far less than
    1e-12 of the total energy; rtol covers the large components."""
    return dict(rtol=1e-9, atol=1e-12 * float(np.abs(ref).sum()))


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
@pytest.mark.parametrize("nx", [2, 3, 12, 16, 48, 96, 256, 768, 1024])
def test_spectrum_matches_oracle(prec, nx):
    say(f"spectrum prec={prec} nx={nx}")
    g, U, P = _state((3, 5, nx), seed=15 + nx, ng=2 if nx % 3 == 0 else 0, prec=prec,
                     special=False)
    E = g.spectrum().cpu().numpy()
    ref = D.spectrum_x(U)
    assert E.shape == ref.shape == (nx // 2 + 1,)
    np.testing.assert_allclose(E, ref, **_spec_tol(ref))
    np.testing.assert_array_equal(E, g.spectrum().cpu().numpy())   # fixed order
    g.close()


def test_spectrum_more_lines_than_workgroups_and_a_single_mode():
    # 37 x 31 = 1147 lines (> 1024 workgroups): every line still counted once
    say("spectrum many lines")
    g, U, P = _state((37, 31, 24), seed=16, special=False)
    ref = D.spectrum_x(U)
    np.testing.assert_allclose(g.spectrum().cpu().numpy(), ref, **_spec_tol(ref))
    g.close()
    # u_x = A cos(2 pi k0 x / n) on every line: E[k0] = A^2 / 4, nothing else
    n, A, k0 = 48, 0.3, 5
    x = np.arange(n)
    shape = (4, 6, n)
    rho = np.ones(shape)
    ux = np.broadcast_to(A * np.cos(2 * np.pi * k0 * x / n), shape)
    U = np.stack([rho, rho * ux, 0 * rho, 0 * rho, 2.5 + 0.5 * rho * ux * ux])
    dev = torch().from_numpy(U.copy()).to("cuda:0")
    g = hydro.Grid(dev, (1.0 / n,) * 3, 1.4, flags=hydro.FLAG_NO_TUNE)
    E = g.spectrum().cpu().numpy()
    np.testing.assert_allclose(E[k0], A * A / 4.0, rtol=1e-13)
    assert np.abs(np.delete(E, k0)).max() < 1e-15 * E[k0]
    g.close()


def test_spectrum_of_the_768_turbulence_state():
    """Full size, FP32: Parseval (sum E = <|u|^2>/2, the right side reduced
    by torch in FP64) and the initial field's band limit (its modes have
    |k| <= 8, so no energy beyond k_x = 8 but FP32 rounding)."""
    say("turbulence 768^3 state")
    U32 = ic.turbulence(768, dtype=np.float32).U
    t = torch()
    dev = t.from_numpy(U32).to("cuda:0")
    del U32
    g = hydro.Grid(dev, (1.0 / 768,) * 3, 5.0 / 3.0, flags=hydro.FLAG_NO_TUNE)
    say("turbulence 768^3 spectrum")
    E = g.spectrum().cpu().numpy()
    r = dev[0].double()
    ke2 = sum(((dev[c].double() / r) ** 2).mean() for c in (1, 2, 3)).item()
    np.testing.assert_allclose(E.sum(), 0.5 * ke2, rtol=1e-10)
    assert E[9:].sum() < 1e-10 * E.sum()
    assert E[1:9].min() > 0.0
    g.close()


# ------------------------------------------------------ shell spectrum

def _shell_tol(ref):
    """Both sides transform in FP64; each coefficient carries an error of a
    few eps log2 N of the field's norm, so every shell differs from the
    oracle by far less than 1e-12 of the total energy (rtol covers the
    large shells)."""
    return dict(rtol=1e-10, atol=1e-12 * float(np.abs(ref).sum()))


SHELL_SHAPES = [(8, 12, 16), (12, 18, 24), (36, 32, 48), (16, 16, 16), (1, 4, 8), (6, 1, 9),
                (3, 2, 1), (9, 27, 3), (4, 2, 1024), (2, 1024, 4), (1024, 2, 3), (24, 96, 256)]


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
@pytest.mark.parametrize("shape", SHELL_SHAPES)
def test_shell_spectrum_matches_oracle(prec, shape):
    say(f"shell spectrum prec={prec} shape={shape}")
    g, U, P = _state(shape, seed=31 + sum(shape), ng=2 if shape[2] % 2 else 0, prec=prec,
                     special=False)
    E = g.spectrum3d().cpu().numpy()
    ref = D.spectrum_shell(U)
    assert E.shape == ref.shape == (D.shell_count(shape),)
    np.testing.assert_allclose(E, ref, **_shell_tol(ref))
    nbytes, nb = g.spectrum3d_workspace()
    assert nb == len(ref)
    # fixed order: a second call into a used workspace gives the same bits
    work = torch().full((nbytes,), 0xA5, dtype=torch().uint8, device="cuda:0")
    np.testing.assert_array_equal(E, g.spectrum3d(work=work).cpu().numpy())
    np.testing.assert_array_equal(E, g.spectrum3d(work=work).cpu().numpy())
    g.close()


def test_shell_spectrum_single_mode_and_errors():
    shape = (12, 16, 24)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    A, k = 0.4, (5, -3, 2)
    wave = A * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz))
    rho = np.full(shape, 1.7)
    U = np.stack([rho, 0 * rho, rho * wave, 0 * rho, 2.5 + 0.5 * rho * wave * wave])
    dev = torch().from_numpy(U.copy()).to("cuda:0")
    g = hydro.Grid(dev, (1.0 / nx,) * 3, 1.4, flags=hydro.FLAG_NO_TUNE)
    say("shell spectrum single mode")
    E = g.spectrum3d().cpu().numpy()
    K = int(round(np.sqrt(25 + 9 + 4)))
    np.testing.assert_allclose(E[K], A * A / 4.0, rtol=1e-13)
    assert np.abs(np.delete(E, K)).max() < 1e-15 * E[K]
    nbytes, nb = g.spectrum3d_workspace()
    out = torch().empty(nb, dtype=torch().float64, device="cuda:0")
    work = torch().empty(nbytes, dtype=torch().uint8, device="cuda:0")
    wp, op = ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(out.data_ptr())
    for args in ((wp, nbytes - 1, op), (ctypes.c_void_p(work.data_ptr() + 8), nbytes - 8, op),
                 (wp, nbytes, ctypes.c_void_p(out.data_ptr() + 4)), (None, nbytes, op)):
        with pytest.raises(hydro.HydroError) as e:
            hydro.hydro_diag_spectrum3d(g.ctx, *args)
        assert e.value.status == hydro.HYDRO_EINVAL
    g.close()
    # an extent that is not 2^a 3^b
    P = ic.smooth_random((8, 10, 8), 3)
    g = hydro.Grid(torch().from_numpy(P.U.copy()).to("cuda:0"), P.dx, P.gamma,
                   flags=hydro.FLAG_NO_TUNE)
    with pytest.raises(hydro.HydroError) as e:
        g.spectrum3d_workspace()
    assert e.value.status == hydro.HYDRO_EINVAL
    g.close()


@pytest.mark.parametrize("prec", [hydro.FP32, hydro.FP64])
def test_shell_spectrum_reads_back_the_turbulence_initial_spectrum(prec):
    # closed form of the initial data (rho = 1, modes only on shells 1..8):
    # E[K] = vrms^2 K^(-5/3) / (2 sum_K' K'^(-5/3)); in FP32 the state's
    # rounding (relative 6e-8 per value) spreads ~1e-15 of the energy into
    # every other shell
    n = 96
    P = ic.turbulence(n)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    dev = torch().from_numpy(P.U.astype(dt)).to("cuda:0")
    g = hydro.Grid(dev, P.dx, P.gamma, flags=hydro.FLAG_NO_TUNE)
    say(f"shell spectrum turbulence {n}^3 prec={prec}")
    E = g.spectrum3d().cpu().numpy()
    vrms2 = 0.3 * 0.3 * (5.0 / 3.0)
    K = np.arange(1, 9)
    want = 0.5 * vrms2 * K ** (-5.0 / 3.0) / np.sum(K ** (-5.0 / 3.0))
    np.testing.assert_allclose(E[1:9], want, rtol=1e-10 if prec == hydro.FP64 else 1e-6)
    rest = np.concatenate([E[:1], E[9:]])
    assert rest.max() < (1e-25 if prec == hydro.FP64 else 1e-12) * E.sum()
    g.close()
