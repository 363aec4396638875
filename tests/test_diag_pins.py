"""Pins of the diagnostics oracle (CPU): closed forms, exact bin placements
and invariants that a wrong formula, axis or bin index would break."""
import numpy as np
import pytest

import hydro_ic as ic
from oracle import diagnostics as D

GAMMA = 5.0 / 3.0


def cons(rho, vx, vy, vz, p, gamma=GAMMA):
    """Conserved state from primitives (arrays of one shape)."""
    rho, vx, vy, vz, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64)
                                               for a in (rho, vx, vy, vz, p)))
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, E])


def at_rest(rho):
    return cons(rho, 0.0, 0.0, 0.0, 1.0)


# ---------------------------------------------------------------- PDF

@pytest.mark.parametrize("nbins,lo,hi", [(8, 0.0, 1.0), (100, -3.0, 5.0), (1, 2.0, 3.0)])
def test_pdf_bin_centres_one_count_each(nbins, lo, hi):
    w = (hi - lo) / nbins
    rho = lo + (np.arange(nbins) + 0.5) * w
    c = D.pdf(at_rest(rho.reshape(1, 1, nbins)), GAMMA, D.RHO, lo, hi, nbins)
    assert c[0] == 0 and c[-1] == 0
    np.testing.assert_array_equal(c[1:-1], np.ones(nbins, np.int64))


def test_pdf_edges_and_out_of_range():
    # power-of-two bin width: every edge lo + i w is exact, so a value on an
    # edge opens bin i; hi itself and beyond overflow; below lo and NaN
    # underflow
    lo, hi, nb = 0.0, 2.0, 8
    edges = lo + np.arange(nb) * (hi - lo) / nb
    extra = np.array([hi, 7.0, np.nextafter(lo, -1.0), -5.0, np.nan])
    rho = np.concatenate([edges, extra]).reshape(1, 1, -1)
    c = D.pdf(at_rest(rho), GAMMA, D.RHO, lo, hi, nb)
    np.testing.assert_array_equal(c[1:-1], np.ones(nb, np.int64))
    assert c[nb + 1] == 2 and c[0] == 3


def test_pdf_total_is_the_cell_count():
    rng = np.random.default_rng(5)
    U = cons(rng.uniform(0.5, 2.0, (6, 7, 9)), rng.normal(size=(6, 7, 9)),
             rng.normal(size=(6, 7, 9)), rng.normal(size=(6, 7, 9)),
             rng.uniform(0.5, 3.0, (6, 7, 9)))
    for q in D.QUANTITIES:
        c = D.pdf(U, GAMMA, q, 0.0, 2.0, 13)
        assert c.sum() == U[0].size


def test_pdf_pressure_speed_mach_of_known_states():
    # rho = 2, p = 2 / gamma, so c = sqrt(gamma p / rho) = 1; |v| = 0.5 (a
    # 3-4-5 direction); every quantity lands in the bin centred on its value
    rho, p = 2.0, 2.0 / GAMMA
    U = cons(np.full((3, 4, 5), rho), 0.3, 0.0, 0.4, p)
    nb = 10
    for q, val in ((D.PRESSURE, p), (D.SPEED, 0.5), (D.MACH, 0.5), (D.RHO, rho)):
        lo = val - 0.05 * nb / 2 - 0.025   # bin 5 is centred on val
        c = D.pdf(U, GAMMA, q, lo, lo + 0.05 * nb, nb)
        assert c[1 + 5] == U[0].size, (q, c)


def test_pressure_of_the_kh_initial_state():
    # the KH layer is built with p = 2.5 everywhere
    spec = ic.batch_specs(1, seed=2, sizes=(16,))[0]
    U = ic.kh_patch(spec, GAMMA)
    p = D.quantity(U, GAMMA, D.PRESSURE)
    np.testing.assert_allclose(p, 2.5, rtol=1e-14)


# ------------------------------------------------------------ profiles

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_profile_follows_the_axis(axis):
    nx, ny, nz = 5, 7, 3
    idx = np.indices((nz, ny, nx))[2 - axis]          # index along the axis
    U = at_rest(1.0 + idx)
    prof = D.profile(U, GAMMA, axis, 0.0, 1.0)
    n = (nx, ny, nz)[axis]
    assert prof.shape == (n, 5)
    np.testing.assert_allclose(prof[:, 0], 1.0 + np.arange(n), rtol=1e-15)
    for other in {0, 1, 2} - {axis}:
        m = (nx, ny, nz)[other]
        np.testing.assert_allclose(D.profile(U, GAMMA, other, 0.0, 1.0)[:, 0],
                                   np.full(m, 1.0 + (n - 1) / 2.0), rtol=1e-15)


def test_profile_pressure_and_kinetic_energy_of_uniform_flow():
    rho, v, p = 1.5, (0.2, -0.4, 0.1), 0.7
    U = cons(np.full((4, 3, 2), rho), *v, p)
    prof = D.profile(U, GAMMA, 2, 1.0, 2.0)
    ke = 0.5 * rho * sum(c * c for c in v)
    np.testing.assert_allclose(prof[:, 1], p, rtol=1e-14)
    np.testing.assert_allclose(prof[:, 2], ke, rtol=1e-14)
    np.testing.assert_allclose(prof[:, 3], 0.5, rtol=1e-15)      # f of 1.5 in [1, 2]
    np.testing.assert_allclose(prof[:, 4], 0.25, rtol=1e-15)


def test_mixing_width_of_a_sharp_interface_is_zero():
    n = 8
    z = np.arange(n).reshape(n, 1, 1)
    U = at_rest(np.broadcast_to(np.where(z < n // 2, 2.0, 1.0), (n, 3, 4)))
    W, theta = D.mixing(D.profile(U, GAMMA, 2, 1.0, 2.0), 1.0 / n)
    assert W == 0.0 and theta == 0.0


@pytest.mark.parametrize("n", [4, 10, 33])
def test_mixing_width_of_a_linear_ramp(n):
    # f_i = (i + 1/2) / n on slab i, uniform inside the slab:
    # W = 4 dz sum f (1 - f) = 4 dz (n/6 + 1/(12 n)), Theta = 1
    dz = 1.0 / n
    f = (np.arange(n) + 0.5) / n
    U = at_rest(np.broadcast_to((1.0 + f).reshape(n, 1, 1), (n, 2, 3)))
    W, theta = D.mixing(D.profile(U, GAMMA, 2, 1.0, 2.0), dz)
    np.testing.assert_allclose(W, 4.0 * dz * (n / 6.0 + 1.0 / (12.0 * n)), rtol=1e-13)
    np.testing.assert_allclose(theta, 1.0, rtol=1e-13)


def test_unmixed_slabs_have_zero_mixedness():
    # every slab half heavy, half light: <f> = 1/2 gives W = n dz = 1, but
    # f (1 - f) = 0 in every cell, so Theta = 0
    n = 6
    x = np.arange(4).reshape(1, 1, 4)
    U = at_rest(np.broadcast_to(np.where(x < 2, 2.0, 1.0), (n, 3, 4)))
    W, theta = D.mixing(D.profile(U, GAMMA, 2, 1.0, 2.0), 1.0 / n)
    np.testing.assert_allclose(W, 1.0, rtol=1e-15)
    assert theta == 0.0


# ------------------------------------------------------------ spectrum

def _line_state(ux, uy=0.0, uz=0.0, rho=1.0, shape=(3, 4)):
    """A state whose every x-line carries the velocity profile (ux, uy, uz)."""
    nx = np.broadcast_shapes(np.shape(ux), np.shape(uy), np.shape(uz), np.shape(rho))[-1]
    full = shape + (nx,)
    return cons(*(np.broadcast_to(a, full) for a in (rho, ux, uy, uz, 1.0)))


@pytest.mark.parametrize("n", [12, 16, 24, 48])
def test_spectrum_single_mode(n):
    # u_x = A cos(2 pi k0 x / n + phi): all the energy A^2 / 4 sits at k0
    A, k0, phi = 0.7, 3, 0.4
    x = np.arange(n)
    E = D.spectrum_x(_line_state(A * np.cos(2 * np.pi * k0 * x / n + phi)))
    assert E.shape == (n // 2 + 1,)
    np.testing.assert_allclose(E[k0], A * A / 4.0, rtol=1e-13)
    rest = np.delete(E, k0)
    assert np.all(np.abs(rest) < 1e-28)


def test_spectrum_uniform_flow_and_nyquist():
    n = 16
    E = D.spectrum_x(_line_state(np.full(n, 0.3), 0.4, -1.2))
    np.testing.assert_allclose(E[0], 0.5 * (0.09 + 0.16 + 1.44), rtol=1e-14)
    assert np.all(np.abs(E[1:]) < 1e-28)
    alt = 0.5 * (-1.0) ** np.arange(n)          # the Nyquist mode
    E = D.spectrum_x(_line_state(0.0, alt))
    np.testing.assert_allclose(E[n // 2], 0.5 * 0.25, rtol=1e-14)
    assert np.all(np.abs(E[:n // 2]) < 1e-28)


def test_spectrum_parseval_and_velocity_not_momentum():
    # sum_k E[k] = <|u|^2> / 2 with u = m / rho; a density that varies along
    # the line must not change the spectrum of a given velocity
    rng = np.random.default_rng(9)
    n = 24
    u = rng.normal(size=(3, 5, 6, n))
    rho = rng.uniform(0.5, 2.0, size=(5, 6, n))
    U = cons(rho, u[0], u[1], u[2], 1.0)
    E = D.spectrum_x(U)
    np.testing.assert_allclose(E.sum(), 0.5 * (u * u).sum(axis=0).mean(), rtol=1e-13)
    np.testing.assert_allclose(E, D.spectrum_x(cons(1.0, u[0], u[1], u[2], 1.0)), rtol=1e-12,
                               atol=1e-15)


# ------------------------------------------------------ shell spectrum

def _field(u, rho=1.0):
    """Conserved state of velocity field u (3, nz, ny, nx) and density rho."""
    return cons(rho, u[0], u[1], u[2], 1.0)


def _grid(shape):
    nz, ny, nx = shape
    return np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")


def test_shell_index_is_the_nearest_integer_of_the_norm():
    # K - 1/2 <= |k| < K + 1/2, i.e. (2K - 1)^2 <= 4 m2 < (2K + 1)^2, in
    # integers, for every |k|^2 of wavevectors up to 512 per axis
    m2 = np.arange(0, 3 * 512 * 512 + 1, dtype=np.int64)
    K = D.shell_index(m2)
    lo_ok = (K == 0) | ((2 * K - 1) ** 2 <= 4 * m2)     # K - 1/2 <= 0 needs no check
    assert np.all(lo_ok) and np.all(4 * m2 < (2 * K + 1) ** 2)
    assert D.shell_count((768, 768, 768)) == 666      # round(sqrt(3) 384) = 665
    assert D.shell_count((1, 1, 16)) == 9 and D.shell_count((6, 4, 12)) == 8  # corner (6, 2, 3): |k| = 7


@pytest.mark.parametrize("shape,k", [((8, 12, 16), (3, 2, 1)), ((6, 9, 12), (5, -4, 2)),
                                     ((16, 16, 16), (0, 7, -7)), ((4, 6, 10), (2, -2, 1))])
def test_shell_spectrum_single_mode(shape, k):
    # u = A e cos(2 pi k . x / n + phi) with e a unit vector: all the energy
    # A^2 / 4 in the shell round(|k|) (no component at a Nyquist frequency)
    nz, ny, nx = shape
    kx, ky, kz = k
    z, y, x = _grid(shape)
    A, phi = 0.8, 0.3
    wave = A * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + phi)
    e = np.array([0.6, 0.0, -0.8])
    E = D.spectrum_shell(_field(e[:, None, None, None] * wave, rho=1.3))
    assert E.shape == (D.shell_count(shape),)
    K = int(round(np.sqrt(kx * kx + ky * ky + kz * kz)))
    np.testing.assert_allclose(E[K], A * A / 4.0, rtol=1e-13)
    assert np.all(np.abs(np.delete(E, K)) < 1e-28)


def test_shell_spectrum_uniform_flow_and_nyquist_corner():
    shape = (6, 8, 10)
    E = D.spectrum_shell(_field(np.broadcast_to(np.array([0.3, -0.4, 1.2])[:, None, None, None],
                                                (3,) + shape)))
    np.testing.assert_allclose(E[0], 0.5 * (0.09 + 0.16 + 1.44), rtol=1e-14)
    assert np.all(np.abs(E[1:]) < 1e-28)
    # (-1)^(x+y+z): the corner wavevector (5, 4, 3), |k| = sqrt(50): shell 7,
    # and <u^2> = 1/4 for amplitude 1/2 (no cosine factor at Nyquist)
    z, y, x = _grid(shape)
    alt = 0.5 * (-1.0) ** (x + y + z)
    E = D.spectrum_shell(_field(np.stack([0 * alt, alt, 0 * alt])))
    assert E.shape == (8,)
    np.testing.assert_allclose(E[7], 0.5 * 0.25, rtol=1e-14)
    assert np.all(np.abs(E[:7]) < 1e-28)


def test_shell_spectrum_brute_force_dft():
    # the definition written out: a direct triple-sum DFT per wavevector,
    # signed wavenumbers and shells taken by integer comparisons
    rng = np.random.default_rng(21)
    shape = (3, 4, 6)
    nz, ny, nx = shape
    u = rng.normal(size=(3,) + shape)
    rho = rng.uniform(0.5, 2.0, size=shape)
    z, y, x = _grid(shape)
    nb = D.shell_count(shape)
    want = np.zeros(nb)
    for jz in range(nz):
        for jy in range(ny):
            for jx in range(nx):
                ph = np.exp(-2j * np.pi * (jx * x / nx + jy * y / ny + jz * z / nz))
                power = sum(abs(np.sum(u[c] * ph)) ** 2 for c in range(3))
                kvec = [j if 2 * j <= n else j - n for j, n in ((jx, nx), (jy, ny), (jz, nz))]
                m2 = sum(q * q for q in kvec)
                K = 0
                while not (4 * m2 < (2 * K + 1) ** 2):
                    K += 1
                want[K] += power
    want /= 2.0 * (nx * ny * nz) ** 2
    np.testing.assert_allclose(D.spectrum_shell(_field(u, rho)), want, rtol=1e-12, atol=1e-16)


def test_shell_spectrum_parseval_and_axis_permutation():
    # sum_K E[K] = <|u|^2> / 2; on a cube, swapping the x and z axes (and the
    # x and z velocity components) maps each wavevector to one of equal norm
    rng = np.random.default_rng(22)
    n = 12
    u = rng.normal(size=(3, n, n, n))
    rho = rng.uniform(0.5, 2.0, size=(n, n, n))
    E = D.spectrum_shell(cons(rho, u[0], u[1], u[2], 1.0))
    np.testing.assert_allclose(E.sum(), 0.5 * (u * u).sum(axis=0).mean(), rtol=1e-13)
    ut = np.stack([u[2], u[1], u[0]]).transpose(0, 3, 2, 1)
    Et = D.spectrum_shell(cons(rho.transpose(2, 1, 0), ut[0], ut[1], ut[2], 1.0))
    np.testing.assert_allclose(Et, E, rtol=1e-12, atol=1e-18)


def test_shell_spectrum_of_x_only_flow_is_the_x_spectrum():
    # a velocity that varies along x alone has its power on (kx, 0, 0),
    # shell |kx|: the shell spectrum equals the x-line spectrum
    rng = np.random.default_rng(23)
    nx = 16
    line = rng.normal(size=(3, nx))
    u = np.broadcast_to(line[:, None, None, :], (3, 4, 6, nx))
    E3 = D.spectrum_shell(_field(u))
    E1 = D.spectrum_x(_field(u))
    np.testing.assert_allclose(E3[:nx // 2 + 1], E1, rtol=1e-12, atol=1e-18)
    assert np.all(np.abs(E3[nx // 2 + 1:]) < 1e-28)


def test_shell_spectrum_reads_back_the_turbulence_initial_spectrum():
    # the turbulence initial data puts vrms^2 K^(-5/3) / sum_K' K'^(-5/3)
    # of <|v|^2> into each shell K = 1..8 (rho = 1): half of it is E[K]
    n, mach, gamma = 24, 0.3, 5.0 / 3.0
    P = ic.turbulence(n, mach=mach, gamma=gamma)
    E = D.spectrum_shell(P.U)
    vrms2 = mach * mach * gamma
    K = np.arange(1, 9)
    want = 0.5 * vrms2 * K ** (-5.0 / 3.0) / np.sum(K ** (-5.0 / 3.0))
    np.testing.assert_allclose(E[1:9], want, rtol=1e-10)
    assert abs(E[0]) < 1e-20 and np.all(np.abs(E[9:]) < 1e-20)
