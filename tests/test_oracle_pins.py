"""Pins of the FP64 CPU oracle against facts fixed outside it.

Each test checks the oracle against mathematics it does not contain:
the exact Riemann solution, discrete conservation laws, mirror symmetry,
reduction to an independent scalar advection scheme, the quasi-linear
Jacobian of the Euler flux obtained by complex-step differentiation,
closed-form limiter values, and the bitwise invariances the scheme has
by construction.  A dropped term, a wrong sign or index, or a transposed
component anywhere in the oracle breaks at least one of them.
"""
import math

import numpy as np
import pytest

import hydro_ic as ic
import oracle
from oracle.exact_riemann import ExactRiemann, RiemannState


def params_of(P, nthreads=0):
    return oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav,
                              nthreads=nthreads)


# --------------------------------------------------------------------------
# point-wise pieces
# --------------------------------------------------------------------------

@pytest.mark.parametrize("a,b,want", [
    (1.0, 2.0, 1.5),        # |a+b|/2 is the smallest
    (1.0, 10.0, 2.0),       # 2|a| is the smallest
    (10.0, 1.0, 2.0),       # 2|b| is the smallest
    (-1.0, -2.0, -1.5),
    (-3.0, -0.5, -1.0),
    (1.0, -1.0, 0.0),       # extremum
    (0.0, 5.0, 0.0),        # flat on one side
    (5.0, 0.0, 0.0),
    (-0.0, -1.0, 0.0),
    (2.0, 2.0, 2.0),        # smooth: central difference
])
def test_mc_limiter_closed_form(a, b, want):
    assert oracle.mc_slope(a, b) == want


def test_mc_limiter_symmetries():
    rng = np.random.default_rng(0)
    for a, b in rng.standard_normal((200, 2)):
        s = oracle.mc_slope(a, b)
        assert oracle.mc_slope(b, a) == s            # symmetric in a, b
        assert oracle.mc_slope(-a, -b) == -s          # odd
        if a * b > 0:
            assert abs(s) <= 2 * min(abs(a), abs(b))  # TVD region
            assert np.sign(s) == np.sign(a)


def _euler_flux_and_state(W, g):
    rho, u, v, w, p = W
    E = p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w)
    U = np.array([rho, rho * u, rho * v, rho * w, E])
    F = np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * w, u * (E + p)])
    return U, F


def _primitive_jacobian(W, g):
    """A(W) = (dU/dW)^-1 dF/dW by complex-step differentiation of the
    conservation law written in primitive variables."""
    h = 1e-30
    dU = np.zeros((5, 5))
    dF = np.zeros((5, 5))
    for j in range(5):
        Wc = np.array(W, dtype=complex)
        Wc[j] += 1j * h
        U, F = _euler_flux_and_state(Wc, g)
        dU[:, j] = U.imag / h
        dF[:, j] = F.imag / h
    return np.linalg.solve(dU, dF)


def test_hancock_matches_euler_jacobian():
    rng = np.random.default_rng(1)
    g = 1.4
    for _ in range(20):
        W = np.array([rng.uniform(0.5, 2), rng.normal(), rng.normal(),
                      rng.normal(), rng.uniform(0.5, 2)])
        D = rng.normal(size=5) * 0.1
        dtdx = rng.uniform(0.05, 0.5)
        Wm, Wp = oracle.hancock(W, D, dtdx, g)
        A = _primitive_jacobian(W, g)
        drift = 0.5 * dtdx * A @ D
        np.testing.assert_allclose(Wp - Wm, D, rtol=0, atol=1e-14)
        np.testing.assert_allclose(0.5 * (Wp + Wm), W - drift, rtol=0, atol=1e-14)
        # gravity: the half kick moves only the normal velocity of both faces
        Wm2, Wp2 = oracle.hancock(W, D, dtdx, g, half_dt_g=0.25, has_g=True)
        np.testing.assert_array_equal(np.delete(Wm2, 1), np.delete(Wm, 1))
        assert Wm2[1] == Wm[1] + 0.25 and Wp2[1] == Wp[1] + 0.25


def _ulp_close(a, b, n):
    a, b = np.asarray(a), np.asarray(b)
    tol = n * np.spacing(np.maximum(np.abs(a), np.abs(b)))
    return np.all(np.abs(a - b) <= tol + 1e-300)


def test_hllc_consistency():
    g = 1.4
    rng = np.random.default_rng(2)
    for _ in range(200):
        rho, p = rng.uniform(0.2, 3, size=2)
        c = math.sqrt(g * p / rho)
        t1, t2 = rng.normal(size=2)
        for u in (0.0, 1.5 * c, -1.5 * c, rng.uniform(-0.9, 0.9) * c):
            W = np.array([rho, u, t1, t2, p])
            _, F = _euler_flux_and_state(W, g)
            got = oracle.hllc(W, W, g)
            if u == 0.0 or abs(u) > c:
                assert _ulp_close(got, F, 1), (W, got, F)
            else:
                assert _ulp_close(got, F, 16) or np.allclose(got, F, rtol=4e-16 * 8, atol=1e-15)


def test_hllc_resolves_stationary_contact():
    g = 1.4
    WL = np.array([1.0, 0.0, 0.3, -0.2, 1.0])
    WR = np.array([0.25, 0.0, -0.7, 0.1, 1.0])
    F = oracle.hllc(WL, WR, g)
    assert F[0] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
    assert F[1] == 1.0


def test_hllc_mirror_antisymmetry():
    g = 1.4
    rng = np.random.default_rng(3)
    for _ in range(200):
        WL = np.array([rng.uniform(0.2, 3), rng.normal(), rng.normal(),
                       rng.normal(), rng.uniform(0.2, 3)])
        WR = np.array([rng.uniform(0.2, 3), rng.normal(), rng.normal(),
                       rng.normal(), rng.uniform(0.2, 3)])
        F = oracle.hllc(WL, WR, g)
        mL = WR * np.array([1, -1, 1, 1, 1])
        mR = WL * np.array([1, -1, 1, 1, 1])
        Fm = oracle.hllc(mL, mR, g)
        # mirrored problem: mass, transverse momenta and energy fluxes flip,
        # the normal momentum flux stays
        want = F * np.array([-1, 1, -1, -1, -1])
        np.testing.assert_allclose(Fm, want, rtol=1e-13, atol=1e-14)


def test_hllc_upwind_supersonic():
    g = 1.4
    WL = np.array([1.0, 5.0, 0.1, 0.2, 1.0])
    WR = np.array([0.5, 4.0, -0.1, 0.0, 0.3])
    _, FL = _euler_flux_and_state(WL, g)
    np.testing.assert_array_equal(oracle.hllc(WL, WR, g), FL)
    WL2 = WL * np.array([1, -1, 1, 1, 1])
    WR2 = WR * np.array([1, -1, 1, 1, 1])
    _, FR2 = _euler_flux_and_state(WR2, g)
    np.testing.assert_array_equal(oracle.hllc(WL2, WR2, g), FR2)


# --------------------------------------------------------------------------
# positivity fallback: a cell whose Hancock face state has rho <= 0 or
# p <= 0 is reconstructed with zero slopes (first order)
# --------------------------------------------------------------------------

def _pencil(U, axis):
    """The single pencil of a grid that is one cell wide across `axis`, as
    (5, n) in the sweep frame (rho, m_axis, m_t1, m_t2, E), transverse
    momenta in ascending axis order."""
    line = [0, 0, 0]
    line[2 - axis] = slice(None)
    V = U[(slice(None),) + tuple(line)]
    t = [a for a in range(3) if a != axis]
    return np.array([V[0], V[1 + axis], V[1 + t[0]], V[1 + t[1]], V[4]])


def _first_order_upwind_sweep(U1, dt, dx, gamma, g, left):
    """One sweep of a pencil (sweep frame) of supersonic flow when every cell
    is reconstructed with zero slopes: each face takes the physical Euler
    flux of its upwind cell (Davis speeds all of one sign make HLLC the
    upwind flux), with the normal velocity raised by the half kick dt g/2,
    followed by the time-centred gravity source.  Outflow ends copy the edge
    cells.  Returns the new pencil and the face fluxes (face i - 1/2 at
    index i)."""
    ext = np.concatenate([U1[:, :1], U1, U1[:, -1:]], axis=1)     # cells -1 .. n
    rho = ext[0]
    u, t1, t2 = ext[1] / rho, ext[2] / rho, ext[3] / rho
    p = (gamma - 1.0) * (ext[4] - 0.5 * rho * (u * u + t1 * t1 + t2 * t2))
    u = u + 0.5 * dt * g
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + t1 * t1 + t2 * t2)
    F = np.array([rho * u, rho * u * u + p, rho * u * t1, rho * u * t2, u * (E + p)])
    face = F[:, 1:] if left else F[:, :-1]
    new = U1 - dt / dx * (face[:, 1:] - face[:, :-1])
    new[1] += dt * g * (0.5 * (U1[0] + new[0]))
    new[4] += dt * g * (0.5 * (face[0, :-1] + face[0, 1:]))
    return new, face


@pytest.mark.parametrize("grav", [0.0, -40.0])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("kind", ["rho_left", "rho_right", "p_left", "p_right"])
def test_positivity_fallback_is_first_order_upwind(kind, axis, grav):
    # Cell k of the staircase 100 | 10 | 1 has the MC slope -18 (2|b|) and,
    # at Courant number 1/2 against the flow, a downstream-side face value
    # 10 - 9 (1 + 1/2) < 0 in the stepped field: it must fall back, and it is
    # the only cell with a nonzero slope, so the whole sweep becomes the
    # textbook first-order upwind scheme.
    P = ic.steep_supersonic(kind, axis=axis, grav=grav)
    n = P.meta["n"]
    dx = P.dx[axis]
    dt = 0.5 * dx / 20.0
    p = params_of(P)
    U = P.U.copy()
    F = oracle.sweep_flux(p, U, dt, axis)
    fb = oracle.sweep(p, P.U.copy(), dt, axis)
    assert fb == 1
    want, face = _first_order_upwind_sweep(_pencil(P.U, axis), dt, dx, P.gamma, grav,
                                           kind.endswith("_left"))
    got_face = _pencil(F, axis)
    for v in range(5):
        tol = 1e-14 * max(np.abs(face[v]).max(), 1e-300)
        assert np.abs(got_face[v] - face[v]).max() <= tol, (v, got_face[v], face[v])
    got = _pencil(U, axis)
    for v in range(5):
        tol = 1e-14 * max(np.abs(want[v]).max(), 1e-300)
        assert np.abs(got[v] - want[v]).max() <= tol, (v, got[v], want[v])
    assert n == got.shape[1]


@pytest.mark.parametrize("kind", ["rho_left", "p_right"])
def test_no_fallback_when_face_states_stay_positive(kind):
    # a gentler staircase (upstream plateau 20): cell k keeps its slope
    # (MC = |a+b|/2 = 9.5, face value 10 - 4.75 (1 + 1/2) > 0), so there is
    # no fallback and the sweep is not the first-order one
    P = ic.steep_supersonic(kind)
    U = P.U.copy()
    k, left = P.meta["k"], kind.endswith("_left")
    up = slice(0, k) if left else slice(k + 1, None)
    field = 0 if kind.startswith("rho") else 4
    W = U[:, 0, 0, :]
    if field == 0:
        rho_up = 20.0
        W[1, up] *= rho_up / W[0, up]
        W[4, up] = 1.0 / (P.gamma - 1.0) + 0.5 * W[1, up] ** 2 / rho_up
        W[0, up] = rho_up
    else:
        W[4, up] += (20.0 - 100.0) / (P.gamma - 1.0)
    dx = P.dx[0]
    dt = 0.5 * dx / 20.0
    p = params_of(P)
    V = U.copy()
    assert oracle.sweep(p, V, dt, 0) == 0
    want, _ = _first_order_upwind_sweep(_pencil(U, 0), dt, dx, P.gamma, 0.0, left)
    assert np.abs(_pencil(V, 0)[0] - want[0]).max() > 1e-3 * np.abs(want[0]).max()


def test_two_rarefactions_reach_fallback_and_stay_positive_and_symmetric():
    # rho = 1, p = 0.4, u = -10 | +10 (vacuum forms between the fans):
    # the near-vacuum centre drives Hancock face states negative; the run
    # falls back, keeps rho and p positive, and stays mirror symmetric
    P = ic.two_rarefactions(64)
    U = P.U.copy()
    t, steps, fb = oracle.run(params_of(P), U, 10 ** 6, t_end=P.t_end)
    assert abs(t - P.t_end) <= 1e-16 and fb > 0
    rho = U[0, 0, 0]
    m = U[1, 0, 0]
    E = U[4, 0, 0]
    p = (P.gamma - 1.0) * (E - 0.5 * m * m / rho)
    assert rho.min() > 0 and p.min() > 0
    assert np.abs(rho - rho[::-1]).max() <= 1e-13 * rho.max()
    assert np.abs(m + m[::-1]).max() <= 1e-13 * np.abs(m).max()
    assert np.abs(E - E[::-1]).max() <= 1e-13 * E.max()


# --------------------------------------------------------------------------
# Sod shock tube
# --------------------------------------------------------------------------

def _sod_run(n):
    P = ic.sod(n)
    U = P.U.copy()
    t, steps, fb = oracle.run(params_of(P), U, 10 ** 6, t_end=P.t_end)
    assert abs(t - 0.2) < 1e-15
    return P, U, steps, fb


def test_sod_discrete_invariants():
    n = 1024
    P = ic.sod(n)
    p = params_of(P)
    U = P.U.copy()
    t, step = 0.0, 0
    dx = 1.0 / n
    while t < 0.2:
        t, step, _ = oracle.run(p, U, 1, t_end=0.2, t=t, step_index=step)
        # the end cells never see the waves: boundary fluxes are (0, p, 0, 0, 0)
        assert abs(U[0].sum() * dx - 0.5625) <= 1e-14 * 0.5625
        assert abs(U[4].sum() * dx - 1.375) <= 1e-14 * 1.375
        assert abs(U[1].sum() * dx - 0.9 * t) <= 1e-14 * max(1.0, 0.9 * t)
        np.testing.assert_array_equal(U[:, 0, 0, 0], P.U[:, 0, 0, 0])
        np.testing.assert_array_equal(U[:, 0, 0, -1], P.U[:, 0, 0, -1])
    assert step > 500


def _exact_avgs(n):
    e = ExactRiemann(RiemannState(1, 0, 1), RiemannState(0.125, 0, 0.1), 1.4)
    return e, e.cell_averages(np.linspace(0, 1, n + 1), 0.2, 0.5)


def test_sod_converges_to_exact_solution():
    errs = {}
    for n in (256, 512, 1024):
        P, U, steps, fb = _sod_run(n)
        assert fb == 0
        e, avg = _exact_avgs(n)
        errs[n] = np.abs(U[0, 0, 0] - avg[:, 0]).mean()
    # first order at discontinuities; the L1 error must fall with resolution
    o1 = math.log2(errs[256] / errs[512])
    o2 = math.log2(errs[512] / errs[1024])
    assert errs[512] < errs[256] and errs[1024] < errs[512]
    assert o1 >= 0.5 and o2 >= 0.5, errs
    # absolute level at N = 1024 (a shock-capturing second-order scheme
    # smears each discontinuity over a few cells: O(dx * jump))
    assert errs[1024] < 1.0e-3, errs


def test_sod_plateaus_and_shock_position():
    n = 1024
    P, U, steps, fb = _sod_run(n)
    e, _ = _exact_avgs(n)
    x = (np.arange(n) + 0.5) / n
    rho = U[0, 0, 0]
    u = U[1, 0, 0] / rho
    p = 0.4 * (U[4, 0, 0] - 0.5 * U[1, 0, 0] ** 2 / rho)
    xt = 0.5 + e.left_tail * 0.2
    xc = 0.5 + e.u_star * 0.2
    xs = 0.5 + e.SR * 0.2
    away = 10.0 / n
    # the tail of the fan is a kink that a limited scheme rounds off over
    # more cells than a jump; keep 16 cells clear of it
    tail = 16.0 / n
    plateau = ((x > xt + tail) & (x < xc - away)) | ((x > xc + away) & (x < xs - away))
    assert plateau.sum() > 100
    np.testing.assert_allclose(p[plateau], e.p_star, rtol=1e-3)
    np.testing.assert_allclose(u[plateau], e.u_star, rtol=1e-3)
    # density jumps at the contact, which no scheme steepens: keep 16 cells
    # clear of it for the density plateaus
    left_star = (x > xt + tail) & (x < xc - tail)
    right_star = (x > xc + tail) & (x < xs - away)
    np.testing.assert_allclose(rho[left_star], e.rho_star_L, rtol=1e-3)
    np.testing.assert_allclose(rho[right_star], e.rho_star_R, rtol=2e-3)
    # shock: where density crosses the mid value between rho*_R and rho_R
    mid = 0.5 * (e.rho_star_R + 0.125)
    i = np.where((rho[:-1] > mid) & (rho[1:] <= mid))[0][-1]
    xshock = x[i] + (rho[i] - mid) / (rho[i] - rho[i + 1]) / n
    assert abs(xshock - xs) < 2.0 / n


# --------------------------------------------------------------------------
# invariants on 3D grids
# --------------------------------------------------------------------------

def test_conservation_on_periodic_grid():
    P = ic.kh(shape=(24, 32, 28), seed=5)
    p = params_of(P)
    U = P.U.copy()
    t0 = oracle.totals(p, U)
    oracle.run(p, U, 40)
    t1 = oracle.totals(p, U)
    absmass = [np.abs(P.U[v]).sum() * np.prod(P.dx) for v in range(5)]
    for v in range(5):
        assert abs(t1[v] - t0[v]) <= 1e-13 * max(1.0, absmass[v]), (v, t0, t1)


def test_totals_match_exact_sum():
    P = ic.smooth_random((6, 7, 9), seed=6, grav=(0.1, -0.2, 0.3))
    p = params_of(P)
    got = oracle.totals(p, P.U)
    vol = np.prod(P.dx)
    for v in range(5):
        assert got[v] == math.fsum((P.U[v] * vol).ravel())
    nz, ny, nx = P.shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * P.dx[2],
                          (np.arange(ny) + 0.5) * P.dx[1],
                          (np.arange(nx) + 0.5) * P.dx[0], indexing="ij")
    phi = -(0.1 * x - 0.2 * y + 0.3 * z)
    assert abs(got[5] - math.fsum(((P.U[4] + P.U[0] * phi) * vol).ravel())) < 1e-15


def test_mirror_symmetry_of_blast():
    n = 24
    P = ic.blast(n)
    p = params_of(P)
    U = P.U.copy()
    oracle.run(p, U, 20)
    scale = np.abs(U).max(axis=(1, 2, 3))
    for axis in range(3):
        arr_axis = 3 - axis            # array axis of physical axis
        M = np.flip(U, axis=arr_axis).copy()
        M[1 + axis] *= -1.0
        for v in range(5):
            assert np.abs(M[v] - U[v]).max() <= 1e-13 * scale[v], (axis, v)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_1d_embedded_in_3d_is_bitwise(axis):
    n = 256
    P1 = ic.sod(n)
    U1 = P1.U.copy()
    t1, s1, _ = oracle.run(params_of(P1), U1, 10 ** 6, t_end=0.2)
    P3 = ic.sod(n, axis=axis, transverse=4)
    U3 = P3.U.copy()
    t3, s3, _ = oracle.run(params_of(P3), U3, 10 ** 6, t_end=0.2)
    assert t1 == t3 and s1 == s3
    line = [slice(None)] * 4
    for a in range(3):
        line[3 - a] = slice(None) if a == axis else 0
    got = U3[tuple(line)]
    want = U1[:, 0, 0, :]
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1 + axis], want[1])
    np.testing.assert_array_equal(got[4], want[4])
    for a in range(3):
        if a != axis:
            assert not np.any(got[1 + a])
    # every transverse copy is the same
    for v in range(5):
        ref = np.expand_dims(got[v], axis=tuple(i for i in range(3) if i != 2 - axis))
        np.testing.assert_array_equal(U3[v], np.broadcast_to(ref, U3[v].shape))


def _scalar_muscl_hancock(rho, nu, steps):
    """Independent scalar scheme for rho_t + rho_x = 0 (speed 1, periodic):
    MC slopes, face value rho_i + (1 - nu) D_i / 2, upwind flux."""
    r = rho.copy()
    for _ in range(steps):
        a = r - np.roll(r, 1)
        b = np.roll(r, -1) - r
        same = ((a > 0) & (b > 0)) | ((a < 0) & (b < 0))
        D = np.where(same, np.sign(a) * np.minimum(np.minimum(2 * abs(a), 2 * abs(b)),
                                                   0.5 * abs(a + b)), 0.0)
        face = r + 0.5 * (1 - nu) * D
        r = r - nu * (face - np.roll(face, 1))
    return r


@pytest.mark.parametrize("kind", ["sine", "square"])
def test_reduces_to_scalar_advection(kind):
    n = 64
    P = ic.advected_profile(n, kind)
    p = params_of(P)
    U = P.U.copy()
    # u + c <= 1 + sqrt(1.4 / 0.5) < 2.7, so nu = 0.25 keeps the CFL number
    # of the sound waves below 0.7
    nu = 0.25
    dt = nu / n
    steps = 40
    for s in range(steps):
        oracle.step(p, U, dt, s)
    want = _scalar_muscl_hancock(P.U[0, 0, 0], nu, steps)
    assert np.abs(U[0, 0, 0] - want).max() <= 1e-13
    u = U[1, 0, 0] / U[0, 0, 0]
    pr = 0.4 * (U[4, 0, 0] - 0.5 * U[1, 0, 0] * u)
    assert np.abs(u - 1).max() < 1e-13 and np.abs(pr - 1).max() < 1e-13


def test_stationary_contact_is_exact():
    P = ic.stationary_contact(64)
    p = params_of(P)
    U = P.U.copy()
    oracle.run(p, U, 50)
    np.testing.assert_array_equal(U, P.U)


def test_second_order_on_smooth_flow():
    errs = []
    for n in (64, 128, 256):
        P = ic.advected_profile(n, "sine")
        p = params_of(P)
        U = P.U.copy()
        nu = 0.25                          # acoustic CFL number < 0.7
        dt = nu / n
        steps = int(round(1.0 / dt))       # one period
        for s in range(steps):
            oracle.step(p, U, dt, s)
        errs.append(np.abs(U[0, 0, 0] - P.U[0, 0, 0]).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.7, (errs, orders)


def test_gravity_energy_with_potential_is_conserved():
    P = ic.rt(nx=16, ny=16, nz=32, seed=7)
    p = params_of(P)
    U = P.U.copy()
    t0 = oracle.totals(p, U)
    _, _, fb = oracle.run(p, U, 100)
    t1 = oracle.totals(p, U)
    for v in (0, 1, 2, 5):
        assert abs(t1[v] - t0[v]) <= 1e-13 * max(1.0, abs(t0[v])), (v, t0, t1)
    # total energy alone is not conserved: the potential term matters
    assert abs(t1[4] - t0[4]) > 1e3 * 1e-13 * abs(t0[4])
    # with gravity along z the walls push on the fluid: mz changes
    assert abs(t1[3] - t0[3]) > 0


def test_uniform_gravity_matches_galilean_solution():
    # A uniform gravity g along a periodic axis is a uniform acceleration of
    # the frame: the advected density profile rho0(x - u0 t - g t^2/2) with
    # u = u0 + g t and uniform p is an exact solution.  The scheme must
    # converge to it at second order in rho, u and p (a source that is not
    # time-centred, or a missing half kick, drops u and p to first order).
    g, u0, T = 0.3, 0.5, 0.5
    errs = []
    for n in (64, 128, 256):
        P = ic.advected_profile(n, "sine", u0=u0)
        p = oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, (g, 0.0, 0.0))
        dt = 0.2 / n
        steps = int(round(T / dt))
        U = P.U.copy()
        for s in range(steps):
            oracle.step(p, U, dt, s)
        x = (np.arange(n) + 0.5) / n
        shift = u0 * T + 0.5 * g * T * T
        a = x - 0.5 / n - shift
        b = x + 0.5 / n - shift
        rho_ex = 1 + 0.5 * (np.cos(2 * math.pi * a) - np.cos(2 * math.pi * b)) / (2 * math.pi / n)
        rho = U[0, 0, 0]
        u = U[1, 0, 0] / rho
        pr = 0.4 * (U[4, 0, 0] - 0.5 * U[1, 0, 0] * u)
        errs.append((np.abs(rho - rho_ex).mean(), np.abs(u - (u0 + g * T)).mean(),
                     np.abs(pr - 1.0).mean()))
    for k in range(3):
        orders = [math.log2(errs[i][k] / errs[i + 1][k]) for i in range(2)]
        assert min(orders) >= 1.8, (k, errs, orders)
    assert errs[0][1] < 1e-5 and errs[0][2] < 1e-5


def test_hydrostatic_column_balances_gravity_source():
    # with zero slopes (uniform density), the mirror walls and half kick
    # keep a column with p = p0 + g rho z nearly at rest (first-order check
    # of the source sign: the wrong sign accelerates the fluid at O(g dt))
    n = 32
    g = -0.1
    z = (np.arange(n) + 0.5) / n
    rho = np.ones((n, 1, 1))
    pz = (2.5 + g * (z - 0.5)).reshape(n, 1, 1)
    zero = np.zeros_like(rho)
    U = ic.conserved(rho, zero, zero, zero, pz, 1.4)
    P = ic.Problem(U=U, dx=(1.0 / n,) * 3, gamma=1.4,
                   bc=(0, 0, 0, 0, ic.REFLECT, ic.REFLECT), grav=(0, 0, g))
    p = params_of(P)
    W = U.copy()
    oracle.run(p, W, 20)
    vz = W[3] / W[0]
    assert np.abs(vz).max() < 2e-3


@pytest.mark.parametrize("bc", [ic.PERIODIC, ic.OUTFLOW, ic.REFLECT])
def test_uniform_state_is_unchanged(bc):
    P = ic.uniform((5, 6, 7), bc=(bc,) * 6)
    p = params_of(P)
    U = P.U.copy()
    oracle.run(p, U, 6)
    np.testing.assert_array_equal(U, P.U)


def test_uniform_flow_on_periodic_grid_is_unchanged():
    P = ic.uniform((5, 6, 7), v=(0.3, -0.7, 1.9))
    p = params_of(P)
    U = P.U.copy()
    oracle.run(p, U, 6)
    np.testing.assert_array_equal(U, P.U)


# --------------------------------------------------------------------------
# dt, sweep order, error path
# --------------------------------------------------------------------------

def test_cfl_dt_definition():
    P = ic.smooth_random((5, 6, 7), seed=8)
    P.dx = (0.1, 0.2, 0.05)
    p = params_of(P)
    U = P.U
    rho = U[0]
    v = U[1:4] / rho
    pr = (P.gamma - 1) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
    c = np.sqrt(P.gamma * pr / rho)
    s = max(((np.abs(v[d]) + c) / P.dx[d]).max() for d in range(3))
    assert abs(oracle.cfl_dt(p, U) - 0.8 / s) <= 1e-15 * 0.8 / s
    # a flat axis (n = 1) takes no part
    Q = ic.smooth_random((1, 6, 7), seed=8)
    q = params_of(Q)
    U = Q.U
    rho = U[0]
    pr = (Q.gamma - 1) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
    c = np.sqrt(Q.gamma * pr / rho)
    s = max(((np.abs(U[1 + d] / rho) + c) / Q.dx[d]).max() for d in range(2))
    assert abs(oracle.cfl_dt(q, U) - 0.8 / s) <= 1e-15 * 0.8 / s


def test_strang_order_alternates():
    P = ic.smooth_random((6, 7, 8), seed=9)
    p = params_of(P)
    dt = 0.5 * oracle.cfl_dt(p, P.U)
    for step, order in ((0, (0, 1, 2)), (1, (2, 1, 0)), (6, (0, 1, 2)), (7, (2, 1, 0))):
        A = P.U.copy()
        oracle.step(p, A, dt, step)
        B = P.U.copy()
        for d in order:
            oracle.sweep(p, B, dt, d)
        np.testing.assert_array_equal(A, B)
    A = P.U.copy()
    oracle.step(p, A, dt, 0)
    B = P.U.copy()
    oracle.step(p, B, dt, 1)
    assert np.abs(A - B).max() > 0


def test_thread_count_does_not_change_results():
    P = ic.smooth_random((8, 9, 10), seed=10)
    A = P.U.copy()
    B = P.U.copy()
    oracle.run(params_of(P, nthreads=1), A, 3)
    oracle.run(params_of(P, nthreads=4), B, 3)
    np.testing.assert_array_equal(A, B)


def test_negative_pressure_is_an_error():
    P = ic.uniform((4, 4, 4))
    U = P.U.copy()
    U[4, 1, 2, 3] = 0.1 * U[4, 1, 2, 3] - 5.0
    with pytest.raises(oracle.OracleError):
        oracle.run(params_of(P), U, 1)


def test_invalid_parameters_are_rejected():
    P = ic.uniform((4, 4, 4), bc=(ic.PERIODIC, ic.OUTFLOW) + (ic.PERIODIC,) * 4)
    with pytest.raises(oracle.OracleError):
        oracle.step(params_of(P), P.U.copy(), 1e-3, 0)
    Q = ic.uniform((4, 4, 4))
    q = params_of(Q)
    q.gamma = 1.0
    with pytest.raises(oracle.OracleError):
        oracle.step(q, Q.U.copy(), 1e-3, 0)
