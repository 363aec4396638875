"""Pins of the exact Riemann solver (Toro 2009 ch. 4) used to check the oracle.

The solver is pinned by (i) the star states printed in Toro's Table 4.3,
(ii) the Rankine-Hugoniot conditions written as flux balances in the shock
frame, (iii) constancy of entropy and of the Riemann invariant across a
rarefaction, and (iv) exact mass/energy content of the cell averages.
"""
import math
import os

import numpy as np
import pytest

from oracle.exact_riemann import ExactRiemann, RiemannState

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toro_table_4_3.txt")


def _rows():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out.append((int(f[0]), [float(x) for x in f[1:]]))
    return out


@pytest.mark.parametrize("test,vals", _rows())
def test_star_state_matches_toro_table(test, vals):
    L = RiemannState(*vals[0:3])
    R = RiemannState(*vals[3:6])
    e = ExactRiemann(L, R, 1.4)
    got = [e.p_star, e.u_star, e.rho_star_L, e.rho_star_R]
    for g, want in zip(got, vals[6:10]):
        assert abs(g - want) <= 1e-5 * max(1.0, abs(want)) + 1e-5, (test, got)


def _flux(rho, u, p, g):
    E = p / (g - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)]), \
        np.array([rho, rho * u, E])


@pytest.mark.parametrize("test,vals", _rows())
def test_shocks_satisfy_rankine_hugoniot(test, vals):
    g = 1.4
    L = RiemannState(*vals[0:3])
    R = RiemannState(*vals[3:6])
    e = ExactRiemann(L, R, g)
    # across a shock of speed S: F(b) - F(a) = S (U(b) - U(a))
    if e.left_shock:
        Fa, Ua = _flux(L.rho, L.u, L.p, g)
        Fb, Ub = _flux(e.rho_star_L, e.u_star, e.p_star, g)
        np.testing.assert_allclose(Fb - Fa, e.SL * (Ub - Ua),
                                   rtol=1e-11, atol=1e-11 * np.abs(Fa).max())
    if e.right_shock:
        Fa, Ua = _flux(e.rho_star_R, e.u_star, e.p_star, g)
        Fb, Ub = _flux(R.rho, R.u, R.p, g)
        np.testing.assert_allclose(Fb - Fa, e.SR * (Ub - Ua),
                                   rtol=1e-11, atol=1e-11 * np.abs(Fa).max())


@pytest.mark.parametrize("test,vals", _rows())
def test_rarefactions_keep_entropy_and_invariant(test, vals):
    g = 1.4
    L = RiemannState(*vals[0:3])
    R = RiemannState(*vals[3:6])
    e = ExactRiemann(L, R, g)
    if not e.left_shock:
        # p / rho^g and u + 2c/(g-1) are constant through the left fan
        s0 = L.p / L.rho ** g
        J0 = L.u + 2 * math.sqrt(g * L.p / L.rho) / (g - 1)
        for xi in np.linspace(e.left_head, e.left_tail, 7):
            rho, u, p = e.sample(xi)
            assert abs(p / rho ** g - s0) <= 1e-12 * s0
            assert abs(u + 2 * math.sqrt(g * p / rho) / (g - 1) - J0) <= 1e-12 * abs(J0) + 1e-13
            # inside the fan the characteristic u - c passes through xi
            assert abs(u - math.sqrt(g * p / rho) - xi) <= 1e-12 * (1 + abs(xi))
        rho, u, p = e.sample(e.left_tail - 1e-12)
        assert abs(p - e.p_star) <= 1e-9 * e.p_star
    if not e.right_shock:
        s0 = R.p / R.rho ** g
        J0 = R.u - 2 * math.sqrt(g * R.p / R.rho) / (g - 1)
        for xi in np.linspace(e.right_tail, e.right_head, 7):
            rho, u, p = e.sample(xi)
            assert abs(p / rho ** g - s0) <= 1e-12 * s0
            assert abs(u - 2 * math.sqrt(g * p / rho) / (g - 1) - J0) <= 1e-12 * abs(J0) + 1e-13
            assert abs(u + math.sqrt(g * p / rho) - xi) <= 1e-12 * (1 + abs(xi))


def test_sod_wave_positions_at_t02():
    e = ExactRiemann(RiemannState(1, 0, 1), RiemannState(0.125, 0, 0.1), 1.4)
    t, x0 = 0.2, 0.5
    # rarefaction head moves at -c_L = -sqrt(1.4)
    assert abs(x0 + e.left_head * t - (0.5 - math.sqrt(1.4) * 0.2)) < 1e-15
    assert abs(x0 + e.left_head * t - 0.263357) < 1e-6
    assert abs(x0 + e.left_tail * t - 0.485945) < 1e-6
    assert abs(x0 + e.u_star * t - 0.685491) < 1e-6
    assert abs(x0 + e.SR * t - 0.850431) < 1e-6


def test_cell_averages_conserve_content():
    # the waves stay inside [0,1] until t = 0.2, so the exact mass, momentum
    # and energy in the box follow from the boundary fluxes alone
    e = ExactRiemann(RiemannState(1, 0, 1), RiemannState(0.125, 0, 0.1), 1.4)
    for n in (64, 1024):
        edges = np.linspace(0.0, 1.0, n + 1)
        avg = e.cell_averages(edges, 0.2, 0.5)
        tot = avg.sum(axis=0) / n
        assert abs(tot[0] - 0.5625) < 1e-13
        assert abs(tot[1] - 0.9 * 0.2) < 1e-13   # pressure push 1 - 0.1
        assert abs(tot[2] - 1.375) < 1e-13
