"""Pins of the reactive-source oracle (CPU): the discrete closed form of the
first link, the Bateman solution as the substep count grows (first-order
convergence), exact mass conservation, the energy identity on a two-species
chain, the stiff limit, no burning at zero rate, and T = p / rho."""
import numpy as np
import pytest

from oracle import burn as B

GAMMA = 1.4


def state(rho, p, v=(0.0, 0.0, 0.0), shape=(2, 3, 4)):
    rho = np.full(shape, rho, dtype=np.float64)
    p = np.full(shape, p, dtype=np.float64)
    vx, vy, vz = (np.full(shape, c) for c in v)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, E])


def pure(M, shape=(2, 3, 4)):
    X = np.zeros((M,) + shape)
    X[0] = 1.0
    return X


def test_first_link_discrete_closed_form_and_temperature():
    # T = p / rho = 0.5 (with a flow: the kinetic energy must be removed);
    # k = A exp(-Ta / T); backward Euler gives X_0 = 1 / (1 + h k)^n exactly
    U = state(2.0, 1.0, v=(0.3, -0.2, 0.1))
    A, Ta, dt, n = [3.0, 1.0], [0.25, 0.1], 0.7, 5
    k0 = 3.0 * np.exp(-0.25 / 0.5)
    _, X = B.burn(U, pure(3), GAMMA, A, Ta, [1.0, 1.0], dt, n)
    np.testing.assert_allclose(X[0], (1.0 + dt / n * k0) ** (-n), rtol=1e-14)
    np.testing.assert_allclose(B.temperature(U, GAMMA), 0.5, rtol=1e-14)


def test_two_species_energy_release():
    # a -> b releasing q: E rises by rho q (X_a0 - X_a)
    U = state(1.5, 0.9)
    q = 2.5
    U2, X = B.burn(U, pure(2), GAMMA, [4.0], [0.0], [q], 0.3, 3)
    k, h = 4.0, 0.1
    Xa = (1.0 + h * k) ** -3
    np.testing.assert_allclose(X[0], Xa, rtol=1e-14)
    np.testing.assert_allclose(X[1], 1.0 - Xa, rtol=1e-14)
    np.testing.assert_allclose(U2[4] - U[4], 1.5 * q * (1.0 - Xa), rtol=1e-13)
    np.testing.assert_array_equal(U2[:4], U[:4])


@pytest.mark.parametrize("M", [3, 5, 13])
def test_backward_euler_converges_to_bateman_at_first_order(M):
    rng = np.random.default_rng(M)
    k = np.sort(rng.uniform(0.3, 3.0, M - 1))[::-1] * (1.0 + 0.01 * np.arange(M - 1))
    T = 1.0
    U = state(1.0, T, shape=(1, 1, 1))
    exact = B.bateman(1.0, k, 1.0)
    errs = []
    for n in (200, 400, 800):
        _, X = B.burn(U, pure(M, (1, 1, 1)), GAMMA, k, np.zeros(M - 1), np.zeros(M - 1), 1.0, n)
        errs.append(np.abs(X[:, 0, 0, 0] - exact).max())
    assert errs[0] < 5e-3
    # halving h halves the error (first order), to within a few per cent
    for a, b in zip(errs, errs[1:]):
        assert 1.9 < a / b < 2.1, errs


def test_mass_is_conserved_and_stiff_links_empty_at_once():
    rng = np.random.default_rng(3)
    M = 13
    X = rng.dirichlet(np.ones(M), size=(2, 3, 4)).transpose(3, 0, 1, 2)
    U = state(1.0, 2.0)
    A = 10.0 ** rng.uniform(-3, 8, M - 1)
    _, X2 = B.burn(U, X, GAMMA, A, np.zeros(M - 1), np.ones(M - 1), 1.0, 1)
    np.testing.assert_allclose(X2.sum(axis=0), X.sum(axis=0), rtol=1e-14)
    # one substep with h k_0 = 1e12: species 0 is gone
    A2 = np.full(M - 1, 1e12)
    _, X3 = B.burn(U, X, GAMMA, A2, np.zeros(M - 1), np.ones(M - 1), 1.0, 1)
    assert np.all(X3[0] < 1e-11)


def test_zero_rate_burns_nothing():
    rng = np.random.default_rng(4)
    X = rng.dirichlet(np.ones(4), size=(2, 3, 4)).transpose(3, 0, 1, 2)
    U = state(1.0, 1.0)
    U2, X2 = B.burn(U, X, GAMMA, np.zeros(3), np.ones(3), np.ones(3), 5.0, 4)
    np.testing.assert_array_equal(X2, X)
    np.testing.assert_array_equal(U2, U)


def test_three_species_energy_counts_the_mass_through_each_link():
    # a -> b (q0) -> c (q1): the energy is q0 times the mass that left a plus
    # q1 times the mass that reached c
    U = state(1.2, 1.0)
    q0, q1 = 0.7, 1.9
    U2, X = B.burn(U, pure(3), GAMMA, [2.0, 1.5], [0.0, 0.0], [q0, q1], 0.8, 4)
    np.testing.assert_allclose(U2[4] - U[4], 1.2 * (q0 * (1.0 - X[0]) + q1 * X[2]), rtol=1e-13)


def test_one_substep_solves_the_implicit_linear_system():
    # backward Euler: (I - h J) X' = X with J the chain's rate matrix,
    # solved here with a general dense solver
    rng = np.random.default_rng(8)
    M = 6
    k = 10.0 ** rng.uniform(-1, 3, M - 1)
    X = rng.dirichlet(np.ones(M))
    J = np.zeros((M, M))
    for i in range(M - 1):
        J[i, i] -= k[i]
        J[i + 1, i] += k[i]
    h = 0.37
    want = np.linalg.solve(np.eye(M) - h * J, X)
    U = state(1.0, 1.0, shape=(1, 1, 1))
    _, got = B.burn(U, X.reshape(M, 1, 1, 1), GAMMA, k, np.zeros(M - 1), np.zeros(M - 1), h, 1)
    np.testing.assert_allclose(got[:, 0, 0, 0], want, rtol=1e-13)
