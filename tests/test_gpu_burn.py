"""The reactive-source step on the GPU against the oracle: compositions and
energy on ragged grids with stored ghost layers (left untouched), FP64 and
FP32 states, species counts 2 to 20, substep counts 1 to 64, stiff and slow
links; the discrete closed form of a two-species chain; conservation at
full KH size; and the argument errors."""
import ctypes

import numpy as np
import pytest

import hydro_ic as ic
from gpu_util import say, torch
from oracle import burn as B
from paper_1510_05061_amd import hydro

pytestmark = pytest.mark.gpu


def _network(M, seed):
    """Links from slow to stiff over the zone temperatures of the test
    states (T = p / rho of order 1): prefactors 10^-1 .. 10^6, activation
    temperatures 0 .. 3, energy releases 0.1 .. 2."""
    rng = np.random.default_rng(seed)
    A = 10.0 ** rng.uniform(-1, 6, M - 1)
    Ta = rng.uniform(0.0, 3.0, M - 1)
    q = rng.uniform(0.1, 2.0, M - 1)
    return A, Ta, q


def _setup(shape, M, seed, prec, ng):
    P = ic.smooth_random(shape, seed, gamma=1.4, mach=0.5)
    rng = np.random.default_rng(seed + 100)
    X = rng.dirichlet(np.ones(M), size=shape).transpose(3, 0, 1, 2)
    dt = np.float64 if prec == hydro.FP64 else np.float32
    U = P.U.astype(dt)
    X = X.astype(dt)

    def padded(a):
        if not ng:
            return np.ascontiguousarray(a)
        full = np.full((a.shape[0],) + tuple(s + 2 * ng for s in shape), np.nan, dtype=dt)
        full[:, ng:-ng, ng:-ng, ng:-ng] = a
        return full

    t = torch()
    Ud = t.from_numpy(padded(U)).to("cuda:0")
    Xd = t.from_numpy(padded(X)).to("cuda:0")
    g = hydro.Grid(Ud, P.dx, P.gamma, ng=ng, flags=hydro.FLAG_NO_TUNE)
    return g, Ud, Xd, U.astype(np.float64), X.astype(np.float64), P


def _interior(a, ng):
    a = a.double().cpu().numpy()
    return a[:, ng:-ng, ng:-ng, ng:-ng] if ng else a


@pytest.mark.parametrize("prec", [hydro.FP64, hydro.FP32])
@pytest.mark.parametrize("M,nsub", [(2, 1), (3, 7), (13, 64), (20, 5)])
def test_burn_matches_oracle(prec, M, nsub):
    ng = 2 if M % 2 else 0
    say(f"burn prec={prec} M={M} nsub={nsub} ng={ng}")
    g, Ud, Xd, U, X, P = _setup((9, 13, 11), M, seed=20 + M, prec=prec, ng=ng)
    A, Ta, q = _network(M, seed=M)
    dt = 0.05
    before_u = Ud.clone()
    before_x = Xd.clone()
    g.burn(Xd, A, Ta, q, dt, nsub)
    Uref, Xref = B.burn(U, X, P.gamma, A, Ta, q, dt, nsub)
    gotU, gotX = _interior(Ud, ng), _interior(Xd, ng)
    if prec == hydro.FP64:
        # every step matches the oracle's operations but for the reciprocal
        # multiplies (one rounding each per substep) and the library exp
        np.testing.assert_allclose(gotX, Xref, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(gotU[4], Uref[4], rtol=1e-12)
    else:
        # FP64 arithmetic, then one rounding to FP32 on store: the oracle's
        # value rounded to FP32, within one FP32 ulp (two FP64 values 1e-14
        # apart can round to neighbouring FP32 values)
        tol = 2.0 ** -22
        np.testing.assert_allclose(gotX, Xref.astype(np.float32), rtol=tol, atol=1e-38)
        np.testing.assert_allclose(gotU[4], Uref[4].astype(np.float32), rtol=tol)
    np.testing.assert_array_equal(gotU[:4], _interior(before_u, ng)[:4])
    if ng:   # ghost layers untouched (NaN stays NaN)
        mask = np.ones(Ud.shape[1:], bool)
        mask[ng:-ng, ng:-ng, ng:-ng] = False
        assert np.isnan(Ud.cpu().numpy()[:, mask]).all() and np.isnan(Xd.cpu().numpy()[:, mask]).all()
    assert before_x.shape == Xd.shape
    g.close()


def test_two_species_discrete_closed_form():
    # X_a = X_a0 / (1 + h k)^n with k = A exp(-Ta / T), T = p / rho; E rises
    # by rho q (X_a0 - X_a)
    say("burn closed form")
    shape = (4, 5, 6)
    rho, p = 1.25, 0.8
    U = np.stack([np.full(shape, rho), np.zeros(shape), np.zeros(shape), np.zeros(shape),
                  np.full(shape, p / 0.4)])
    X = np.stack([np.full(shape, 0.9), np.full(shape, 0.1)])
    t = torch()
    Ud, Xd = t.from_numpy(U.copy()).to("cuda:0"), t.from_numpy(X.copy()).to("cuda:0")
    g = hydro.Grid(Ud, (0.1, 0.1, 0.1), 1.4, flags=hydro.FLAG_NO_TUNE)
    A, Ta, q, dt, n = 7.0, 0.3, 1.7, 0.2, 9
    g.burn(Xd, [A], [Ta], [q], dt, n)
    k = A * np.exp(-Ta / (p / rho))
    xa = 0.9 * (1.0 + dt / n * k) ** (-n)
    np.testing.assert_allclose(Xd[0].cpu().numpy(), xa, rtol=1e-13)
    np.testing.assert_allclose(Xd[1].cpu().numpy(), 1.0 - xa, rtol=1e-13)
    np.testing.assert_allclose(Ud[4].cpu().numpy(), p / 0.4 + rho * q * (0.9 - xa), rtol=1e-13)
    g.close()


def test_burn_full_kh_grid_conserves_and_burns_the_first_link_exactly():
    """KH 256^3 FP32 with 13 species (all species 0), 32 substeps: the sum
    of the fractions stays 1 (to FP32 rounding) and species 0 follows its
    discrete closed form at every zone's own temperature."""
    say("burn kh256")
    P = ic.kh(256)
    t = torch()
    Ud = t.from_numpy(P.U.astype(np.float32)).to("cuda:0")
    M = 13
    Xd = t.zeros((M,) + tuple(Ud.shape[1:]), dtype=t.float32, device="cuda:0")
    Xd[0] = 1.0
    g = hydro.Grid(Ud, P.dx, P.gamma, flags=hydro.FLAG_NO_TUNE)
    A, Ta, q = _network(M, seed=99)
    dt, n = 0.01, 32
    r = Ud[0].double()
    m2 = Ud[1].double() ** 2 + Ud[2].double() ** 2 + Ud[3].double() ** 2
    T = ((P.gamma - 1.0) * (Ud[4].double() - 0.5 * m2 / r)) / r
    g.burn(Xd, A, Ta, q, dt, n)
    s = Xd.double().sum(dim=0)
    assert (s - 1.0).abs().max().item() < 16 * 2.0 ** -24
    x0 = (1.0 + dt / n * A[0] * t.exp(-Ta[0] / T)) ** (-n)
    assert ((Xd[0].double() - x0).abs() / x0).max().item() < 2.0 ** -22
    g.close()


def test_burn_argument_errors():
    g, Ud, Xd, U, X, P = _setup((4, 4, 4), 3, seed=30, prec=hydro.FP64, ng=0)
    ptr, nbytes = ctypes.c_void_p(Xd.data_ptr()), Xd.numel() * Xd.element_size()
    A, Ta, q = _network(3, seed=1)
    good = hydro.make_network(A, Ta, q)
    bad_n1 = hydro.make_network([], [], [])
    cases = [(bad_n1, 0.1, 1, nbytes), (good, 0.1, 0, nbytes), (good, float("nan"), 1, nbytes),
             (good, -1.0, 1, nbytes), (good, 0.1, 1, nbytes - 8)]
    neg = hydro.make_network([-1.0, 1.0], Ta, q)
    cases.append((neg, 0.1, 1, nbytes))
    big = hydro.make_network(A, Ta, q)
    big.nspec = 21
    cases.append((big, 0.1, 1, nbytes))
    for net, dt, nsub, nb in cases:
        with pytest.raises(hydro.HydroError) as e:
            hydro.hydro_burn(g.ctx, ptr, nb, net, dt, nsub)
        assert e.value.status == hydro.HYDRO_EINVAL
    g.close()
