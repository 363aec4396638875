"""Pins of the seeded input generators (shared by the oracle and the HIP
path): determinism, the stated structure of each workload, and the
turbulence spectrum's defining properties."""
import math

import numpy as np
import pytest

import hydro_ic as ic


def test_generators_are_deterministic():
    a = ic.kh(shape=(8, 16, 12), seed=1).U
    b = ic.kh(shape=(8, 16, 12), seed=1).U
    c = ic.kh(shape=(8, 16, 12), seed=2).U
    np.testing.assert_array_equal(a, b)
    assert np.abs(a - c).max() > 0
    np.testing.assert_array_equal(ic.rt(8, 8, 16).U, ic.rt(8, 8, 16).U)
    np.testing.assert_array_equal(ic.turbulence(24).U, ic.turbulence(24).U)


def _prim(P):
    U = P.U
    rho = U[0]
    v = U[1:4] / rho
    p = (P.gamma - 1) * (U[4] - 0.5 * rho * (v ** 2).sum(0))
    return rho, v, p


def test_kh_layer_structure():
    P = ic.kh(shape=(4, 32, 8), seed=1)
    rho, v, p = _prim(P)
    y = (np.arange(32) + 0.5) / 32
    inner = np.abs(y - 0.5) < 0.25
    assert np.all(rho[:, inner] == 2.0) and np.all(rho[:, ~inner] == 1.0)
    np.testing.assert_allclose(v[0][:, inner], 0.5, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[0][:, ~inner], -0.5, rtol=0, atol=1e-15)
    assert np.abs(v[1]).max() <= 0.01 and np.abs(v[1]).max() > 0.009
    assert not np.any(P.U[3])
    np.testing.assert_allclose(p, 2.5, rtol=1e-14)
    assert P.gamma == 5.0 / 3.0 and P.bc == (ic.PERIODIC,) * 6


def test_rt_is_hydrostatic_with_walls():
    P = ic.rt(nx=8, ny=8, nz=32)
    rho, v, p = _prim(P)
    z = (np.arange(32) + 0.5) / 32
    assert np.all(rho[z > 0.5] == 2.0) and np.all(rho[z < 0.5] == 1.0)
    dpdz = np.diff(p[:, 0, 0]) / (1 / 32)
    rho_face = 0.5 * (rho[1:, 0, 0] + rho[:-1, 0, 0])
    np.testing.assert_allclose(dpdz, -0.1 * rho_face, rtol=1e-9)
    assert P.bc[4:] == (ic.REFLECT, ic.REFLECT) and P.grav == (0.0, 0.0, -0.1)
    assert np.abs(v[2]).max() <= 0.01 and not np.any(P.U[1]) and not np.any(P.U[2])
    assert P.dx == (0.5 / 8, 0.5 / 8, 1.0 / 32)


def test_batch_specs():
    specs = ic.batch_specs(4096, seed=3)
    n = np.array([s.n for s in specs])
    assert set(n) == {16, 32, 48, 64}
    for k in (16, 32, 48, 64):
        assert abs((n == k).mean() - 0.25) < 0.03
    sh = np.array([s.shear for s in specs])
    ra = np.array([s.ratio for s in specs])
    assert sh.min() >= 0.1 and sh.max() <= 1.0 and ra.min() >= 1.0 and ra.max() <= 4.0
    # each patch regenerates on its own
    again = ic.batch_specs(4096, seed=3)
    np.testing.assert_array_equal(ic.kh_patch(specs[17]), ic.kh_patch(again[17]))
    U = ic.kh_patch(specs[5])
    assert U.shape == (5, specs[5].n, specs[5].n, specs[5].n)
    assert np.isclose(U[0].max(), specs[5].ratio)


def test_turbulence_modes_are_solenoidal_hermitian_and_follow_the_spectrum():
    A, (KX, KY, KZ), shell, active = ic.turbulence_modes(seed=4)
    assert active.sum() == 2552
    kdotA = KX * A[0] + KY * A[1] + KZ * A[2]
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    amag = np.sqrt((np.abs(A) ** 2).sum(0))
    assert np.all(np.abs(kdotA) <= 1e-12 * kmag * amag + 1e-300)
    # Hermitian symmetry a(-k) = conj(a(k)) makes the field real
    np.testing.assert_array_equal(A[:, ::-1, ::-1, ::-1], np.conj(A))
    assert not np.any(A[:, ~active])
    E = np.array([(np.abs(A[:, shell == K]) ** 2).sum() for K in range(1, 9)])
    slope = np.polyfit(np.log(np.arange(1, 9)), np.log(E), 1)[0]
    assert abs(slope + 5.0 / 3.0) < 0.05
    assert abs(np.sum(np.abs(A) ** 2) - 1.0) < 1e-13


def test_turbulence_field_mach_and_mean():
    n = 40
    P = ic.turbulence(n, slab=16)
    rho, v, p = _prim(P)
    assert np.all(rho == 1.0)
    np.testing.assert_allclose(p, 1.0, rtol=1e-12)
    vrms = math.sqrt((v ** 2).sum(0).mean())
    assert abs(vrms / math.sqrt(5.0 / 3.0) - 0.3) < 1e-12
    assert np.abs(v.mean(axis=(1, 2, 3))).max() < 1e-14
    # spectral divergence of the sampled field vanishes
    vh = [np.fft.fftn(v[c]) for c in range(3)]
    k = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    div = KX * vh[0] + KY * vh[1] + KZ * vh[2]
    assert np.abs(div).max() <= 1e-12 * np.abs(np.stack(vh)).max() * 8
    # slab construction equals the one-shot evaluation
    v2 = ic.turbulence_velocity(n)
    np.testing.assert_allclose(v, v2, rtol=0, atol=1e-15)


def test_sod_embedding_layout():
    P = ic.sod(64, axis=1, transverse=4)
    assert P.shape == (4, 64, 4)
    assert P.bc == (ic.PERIODIC, ic.PERIODIC, ic.OUTFLOW, ic.OUTFLOW,
                    ic.PERIODIC, ic.PERIODIC)
    assert np.all(P.U[0][:, :32] == 1.0) and np.all(P.U[0][:, 32:] == 0.125)
