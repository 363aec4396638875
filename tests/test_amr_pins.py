"""Pins of the AMR operators' oracle (CPU): ghost fills against numpy's pad
of the whole interior and against symmetry, restriction and prolongation
against linear data (closed forms), conservation (the children of a coarse
cell average back to it), and the limiter's bounds."""
import numpy as np
import pytest

from oracle import amr

P, O, R = amr.PERIODIC, amr.OUTFLOW, amr.REFLECT


def stored(U, ng):
    S = np.full((5,) + tuple(s + 2 * ng for s in U.shape[1:]), np.nan)
    S[:, ng:S.shape[1] - ng, ng:S.shape[2] - ng, ng:S.shape[3] - ng] = U
    return S


def rand_state(shape, seed):
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(5,) + shape)
    U[0] = rng.uniform(0.5, 2.0, shape)
    U[4] = rng.uniform(2.0, 4.0, shape)
    return U


@pytest.mark.parametrize("ng", [1, 2, 4])
def test_periodic_and_outflow_fill_equal_numpy_pad_of_the_interior(ng):
    U = rand_state((5, 6, 7), 1)
    for bc, mode in ((P, "wrap"), (O, "edge")):
        S = amr.fill_ghosts(stored(U, ng), ng, (bc,) * 6)
        want = np.pad(U, [(0, 0)] + [(ng, ng)] * 3, mode=mode)
        np.testing.assert_array_equal(S, want)


@pytest.mark.parametrize("ng", [1, 3])
def test_periodic_and_outflow_fill_by_index_formula(ng):
    # every stored cell (i, j, k), ghosts included, from the interior cell
    # the boundary maps it to, written out with Python loops: periodic
    # i -> i mod n, outflow i -> min(max(i, 0), n - 1), per axis
    U = rand_state((3, 4, 5), 4)
    nz, ny, nx = U.shape[1:]
    for bc in (P, O):
        S = amr.fill_ghosts(stored(U, ng), ng, (bc,) * 6)
        def src(i, n):
            return i % n if bc == P else min(max(i, 0), n - 1)
        for k in range(-ng, nz + ng):
            for j in range(-ng, ny + ng):
                for i in range(-ng, nx + ng):
                    want = U[:, src(k, nz), src(j, ny), src(i, nx)]
                    assert np.array_equal(S[:, k + ng, j + ng, i + ng], want), (bc, i, j, k)


def test_reflect_fill_is_a_mirror_with_the_normal_momentum_negated():
    ng = 3
    U = rand_state((6, 5, 7), 2)
    S = amr.fill_ghosts(stored(U, ng), ng, (R,) * 6)
    for axis in range(3):
        a = 3 - axis
        n = U.shape[a]
        for k in range(ng):
            g = np.take(S, ng - 1 - k, axis=a)      # ghost -(k+1)
            c = np.take(S, ng + k, axis=a)          # cell k
            gh = np.take(S, ng + n + k, axis=a)     # ghost n + k
            ch = np.take(S, ng + n - 1 - k, axis=a)  # cell n - 1 - k
            for v in range(5):
                sgn = -1.0 if v == 1 + axis else 1.0
                np.testing.assert_array_equal(g[v], sgn * c[v])
                np.testing.assert_array_equal(gh[v], sgn * ch[v])


def test_mixed_fill_does_not_depend_on_the_axis_order():
    # the per-axis maps are separable, so filling z, y, x in reverse order
    # with numpy's pad gives the same array (corners included)
    ng = 2
    U = rand_state((4, 5, 6), 3)
    bc = (P, P, O, R, R, O)
    S = amr.fill_ghosts(stored(U, ng), ng, bc)
    mode = {P: "wrap", O: "edge", R: "symmetric"}
    T = U.copy()
    for axis in (2, 1, 0):
        a = 3 - axis
        lo = np.pad(T, [(ng, 0) if i == a else (0, 0) for i in range(4)], mode=mode[bc[2 * axis]])
        hi = np.pad(T, [(0, ng) if i == a else (0, 0) for i in range(4)],
                    mode=mode[bc[2 * axis + 1]])
        glo = np.take(lo, range(ng), axis=a).copy()
        ghi = np.take(hi, range(T.shape[a], T.shape[a] + ng), axis=a).copy()
        if bc[2 * axis] == R:
            glo[1 + axis] *= -1.0
        if bc[2 * axis + 1] == R:
            ghi[1 + axis] *= -1.0
        T = np.concatenate([glo, T, ghi], axis=a)
    np.testing.assert_array_equal(S, T)


def linear(shape, ng, grad, h, origin):
    """Stored array of a linear field sampled at cell centres (all 5
    variables the same field plus a per-variable offset)."""
    nz, ny, nx = (s + 2 * ng for s in shape)
    z = origin[2] + (np.arange(nz) - ng + 0.5) * h
    y = origin[1] + (np.arange(ny) - ng + 0.5) * h
    x = origin[0] + (np.arange(nx) - ng + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    f = grad[0] * X + grad[1] * Y + grad[2] * Z
    return np.stack([f + 3.0 + v for v in range(5)])


def test_restrict_linear_data_gives_coarse_centre_values_and_conserves():
    g = (0.3, -0.7, 1.1)
    F = linear((4, 6, 8), 2, g, 0.5, (1.0, 0.5, 2.0))        # fine cells of width 1/2
    C0 = np.zeros((5, 4 + 2, 5 + 2, 7 + 2))
    C = amr.restrict(F, 2, C0, 1, (1, 0, 2))
    # the covered coarse cells (width 1) are centred where a coarse linear
    # field with the same origin shift would be
    want = linear((2, 3, 4), 0, g, 1.0, (1.0, 0.5, 2.0))
    got = C[:, 1 + 2:1 + 2 + 2, 1:1 + 3, 1 + 1:1 + 1 + 4]
    np.testing.assert_allclose(got, want, rtol=1e-14)
    fi = F[:, 2:-2, 2:-2, 2:-2]
    np.testing.assert_allclose(got.sum(axis=(1, 2, 3)) * 8, fi.sum(axis=(1, 2, 3)), rtol=1e-14)


def test_prolong_reproduces_linear_data():
    g = (0.4, 0.9, -0.6)
    C = linear((6, 7, 8), 2, g, 1.0, (0.0, 0.0, 0.0))
    o = (2, 1, 2)                      # fine cell 0 is the first child of coarse (2, 1, 2)
    F0 = np.zeros((5, 4 + 4, 6 + 4, 4 + 4))
    F = amr.prolong(C, 2, F0, 2, o)
    # fine cells of width 1/2 starting at the low corner of coarse cell o
    want = linear((4, 6, 4), 0, g, 0.5, (2.0, 1.0, 2.0))
    np.testing.assert_allclose(F[:, 2:-2, 2:-2, 2:-2], want, rtol=1e-14)
    # ghosts only: the fine ghost shell from the same field, interior untouched
    G = amr.prolong(C, 2, F0, 2, o, ghosts_only=True)
    assert np.all(G[:, 2:-2, 2:-2, 2:-2] == 0.0)
    wantg = linear((4, 6, 4), 2, g, 0.5, (2.0, 1.0, 2.0))
    mask = np.ones(G.shape[1:], bool)
    mask[2:-2, 2:-2, 2:-2] = False
    np.testing.assert_allclose(G[:, mask], wantg[:, mask], rtol=1e-14)


def test_restrict_of_prolong_is_the_identity_and_no_new_extrema():
    U = rand_state((6, 6, 6), 4)
    C = amr.fill_ghosts(stored(U, 2), 2, (P,) * 6)
    o = (1, 2, 1)
    F = amr.prolong(C, 2, np.zeros((5, 8, 8, 8)), 0, o)        # 8^3 fine, no ghosts
    back = amr.restrict(F, 0, C, 2, o)
    np.testing.assert_allclose(back, C, rtol=1e-14, atol=1e-14)
    # every child lies within its parent's neighbourhood range (MC limiting)
    for v in range(5):
        for k in range(8):
            for j in range(8):
                for i in range(8):
                    ck, cj, ci = 2 + o[2] + k // 2, 2 + o[1] + j // 2, 2 + o[0] + i // 2
                    nb = C[v, ck - 1:ck + 2, cj - 1:cj + 2, ci - 1:ci + 2]
                    assert nb.min() - 1e-12 <= F[v, k, j, i] <= nb.max() + 1e-12


def test_prolong_of_a_jump_keeps_flat_regions_flat():
    C = np.ones((5, 8, 8, 8))
    C[:, :, :, 4:] = 2.0                                      # jump along x
    F = amr.prolong(C, 2, np.zeros((5, 4, 4, 8)), 0, (0, 1, 1))
    # coarse x-cells 0..3 with interior index <= 1 (stored 2..3) sit on flat
    # ground: their children equal the coarse value exactly
    np.testing.assert_array_equal(F[:, :, :, :2], 1.0)


def test_limiter_is_a_sign_test_not_a_product():
    # two one-sided differences of one strict sign whose product underflows
    # keep the limited slope min(2|a|, 2|b|, |a+b|/2); opposite signs or a
    # zero give none (van Leer's limiter; the sweeps read it the same way)
    a = np.array([1e-200, -1e-200, 1e-200, 0.0, 3.0])
    b = np.array([3e-200, -1e-200, -1e-200, 1.0, 1.0])
    assert np.all(a * b == np.array([0.0, 0.0, -0.0, 0.0, 3.0]))   # the products underflow
    np.testing.assert_array_equal(amr.mc(a, b),
                                  np.array([2e-200, -1e-200, 0.0, 0.0, 2.0]))
