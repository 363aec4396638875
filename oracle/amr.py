"""FP64 oracle of the AMR operators around the batched patches.

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product package.
It shares no code with the HIP path.

The paper's runs use adaptive mesh refinement around the hydrodynamics (its
description of the codes' capabilities) without fixing the operators; these
are the standard conservative ones for a refinement ratio of 2, written out
plainly with numpy on stored patch arrays (5, nz + 2 ng, ny + 2 ng, nx + 2 ng)
of (rho, mx, my, mz, E):

* fill_ghosts: the stored ghost layers from the interior, axis by axis
  (x, then y, then z, each over the full extent of the axes already filled):
  periodic wraps, outflow copies the edge cell, reflect mirrors (ghost -k
  copies cell k - 1) with the normal momentum negated.

* restrict: each coarse cell covered by a fine patch becomes the mean of its
  2 x 2 x 2 fine children, summed in the fixed order (dz, dy, dx) =
  (0,0,0), (0,0,1), (0,1,0), (0,1,1), (1,0,0), (1,0,1), (1,1,0), (1,1,1)
  and scaled by 1/8.

* prolong: fine cell (I, J, K) (fine interior indices; negative or past the
  end for ghosts) lies in coarse cell (ox + floor(I/2), oy + floor(J/2),
  oz + floor(K/2)), offset s = -1/4 (even index) or +1/4 (odd) of a coarse
  width along each axis, and takes
      U_f = ((U_c + s_x D_x) + s_y D_y) + s_z D_z
  with D the monotonised-central slope of U_c along each axis from its two
  coarse neighbours: D = 0 unless a = U_c - U_(c-1) and b = U_(c+1) - U_c
  have a positive product, else sign(a) min(min(2|a|, 2|b|), |a + b| / 2).
  The eight children of a coarse cell average to it (the offsets cancel),
  and linear data are reproduced exactly.
"""
import numpy as np

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2


def fill_ghosts(S, ng, bc):
    """Stored patch S (5, nz+2ng, ny+2ng, nx+2ng) with its ghost layers
    filled from the interior; bc = (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi)."""
    S = np.array(S, dtype=np.float64)
    if ng == 0:
        return S
    for axis in range(3):               # x, y, z
        arr_axis = 3 - axis             # array axes are (var, z, y, x)
        lo, hi = bc[2 * axis], bc[2 * axis + 1]
        n = S.shape[arr_axis] - 2 * ng
        inner = [slice(None)] * 4
        inner[arr_axis] = slice(ng, ng + n)
        core = S[tuple(inner)]
        mode = {PERIODIC: "wrap", OUTFLOW: "edge", REFLECT: "symmetric"}
        pad_lo = np.pad(core, [(ng, 0) if a == arr_axis else (0, 0) for a in range(4)],
                        mode=mode[lo])
        pad_hi = np.pad(core, [(0, ng) if a == arr_axis else (0, 0) for a in range(4)],
                        mode=mode[hi])
        sl_lo = [slice(None)] * 4
        sl_lo[arr_axis] = slice(0, ng)
        sl_hi = [slice(None)] * 4
        sl_hi[arr_axis] = slice(ng + n, 2 * ng + n)
        glo = pad_lo[tuple(sl_lo)].copy()
        ghi = pad_hi[tuple([slice(None)] * arr_axis + [slice(n, n + ng)])].copy()
        if lo == REFLECT:
            glo[1 + axis] *= -1.0
        if hi == REFLECT:
            ghi[1 + axis] *= -1.0
        S[tuple(sl_lo)] = glo
        S[tuple(sl_hi)] = ghi
    return S


def restrict(F, ng_f, C, ng_c, o):
    """Coarse stored patch C with the cells covered by the fine patch F
    (stored, ng_f ghosts; even interior extents) replaced by the means of
    their children; o = (ox, oy, oz), the coarse cell of fine cell (0,0,0)."""
    F = np.asarray(F, dtype=np.float64)
    C = np.array(C, dtype=np.float64)
    nzf, nyf, nxf = (s - 2 * ng_f for s in F.shape[1:])
    f = F[:, ng_f:ng_f + nzf, ng_f:ng_f + nyf, ng_f:ng_f + nxf]
    acc = None
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                child = f[:, dz::2, dy::2, dx::2]
                acc = child.copy() if acc is None else acc + child
    ox, oy, oz = o
    C[:, ng_c + oz:ng_c + oz + nzf // 2, ng_c + oy:ng_c + oy + nyf // 2,
      ng_c + ox:ng_c + ox + nxf // 2] = acc * 0.125
    return C


def mc(a, b):
    """Monotonised-central slope from one-sided differences a, b."""
    with np.errstate(invalid="ignore"):
        m = np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))
    return np.where(a * b > 0.0, np.copysign(m, a), 0.0)


def prolong(C, ng_c, F, ng_f, o, ghosts_only=False):
    """Fine stored patch F with its interior cells (or only its ghost cells)
    replaced by the limited linear prolongation of the coarse stored patch C
    (whose cells, ghosts included, must cover the parents and their
    neighbours); o = (ox, oy, oz)."""
    C = np.asarray(C, dtype=np.float64)
    F = np.array(F, dtype=np.float64)
    nzf, nyf, nxf = (s - 2 * ng_f for s in F.shape[1:])
    ox, oy, oz = o
    K, J, I = np.meshgrid(np.arange(-ng_f, nzf + ng_f), np.arange(-ng_f, nyf + ng_f),
                          np.arange(-ng_f, nxf + ng_f), indexing="ij")
    interior = (I >= 0) & (I < nxf) & (J >= 0) & (J < nyf) & (K >= 0) & (K < nzf)
    sel = ~interior if ghosts_only else interior
    I, J, K = I[sel], J[sel], K[sel]
    ci = ng_c + ox + np.floor_divide(I, 2)
    cj = ng_c + oy + np.floor_divide(J, 2)
    ck = ng_c + oz + np.floor_divide(K, 2)
    sx = np.where(I % 2 == 0, -0.25, 0.25)
    sy = np.where(J % 2 == 0, -0.25, 0.25)
    sz = np.where(K % 2 == 0, -0.25, 0.25)
    out = np.empty((5, I.size))
    for v in range(5):
        c = C[v][ck, cj, ci]
        dx = mc(c - C[v][ck, cj, ci - 1], C[v][ck, cj, ci + 1] - c)
        dy = mc(c - C[v][ck, cj - 1, ci], C[v][ck, cj + 1, ci] - c)
        dz = mc(c - C[v][ck - 1, cj, ci], C[v][ck + 1, cj, ci] - c)
        out[v] = ((c + sx * dx) + sy * dy) + sz * dz
    Fv = F.reshape(5, -1)
    flat = ((K + ng_f) * (nyf + 2 * ng_f) + (J + ng_f)) * (nxf + 2 * ng_f) + (I + ng_f)
    Fv[:, flat] = out
    return F
