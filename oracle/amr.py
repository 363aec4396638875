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

* level_step: one step of a two-level hierarchy (one coarse grid, fine
  patches of half the cell width), the standard subcycled scheme with
  refluxing (Berger & Colella 1989), written for the split sweeps:
    1. the coarse grid takes one Strang step of dt; the flux of each sweep
       through every coarse face on the boundary of a fine patch is kept,
       times dt, in a coarse register;
    2. each fine patch takes two steps of dt/2 (sweep orders by the fine
       step counter).  Before substep s its ghost shell (g >= 2 layers) is
       prolonged from the coarse grid interpolated linearly in time,
       C_old + theta (C_new - C_old) with theta = s/2 (at theta = 0 the
       start-of-step state itself).  The whole stored box
       (interior and ghosts, outflow at its outer edge) is swept, so ghost
       cells move with each sweep and the next sweep sees advanced values;
       the interior depends only on cells within 2 of it per sweep, never on
       the box's outer edge.  The flux of each sweep through the fine faces
       on the patch boundary, averaged over the 2 x 2 fine faces of a coarse
       face (summed in (t2, t1) order: (0,0), (0,1), (1,0), (1,1), times
       1/4), times dt/2, adds to a fine register;
    3. restriction of every fine interior onto the coarse cells it covers;
    4. refluxing: the uncovered coarse cell across each coarse-fine face
       replaces the coarse flux by the fine one, U += (R_c - R_f) / dx on a
       patch's low side and U += (R_f - R_c) / dx on its high side, applied
       for axis x, y, z and, per axis, the low sides of all patches before
       the high sides.
  With a periodic coarse grid the coarse total after the step equals the
  uncovered coarse cells' total before it plus the fine interiors' totals
  (each fine cell weighs 1/8), to rounding.
"""
import numpy as np

import oracle as _core

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
    """Monotonised-central slope from one-sided differences a, b: zero unless
    a and b are both strictly positive or both strictly negative, else
    sign(a) min(2|a|, 2|b|, |a+b|/2) (van Leer 1977), the sweeps' reading
    (a sign test, not a product that can underflow)."""
    with np.errstate(invalid="ignore"):
        m = np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))
    same = ((a > 0.0) & (b > 0.0)) | ((a < 0.0) & (b < 0.0))
    return np.where(same, np.copysign(m, a), 0.0)


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


def _face_slices(axis, o, n, side, coarse, g=0):
    """Index of the coarse-fine faces of a patch along `axis` in a face-flux
    array: coarse (o, n: coarse offset and fine interior extents) or fine
    (inset g).  Returns the (z, y, x) slices."""
    sl = [None, None, None]          # x, y, z
    for a in range(3):
        if a == axis:
            if coarse:
                f = o[a] + (0 if side == 0 else n[a] // 2)
            else:
                f = g + (0 if side == 0 else n[a])
            sl[a] = slice(f, f + 1)
        elif coarse:
            sl[a] = slice(o[a], o[a] + n[a] // 2)
        else:
            sl[a] = slice(g, g + n[a])
    return (slice(None), sl[2], sl[1], sl[0])


def _coarse_face_mean(Ff, axis):
    """(5, ..) fine face fluxes on one patch side -> the mean over the 2 x 2
    fine faces of each coarse face, summed in (t2, t1) order."""
    A = np.squeeze(Ff, axis=3 - axis)            # (5, t2, t1)
    s = A[:, 0::2, 0::2] + A[:, 0::2, 1::2]
    s = s + A[:, 1::2, 0::2]
    s = s + A[:, 1::2, 1::2]
    return 0.25 * s


def check_level(shape_c, shapes_f, offsets, g):
    """Raises ValueError unless the patches satisfy level_step's placement
    rules (shapes in (z, y, x) order, fine shapes stored)."""
    if g < 2:
        raise ValueError("fine patches need at least 2 ghost layers")
    m = (g + 1) // 2 + 1
    boxes = []
    for sf, o in zip(shapes_f, offsets):
        n = [sf[2 - a] - 2 * g for a in range(3)]
        lo, hi = [], []
        for a in range(3):
            N = shape_c[2 - a]
            if N < 2 or n[a] < 2 or n[a] % 2:
                raise ValueError("every axis needs > 1 coarse cell and even fine extents")
            if o[a] < m or o[a] + n[a] // 2 + m > N:
                raise ValueError("fine patch too close to the coarse edge")
            lo.append(o[a])
            hi.append(o[a] + n[a] // 2)
        boxes.append((lo, hi))
    for i in range(len(boxes)):
        for j in range(i):
            (al, ah), (bl, bh) = boxes[i], boxes[j]
            if not any(bl[a] >= ah[a] + 1 or al[a] >= bh[a] + 1 for a in range(3)):
                raise ValueError("fine patches must be a coarse cell apart")


def level_step(C, fines, offsets, g, dt, gamma, dx, grav=(0.0, 0.0, 0.0),
               bc=(PERIODIC,) * 6, step_c=0, step_f=0, reflux=True):
    """One subcycled step of a coarse interior C (5, Nz, Ny, Nx) with cell
    widths dx = (dx, dy, dz) and fine stored patches fines[i] (5, nz + 2g,
    ny + 2g, nx + 2g) whose interior cell (0,0,0) is the first child of
    coarse cell offsets[i] = (ox, oy, oz).  Every axis needs more than one
    coarse cell; patches (even interior extents, g >= 2) must sit at least
    ceil(g/2) + 1 coarse cells inside C and be separated by at least one
    coarse cell along some axis.  Returns (C, fines) after the step; the
    inputs are not modified."""
    check_level(C.shape[1:], [F.shape[1:] for F in fines], offsets, g)
    C = np.array(C, dtype=np.float64)
    fines = [np.array(F, dtype=np.float64) for F in fines]
    dx = tuple(float(v) for v in dx)
    dxf = tuple(v / 2 for v in dx)
    shape_c = C.shape[1:]
    active = [shape_c[2 - a] > 1 for a in range(3)]
    order = lambda k: (0, 1, 2) if k % 2 == 0 else (2, 1, 0)
    ns = [tuple(F.shape[3 - a] - 2 * g for a in range(3)) for F in fines]
    pc = _core.make_params(shape_c, dx, gamma, bc=bc, grav=grav)
    regc = {}
    regf = {}
    Cold = C.copy()
    # 1. coarse step
    for d in order(step_c):
        if not active[d]:
            continue
        Fc = _core.sweep_flux(pc, C, dt, d)
        for i, o in enumerate(offsets):
            for side in (0, 1):
                face = Fc[_face_slices(d, o, ns[i], side, True)]
                regc[i, d, side] = dt * np.squeeze(face, axis=3 - d)
    # 2. two fine substeps
    h = 0.5 * dt
    for s in (0, 1):
        theta = 0.5 * s
        Ct = Cold if theta == 0.0 else Cold + theta * (C - Cold)
        for i, o in enumerate(offsets):
            fines[i] = prolong(Ct, 0, fines[i], g, o, ghosts_only=True)
        for d in order(step_f + s):
            if not active[d]:
                continue
            for i in range(len(fines)):
                pf = _core.make_params(fines[i].shape[1:], dxf, gamma,
                                       bc=(OUTFLOW,) * 6, grav=grav)
                Ff = _core.sweep_flux(pf, fines[i], h, d)
                for side in (0, 1):
                    face = Ff[_face_slices(d, None, ns[i], side, False, g)]
                    r = h * _coarse_face_mean(face, d)
                    key = (i, d, side)
                    regf[key] = r if key not in regf else regf[key] + r
    # 3. restriction
    for i, o in enumerate(offsets):
        C = restrict(fines[i], g, C, 0, o)
    # 4. refluxing
    if reflux:
        for d in range(3):
            if not active[d]:
                continue
            for side in (0, 1):
                for i, o in enumerate(offsets):
                    n = ns[i]
                    sl = [None, None, None]
                    for a in range(3):
                        if a == d:
                            c = o[a] - 1 if side == 0 else o[a] + n[a] // 2
                            sl[a] = slice(c, c + 1)
                        else:
                            sl[a] = slice(o[a], o[a] + n[a] // 2)
                    idx = (slice(None), sl[2], sl[1], sl[0])
                    delta = (regc[i, d, side] - regf[i, d, side] if side == 0
                             else regf[i, d, side] - regc[i, d, side])
                    C[idx] = C[idx] + np.expand_dims(delta / dx[d], axis=3 - d)
    return C, fines
