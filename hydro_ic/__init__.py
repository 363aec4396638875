"""Seeded synthetic initial data for the compressible-Euler zone update.

This module holds only the definitions of the initial states (and of the
patch lists of the batched workload).  It contains none of the scheme's
arithmetic and is the one module that both the FP64 oracle tests and the
HIP path consume.  Every array is float64 of shape (5, nz, ny, nx) in C order
holding the conserved variables (rho, mx, my, mz, E); an ideal gas with
E = p/(gamma-1) + rho |v|^2 / 2 states the initial data.

Workloads (all synthetic, seeded; the paper prints no data):
  sod            1D shock tube (Sod 1978), 1024 cells on [0,1], gamma 1.4,
                 outflow ends, run to t = 0.2.
  kh             3D periodic Kelvin-Helmholtz layer, unit cube, gamma 5/3,
                 seed 1.
  rt             3D Rayleigh-Taylor, [0,0.5]^2 x [0,1], gravity -0.1 along z,
                 reflecting z walls, gamma 1.4, seed 2.
  batch          uneven periodic KH patches (edges 16/32/48/64, 4 ghost
                 layers), gamma 5/3, seed 3.
  turbulence     3D periodic solenoidal random-phase field, shells 1..8 with
                 E(k) ~ k^-5/3, rms Mach 0.3, gamma 5/3, seed 4.
These are the chaotic-flow, instability and turbulence workloads of the
paper's section "Increasing computing power", and the suites of independent
runs of its capacity-computing argument.
"""
from dataclasses import dataclass, field
import math
from typing import Tuple

import numpy as np

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2


@dataclass
class Problem:
    U: np.ndarray                      # (5, nz, ny, nx) float64
    dx: Tuple[float, float, float]     # cell widths (x, y, z)
    gamma: float
    bc: Tuple[int, ...] = (PERIODIC,) * 6
    grav: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    cfl: float = 0.8
    t_end: float = 0.0                 # 0: no final time
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.U.shape[1:])

    @property
    def zones(self):
        return int(np.prod(self.U.shape[1:]))


def conserved(rho, vx, vy, vz, p, gamma):
    """Stack primitive fields into the conserved state (initial-data
    definition for an ideal gas)."""
    rho = np.asarray(rho, dtype=np.float64)
    U = np.empty((5,) + rho.shape)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return U


def centres(n, length=1.0):
    return (np.arange(n) + 0.5) * (length / n)


# --------------------------------------------------------------------------
# 1D and textbook cases
# --------------------------------------------------------------------------

def sod(n=1024, gamma=1.4, axis=0, transverse=1):
    """Sod shock tube along `axis`; interface at x = 0.5 (a cell face for even
    n).  transverse > 1 embeds it in a 3D grid with periodic transverse
    axes and equal cell widths."""
    x = centres(n)
    left = x < 0.5
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    dims = [transverse, transverse, transverse]
    dims[axis] = n
    if transverse == 1:
        dims = [1, 1, 1]
        dims[axis] = n
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    rho = np.broadcast_to(rho1.reshape(bshape), shape)
    p = np.broadcast_to(p1.reshape(bshape), shape)
    z = np.zeros(shape)
    U = conserved(rho, z, z, z, p, gamma)
    bc = [PERIODIC] * 6
    bc[2 * axis] = OUTFLOW
    bc[2 * axis + 1] = OUTFLOW
    dx = 1.0 / n
    return Problem(U=np.ascontiguousarray(U), dx=(dx, dx, dx), gamma=gamma,
                   bc=tuple(bc), cfl=0.8, t_end=0.2, name="sod",
                   meta={"axis": axis, "n": n})


def advected_profile(n=64, kind="sine", gamma=1.4, u0=1.0, p0=1.0):
    """Uniform velocity u0 and pressure p0 carrying a density profile along x
    on a periodic [0,1]: 'sine' rho = 1 + 0.5 sin(2 pi x); 'square' rho = 2 on
    [0.25, 0.75), 1 elsewhere."""
    x = centres(n)
    if kind == "sine":
        rho = 1.0 + 0.5 * np.sin(2.0 * math.pi * x)
    elif kind == "square":
        rho = np.where((x >= 0.25) & (x < 0.75), 2.0, 1.0)
    else:
        raise ValueError(kind)
    rho = rho.reshape(1, 1, n)
    one = np.ones_like(rho)
    U = conserved(rho, u0 * one, 0 * one, 0 * one, p0 * one, gamma)
    return Problem(U=U, dx=(1.0 / n,) * 3, gamma=gamma, name=f"advect_{kind}")


def _embed_along(profile_fields, axis, n, transverse):
    """Fields given as 1D arrays of n cells along `axis`, repeated over a
    (transverse, transverse) cross-section: returns the grid shape (nz, ny,
    nx) and the broadcast fields."""
    dims = [transverse] * 3
    dims[axis] = n
    shape = (dims[2], dims[1], dims[0])
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    return shape, [np.broadcast_to(np.asarray(f, dtype=np.float64).reshape(bshape), shape)
                   for f in profile_fields]


def steep_supersonic(kind, n=16, k=7, axis=0, transverse=1, gamma=1.4, speed=20.0,
                     grav=0.0):
    """A supersonic flow along `axis` (|u| = speed, above every sound speed)
    carrying a three-level staircase in one field: 100 upstream of cell k,
    10 in cell k, 1 downstream ('rho_*': density with p = 1; 'p_*': pressure
    with rho = 1).  '*_left' flows towards low indices with the staircase
    falling towards high indices; '*_right' is its mirror image.  Only cell
    k has a nonzero limited slope, and its Hancock face state on the side
    away from the upstream plateau has a negative density or pressure.
    Outflow ends along the axis, periodic transverse axes, equal cell widths
    1/n; `grav` is the gravity along the axis."""
    i = np.arange(n)
    left = kind.endswith("_left")
    if kind not in ("rho_left", "rho_right", "p_left", "p_right"):
        raise ValueError(kind)
    up = (i < k) if left else (i > k)
    stair = np.where(up, 100.0, np.where(i == k, 10.0, 1.0))
    one = np.ones(n)
    rho, p = (stair, one) if kind.startswith("rho") else (one, stair)
    u = (-speed if left else speed) * one
    shape, (rho, u, p) = _embed_along((rho, u, p), axis, n, transverse)
    z = np.zeros(shape)
    vel = [z, z, z]
    vel[axis] = u
    U = conserved(rho, vel[0], vel[1], vel[2], p, gamma)
    bc = [PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = OUTFLOW
    g = [0.0, 0.0, 0.0]
    g[axis] = grav
    return Problem(U=np.ascontiguousarray(U), dx=(1.0 / n,) * 3, gamma=gamma, bc=tuple(bc),
                   grav=tuple(g), name=f"steep_{kind}", meta={"axis": axis, "k": k, "n": n})


def two_rarefactions(n=64, speed=10.0, gamma=1.4, axis=0, transverse=1):
    """Two strong rarefactions moving apart from x = 0.5 (rho = 1, p = 0.4,
    u = -speed | +speed; Toro's test 2 has speed 2): the near-vacuum centre
    drives Hancock face states non-positive.  Outflow ends, t_end = 0.02."""
    x = centres(n)
    u1 = np.where(x < 0.5, -speed, speed)
    shape, (rho, u, p) = _embed_along((np.ones(n), u1, 0.4 * np.ones(n)), axis, n, transverse)
    z = np.zeros(shape)
    vel = [z, z, z]
    vel[axis] = u
    U = conserved(rho, vel[0], vel[1], vel[2], p, gamma)
    bc = [PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = OUTFLOW
    return Problem(U=np.ascontiguousarray(U), dx=(1.0 / n,) * 3, gamma=gamma, bc=tuple(bc),
                   t_end=0.02, name="two_rarefactions", meta={"axis": axis, "n": n})


def stationary_contact(n=64, gamma=1.4, bc=OUTFLOW):
    """u = 0, uniform p = 1, density 1 | 0.25 at x = 0.5."""
    x = centres(n)
    rho = np.where(x < 0.5, 1.0, 0.25).reshape(1, 1, n)
    one = np.ones_like(rho)
    U = conserved(rho, 0 * one, 0 * one, 0 * one, one, gamma)
    return Problem(U=U, dx=(1.0 / n,) * 3, gamma=gamma,
                   bc=(bc, bc, PERIODIC, PERIODIC, PERIODIC, PERIODIC),
                   name="stationary_contact")


def uniform(shape, rho=1.3, v=(0.0, 0.0, 0.0), p=0.7, gamma=1.4,
            bc=(PERIODIC,) * 6):
    nz, ny, nx = shape
    one = np.ones(shape)
    U = conserved(rho * one, v[0] * one, v[1] * one, v[2] * one, p * one, gamma)
    return Problem(U=U, dx=(1.0 / nx, 1.0 / ny, 1.0 / nz), gamma=gamma, bc=bc,
                   name="uniform")


def blast(n=32, gamma=1.4, bc=(PERIODIC,) * 6, amp=10.0, radius=0.2):
    """Centred spherical overpressure on the unit cube at rest (mirror
    symmetric about every mid-plane)."""
    x = centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    p = 1.0 + amp * np.exp(-r2 / (radius * radius))
    rho = 1.0 + 0.5 * np.exp(-r2 / (0.5 * radius * radius))
    z = np.zeros_like(p)
    U = conserved(rho, z, z, z, p, gamma)
    return Problem(U=U, dx=(1.0 / n,) * 3, gamma=gamma, bc=bc, name="blast")


def smooth_random(shape, seed, gamma=1.4, mach=0.5, bc=(PERIODIC,) * 6,
                  lengths=(1.0, 1.0, 1.0), grav=(0.0, 0.0, 0.0)):
    """Positive random state with a few random Fourier modes per field plus
    sharp seeded jumps (a generic parity input that exercises every branch
    of a limiter and a Riemann solver)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    x = centres(nx, lengths[0])
    y = centres(ny, lengths[1])
    z = centres(nz, lengths[2])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")

    def field_(scale):
        f = np.zeros(shape)
        for _ in range(4):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            a = rng.uniform(-1, 1)
            f += a * (np.sin(2 * math.pi * k[0] * X / lengths[0] + ph[0]) *
                      np.sin(2 * math.pi * k[1] * Y / lengths[1] + ph[1]) *
                      np.sin(2 * math.pi * k[2] * Z / lengths[2] + ph[2]))
        return scale * f

    # |field_(1)| <= 4, so rho and p stay >= 0.4
    rho = 1.0 + 0.15 * field_(1.0) + 0.5 * (rng.uniform(size=shape) > 0.85)
    p = 1.0 + 0.15 * field_(1.0) + 0.6 * (rng.uniform(size=shape) > 0.9)
    vx = mach * field_(0.25) + 0.05 * rng.standard_normal(shape)
    vy = mach * field_(0.25) + 0.05 * rng.standard_normal(shape)
    vz = mach * field_(0.25) + 0.05 * rng.standard_normal(shape)
    U = conserved(rho, vx, vy, vz, p, gamma)
    dx = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    return Problem(U=U, dx=dx, gamma=gamma, bc=bc, grav=grav,
                   name="smooth_random")


# --------------------------------------------------------------------------
# Kelvin-Helmholtz (3D periodic unit cube)
# --------------------------------------------------------------------------

def kh(n=256, seed=1, gamma=5.0 / 3.0, shape=None):
    """rho = 2 and u_x = +0.5 for |y - 0.5| < 0.25, else rho = 1 and
    u_x = -0.5; p = 2.5; u_y = 0.01 (2 xi - 1) with xi ~ U[0,1) drawn by
    numpy.random.default_rng(seed) as one (nz, ny, nx) array; u_z = 0."""
    if shape is None:
        shape = (n, n, n)
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    xi = rng.random(shape)
    y = centres(ny)
    inner = (np.abs(y - 0.5) < 0.25).reshape(1, ny, 1)
    rho = np.broadcast_to(np.where(inner, 2.0, 1.0), shape)
    vx = np.broadcast_to(np.where(inner, 0.5, -0.5), shape)
    vy = 0.01 * (2.0 * xi - 1.0)
    U = conserved(rho, vx, vy, np.zeros(shape), 2.5 * np.ones(shape), gamma)
    return Problem(U=U, dx=(1.0 / nx, 1.0 / ny, 1.0 / nz), gamma=gamma,
                   name="kh", meta={"seed": seed})


# --------------------------------------------------------------------------
# Rayleigh-Taylor ([0,0.5]^2 x [0,1], gravity along -z)
# --------------------------------------------------------------------------

def rt(nx=256, ny=256, nz=512, seed=2, gamma=1.4, g=-0.1, lengths=None):
    """Heavy (rho 2) over light (rho 1) fluid at z = 0.5 in hydrostatic
    balance p = 2.5 + g rho (z - 0.5); interface velocity
    u_z = 0.01 exp(-((z-0.5)/0.05)^2) [cos(2 pi x/Lx) cos(2 pi y/Ly) +
    (2 xi - 1)] / 2 with xi from numpy.random.default_rng(seed); periodic
    x, y; reflecting z walls."""
    if lengths is None:
        lengths = (0.5, 0.5, 1.0)
    Lx, Ly, Lz = lengths
    shape = (nz, ny, nx)
    rng = np.random.default_rng(seed)
    xi = rng.random(shape)
    x = centres(nx, Lx).reshape(1, 1, nx)
    y = centres(ny, Ly).reshape(1, ny, 1)
    z = centres(nz, Lz).reshape(nz, 1, 1)
    zi = 0.5 * Lz
    rho = np.broadcast_to(np.where(z > zi, 2.0, 1.0), shape)
    p = 2.5 + g * rho * (z - zi)
    env = 0.01 * np.exp(-(((z - zi) / 0.05) ** 2))
    vz = env * 0.5 * (np.cos(2 * math.pi * x / Lx) * np.cos(2 * math.pi * y / Ly)
                      + (2.0 * xi - 1.0))
    zero = np.zeros(shape)
    U = conserved(rho, zero, zero, vz, p, gamma)
    bc = (PERIODIC, PERIODIC, PERIODIC, PERIODIC, REFLECT, REFLECT)
    return Problem(U=U, dx=(Lx / nx, Ly / ny, Lz / nz), gamma=gamma, bc=bc,
                   grav=(0.0, 0.0, g), name="rt", meta={"seed": seed})


# --------------------------------------------------------------------------
# Batched AMR-style patches
# --------------------------------------------------------------------------

@dataclass
class PatchSpec:
    n: int            # interior cells per edge
    shear: float      # |u_x| jump across the layer
    ratio: float      # inner / outer density
    seed: np.random.SeedSequence


def batch_specs(count=4096, seed=3, sizes=(16, 32, 48, 64)):
    """Per-patch edge, shear and density ratio from default_rng(seed); the
    velocity noise of patch p uses SeedSequence(seed).spawn(count)[p], so any
    subset of patches can be regenerated on its own."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.array(sizes), size=count)
    shear = rng.uniform(0.1, 1.0, size=count)
    ratio = rng.uniform(1.0, 4.0, size=count)
    kids = np.random.SeedSequence(seed).spawn(count)
    return [PatchSpec(int(n[i]), float(shear[i]), float(ratio[i]), kids[i])
            for i in range(count)]


def kh_patch(spec: PatchSpec, gamma=5.0 / 3.0):
    """Interior state of one patch: unit cube, dx = 1/n, rho = ratio inside
    |y-0.5| < 0.25 (else 1), u_x = +shear/2 inside (else -shear/2),
    p = 2.5, u_y = 0.01 (2 xi - 1)."""
    n = spec.n
    shape = (n, n, n)
    xi = np.random.default_rng(spec.seed).random(shape)
    y = centres(n)
    inner = (np.abs(y - 0.5) < 0.25).reshape(1, n, 1)
    rho = np.broadcast_to(np.where(inner, spec.ratio, 1.0), shape)
    vx = np.broadcast_to(np.where(inner, 0.5 * spec.shear, -0.5 * spec.shear),
                         shape)
    vy = 0.01 * (2.0 * xi - 1.0)
    return conserved(rho, vx, vy, np.zeros(shape), 2.5 * np.ones(shape), gamma)


# --------------------------------------------------------------------------
# Decaying turbulence
# --------------------------------------------------------------------------

def turbulence_modes(seed=4, kmax=8, slope=-5.0 / 3.0):
    """Fourier amplitudes a_k (3 complex components) on the integer lattice
    -kmax..kmax per axis, indexed [kz, ky, kx], Hermitian (a_-k = conj a_k),
    solenoidal (k . a_k = 0), nonzero only on shells K = round(|k|) in
    1..kmax, with every mode of shell K carrying the same |a_k|^2 and the
    shell total proportional to K^slope.  Normalised so that the mean of
    |v|^2 over the periodic unit cube is 1."""
    rng = np.random.default_rng(seed)
    k1 = np.arange(-kmax, kmax + 1)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = np.rint(kk).astype(int)
    active = (shell >= 1) & (shell <= kmax)
    half = (KZ > 0) | ((KZ == 0) & (KY > 0)) | ((KZ == 0) & (KY == 0) & (KX > 0))
    A = np.zeros((3,) + KX.shape, dtype=np.complex128)
    sel = np.argwhere(active & half)
    # per-shell mode counts over the full lattice (both members of each pair)
    counts = np.bincount(shell[active], minlength=kmax + 1)
    for (iz, iy, ix) in sel:
        k = np.array([KX[iz, iy, ix], KY[iz, iy, ix], KZ[iz, iy, ix]], float)
        a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        a = a - k * (np.dot(k, a) / np.dot(k, k))
        a = a / np.linalg.norm(a)
        K = shell[iz, iy, ix]
        a = a * math.sqrt(K ** slope / counts[K])
        A[:, iz, iy, ix] = a
        A[:, 2 * kmax - iz, 2 * kmax - iy, 2 * kmax - ix] = np.conj(a)
    norm = math.sqrt(np.sum(np.abs(A) ** 2))
    return A / norm, (KX, KY, KZ), shell, active


def _turbulence_planes(n, seed, kmax, vrms):
    """Per component, the partial sums over kx and ky at every (y, x):
    T[c][kz, y, x], plus the z phase factors E[kz, z]."""
    A, _, _, _ = turbulence_modes(seed, kmax)
    A = A * vrms
    k1 = np.arange(-kmax, kmax + 1)
    x = centres(n)
    E = np.exp(2j * math.pi * np.outer(k1, x))          # (2k+1, n)
    T = []
    for c in range(3):
        T1 = np.tensordot(A[c], E, axes=([2], [0]))     # [kz, ky, x]
        T.append(np.einsum("zyx,yj->zjx", T1, E))       # [kz, y, x]
    return T, E


def turbulence_velocity(n, seed=4, kmax=8, mach=0.3, gamma=5.0 / 3.0,
                        vrms=None):
    """Velocity (3, n, n, n) of the turbulence field on an n^3 grid by a
    separable inverse DFT over the 2 kmax + 1 frequencies of each axis."""
    if vrms is None:
        vrms = mach * math.sqrt(gamma)   # rho = p = 1  =>  c = sqrt(gamma)
    T, E = _turbulence_planes(n, seed, kmax, vrms)
    return np.stack([np.tensordot(E, T[c], axes=([0], [0])).real
                     for c in range(3)])


def turbulence(n=768, seed=4, kmax=8, mach=0.3, gamma=5.0 / 3.0,
               dtype=np.float64, slab=32):
    """rho = 1, p = 1, solenoidal random-phase velocity with rms Mach `mach`
    (sound speed sqrt(gamma)).  Built slab by slab of z planes straight into
    `dtype`."""
    U = np.empty((5, n, n, n), dtype=dtype)
    vrms = mach * math.sqrt(gamma)
    T, E = _turbulence_planes(n, seed, kmax, vrms)
    for z0 in range(0, n, slab):
        z1 = min(n, z0 + slab)
        Ez = E[:, z0:z1]
        v = [np.tensordot(Ez, T[c], axes=([0], [0])).real for c in range(3)]
        one = np.ones(v[0].shape)
        sl = conserved(one, v[0], v[1], v[2], one, gamma)
        U[:, z0:z1] = sl.astype(dtype)
    return Problem(U=U, dx=(1.0 / n,) * 3, gamma=gamma, name="turbulence",
                   meta={"seed": seed, "mach": mach})


def batch_pool(specs, ng=4, dtype=np.float64, align=64, gamma=5.0 / 3.0, pad_rows=0):
    """Pack the interior states of `specs` into one flat pool.  Patch p holds
    5 planes with its interior and `ng` ghost layers on every side (the ghost
    layers hold the periodic wrap of the interior), starting at a multiple of
    `align` elements.  pad_rows = 0 stores rows of n + 2 ng elements back to
    back; pad_rows = A > 0 places interior cell x = 0 of every row on a
    multiple of A elements (A = 32 puts it on a 128-byte boundary in FP32)
    and pads the row pitch to a multiple of A.  Returns (pool, patches) with
    patches[p] = (offset_elems, nx, ny, nz, ng, dx, dy, dz, row_pitch,
    slab_pitch, plane_pitch, interior_offset)."""
    layout = []
    off = 0
    for s in specs:
        m = s.n + 2 * ng
        if pad_rows:
            A = pad_rows
            rp = -(-(A + s.n + ng) // A) * A
            x0 = A - ng                     # element of ghost x = -ng in its row
        else:
            rp = m
            x0 = 0
        sp = rp * m
        pp = sp * m
        io = x0 + ng + ng * rp + ng * sp
        layout.append((off, rp, sp, pp, io, x0))
        off += 5 * pp
        off = (off + align - 1) // align * align
    pool = np.zeros(off, dtype=dtype)
    patches = []
    for s, (o, rp, sp, pp, io, x0) in zip(specs, layout):
        m = s.n + 2 * ng
        U = kh_patch(s, gamma)
        if ng:
            U = np.pad(U, ((0, 0), (ng, ng), (ng, ng), (ng, ng)), mode="wrap")
        blk = pool[o:o + 5 * pp].reshape(5, m, m, rp)[:, :, :, x0:x0 + m]
        blk[...] = U.astype(dtype)
        d = 1.0 / s.n
        patches.append((o, s.n, s.n, s.n, ng, d, d, d, rp, sp, pp, io))
    return pool, patches


def patch_view(pool, patch):
    """(5, nz+2ng, ny+2ng, nx+2ng) view (ghosts included) of one patch of a
    pool, for either layout of batch_pool."""
    o, nx, ny, nz, ng = patch[:5]
    if len(patch) > 8 and patch[8]:
        rp, sp, pp, io = patch[8:12]
    else:
        rp = nx + 2 * ng
        sp = rp * (ny + 2 * ng)
        pp = sp * (nz + 2 * ng)
        io = ng * (1 + rp + sp)
    start = o + io - ng * (1 + rp + sp)
    it = pool.itemsize
    return np.lib.stride_tricks.as_strided(
        pool[start:], shape=(5, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng),
        strides=(pp * it, sp * it, rp * it, it), writeable=False)
