"""FP64 oracle of the in-situ diagnostics.

TEST INFRASTRUCTURE ONLY: imported by tests/ and by bench.py's cpu_baseline
leg, never by the product package.  It shares no code with the HIP path.

The paper names in-situ analysis of the flow as a capability large runs
need (its discussion of the capabilities needed at the exascale) but fixes
no diagnostic.  These are the definitions the library implements, written
out plainly with numpy, on states of shape (5, nz, ny, nx) holding
(rho, mx, my, mz, E) (interior cells only).

Cell quantities, in FP64 with IEEE operations in exactly this order (an
FP32 state is widened to FP64 first, which is exact):
    m2    = mx*mx + my*my + mz*mz
    ke    = (0.5 * m2) / rho                 kinetic energy density
    p     = (gamma - 1) * (E - ke)           pressure
    speed = sqrt(m2) / rho                   |v|
    mach  = sqrt(m2 / ((gamma * p) * rho))   |v| / c = sqrt(|m|^2 / (gamma p rho))

PDF of a quantity q over [lo, hi) in nbins bins, with w = nbins / (hi - lo):
    counts[0]          cells with not (q >= lo)  (below range, or NaN)
    counts[1 + b]      cells with b = floor((q - lo) * w) in [0, nbins)
    counts[nbins + 1]  the rest (at or above hi)
The bin decision is taken in FP64 on both sides, so the counts are exact.

Slab profiles along an axis: for every slab i (cells with equal index along
the axis) the means of rho, p, ke, f and f (1 - f), with the heavy-fluid
fraction f = clip((rho - rho_lo) / (rho_hi - rho_lo), 0, 1) of a layer
between densities rho_lo and rho_hi.  From them:
    mixing width  W     = sum_i 4 <f>_i (1 - <f>_i) dx_axis
    mixedness     Theta = sum_i <f (1-f)>_i / sum_i <f>_i (1 - <f>_i)
                          (0 when the denominator is 0)

Kinetic-energy spectrum along x: the x-line DFTs of the velocity m / rho,
their power summed over components, averaged over lines and folded onto
k = 0 .. nx//2 so that the spectrum sums to the mean specific kinetic
energy (spectrum_x).

Shell kinetic-energy spectrum (spectrum_shell): the three-dimensional DFT of
the velocity m / rho over the grid, its power summed over components and
over the integer wavevectors of each shell K = round(|k|), scaled so that
the shells sum to the mean specific kinetic energy (Parseval).  The shells
are those that set the turbulence initial data's spectrum (E(K) ~ K^(-5/3)
over shells 1..8), so the diagnostic reads that spectrum back.
"""
import numpy as np

RHO, PRESSURE, SPEED, MACH = 0, 1, 2, 3
QUANTITIES = (RHO, PRESSURE, SPEED, MACH)
PROFILE_FIELDS = ("rho", "p", "ke", "f", "f1mf")


def quantity(U, gamma, q):
    """Cell values of quantity q (RHO, PRESSURE, SPEED, MACH), FP64."""
    U = np.asarray(U, dtype=np.float64)
    r, mx, my, mz, e = U[0], U[1], U[2], U[3], U[4]
    if q == RHO:
        return r.copy()
    with np.errstate(all="ignore"):
        m2 = mx * mx + my * my + mz * mz
        ke = (0.5 * m2) / r
        p = (gamma - 1.0) * (e - ke)
        if q == PRESSURE:
            return p
        if q == SPEED:
            return np.sqrt(m2) / r
        if q == MACH:
            return np.sqrt(m2 / ((gamma * p) * r))
    raise ValueError(f"unknown quantity {q}")


def pdf(states, gamma, q, lo, hi, nbins):
    """Counts (int64, nbins + 2) of quantity q over every cell of the given
    states (one state, or a list of patch interiors)."""
    if isinstance(states, np.ndarray):
        states = [states]
    w = nbins / (hi - lo)
    counts = np.zeros(nbins + 2, dtype=np.int64)
    for U in states:
        v = quantity(U, gamma, q).ravel()
        below = ~(v >= lo)
        with np.errstate(invalid="ignore"):
            t = (v - lo) * w
        inside = ~below & (t < nbins)
        b = np.floor(t[inside]).astype(np.int64)
        counts[0] += int(below.sum())
        counts[1:nbins + 1] += np.bincount(b, minlength=nbins)[:nbins]
        counts[nbins + 1] += int((~below & ~inside).sum())
    return counts


def profile(U, gamma, axis, rho_lo, rho_hi):
    """(n_axis, 5) slab means of (rho, p, ke, f, f (1 - f)) along axis
    (0: x, 1: y, 2: z)."""
    U = np.asarray(U, dtype=np.float64)
    r = U[0]
    with np.errstate(all="ignore"):
        m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3]
        ke = (0.5 * m2) / r
        p = (gamma - 1.0) * (U[4] - ke)
    f = np.clip((r - rho_lo) / (rho_hi - rho_lo), 0.0, 1.0)
    fields = (r, p, ke, f, f * (1.0 - f))
    # array axes are (z, y, x): sweep axis a is array axis 2 - a
    other = tuple(i for i in range(3) if i != 2 - axis)
    return np.stack([v.mean(axis=other) for v in fields], axis=1)


def mixing(prof, dx_axis):
    """(W, Theta) from a profile as returned by profile()."""
    fbar = prof[:, 3]
    den = float(np.sum(fbar * (1.0 - fbar)))
    width = float(np.sum(4.0 * fbar * (1.0 - fbar)) * dx_axis)
    theta = float(np.sum(prof[:, 4]) / den) if den > 0.0 else 0.0
    return width, theta


def spectrum_x(U):
    """One-dimensional kinetic-energy spectrum along x of the velocity
    u = m / rho: with P[k] the mean over the x-lines of sum over the three
    components of |FFT_x(u)[k]|^2 (numpy's unnormalised DFT, N = nx),
        E[0] = P[0] / (2 N^2),  E[k] = P[k] / N^2 (0 < k < N/2),
        E[N/2] = P[N/2] / (2 N^2) for even N,
    k = 0 .. N//2 (the +k and -k halves folded), so that by Parseval
    sum_k E[k] = (1/2) <|u|^2>, the mean specific kinetic energy."""
    U = np.asarray(U, dtype=np.float64)
    n = U.shape[3]
    with np.errstate(all="ignore"):
        u = U[1:4] / U[0]
    P = (np.abs(np.fft.fft(u, axis=-1)) ** 2).sum(axis=0).reshape(-1, n).mean(axis=0)
    E = P[:n // 2 + 1] / float(n * n)
    E[0] *= 0.5
    if n % 2 == 0:
        E[n // 2] *= 0.5
    return E


def wavenumbers(n):
    """Signed integer wavenumbers of a DFT of length n in numpy's order:
    0, 1, .., then the negative ones (-n/2 at index n/2 for even n)."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def shell_index(m2):
    """Shell K = round(sqrt(m2)) of integer wavevectors with |k|^2 = m2
    (int64 array).  sqrt of an integer is never a half-integer, so the
    rounding has no ties; K is the integer with K - 1/2 <= |k| < K + 1/2."""
    return np.rint(np.sqrt(np.asarray(m2, dtype=np.float64))).astype(np.int64)


def shell_count(shape):
    """Number of shells K = 0 .. K_max of a (nz, ny, nx) grid: K_max is the
    shell of the corner wavevector (nx//2, ny//2, nz//2)."""
    nz, ny, nx = shape
    return int(shell_index((nx // 2) ** 2 + (ny // 2) ** 2 + (nz // 2) ** 2)) + 1


def spectrum_shell(U):
    """Shell kinetic-energy spectrum of the velocity u = m / rho over the
    grid: with u_hat_c the unnormalised three-dimensional DFT of component c
    (numpy's fftn over the grid, N = nx ny nz cells) and k the signed integer
    wavevector of each coefficient,
        E[K] = sum over k with round(|k|) = K of sum_c |u_hat_c(k)|^2 / (2 N^2),
    K = 0 .. K_max (shell_count), so that by Parseval
    sum_K E[K] = (1/2) <|u|^2>, the mean specific kinetic energy."""
    U = np.asarray(U, dtype=np.float64)
    nz, ny, nx = U.shape[1:]
    with np.errstate(all="ignore"):
        u = U[1:4] / U[0]
    F = np.fft.fftn(u, axes=(1, 2, 3))
    P = (F.real * F.real + F.imag * F.imag).sum(axis=0)
    kz, ky, kx = (wavenumbers(n) for n in (nz, ny, nx))
    m2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    K = shell_index(m2)
    nb = shell_count((nz, ny, nx))
    N = float(nx) * ny * nz
    return np.bincount(K.ravel(), weights=P.ravel(), minlength=nb) / (2.0 * N * N)
