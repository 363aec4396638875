"""FP64 oracle of the operator-split reactive source (a toy network).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by bench.py's cpu_baseline
leg, never by the product package.  It shares no code with the HIP path.

The paper's explosion models carry nuclear networks of 10-20 nuclei in the
hydrodynamics (its discussion of the physics the simulations need) and gives
no rates; the build's stand-in is a self-contained chain of M species with
the same structure of a stiff per-zone source:

    species 0 -> 1 -> ... -> M-1 (the last is stable), link i (species i to
    i+1) with rate k_i(T) = A_i exp(-Ta_i / T), T = p / rho (code units,
    from the zone's state, held fixed over the step: operator splitting
    with frozen thermodynamics), releasing q_i per unit mass converted.

    dX_0/dt = -k_0 X_0,  dX_i/dt = k_{i-1} X_{i-1} - k_i X_i,  dX_{M-1}/dt = k_{M-2} X_{M-2}

Integrator: nsub equal substeps h = dt / nsub of backward Euler.  For this
lower-bidiagonal system each substep is solved exactly by forward
substitution:
    X_0' = X_0 / (1 + h k_0),  X_i' = (X_i + h k_{i-1} X_{i-1}') / (1 + h k_i),
with k_{M-1} = 0.  Backward Euler conserves sum_i X_i exactly (in exact
arithmetic) and is L-stable, so stiff links (h k >> 1) empty in one substep.

Energy: the total energy density gains rho * sum_i B_i (X_i' - X_i) over the
step, with B_i = q_0 + ... + q_{i-1} the energy released in making species i
from species 0.

States are (5, nz, ny, nx) (rho, mx, my, mz, E) and compositions
(M, nz, ny, nx), interior cells only.
"""
import numpy as np


def temperature(U, gamma):
    """T = p / rho with p = (gamma - 1)(E - |m|^2 / (2 rho))."""
    U = np.asarray(U, dtype=np.float64)
    r = U[0]
    m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3]
    p = (gamma - 1.0) * (U[4] - (0.5 * m2) / r)
    return p / r


def rates(T, A, Ta):
    """k_i(T) = A_i exp(-Ta_i / T) for each link; shape (M - 1,) + T.shape."""
    A = np.asarray(A, dtype=np.float64).reshape((-1,) + (1,) * np.ndim(T))
    Ta = np.asarray(Ta, dtype=np.float64).reshape((-1,) + (1,) * np.ndim(T))
    return A * np.exp(-Ta / T)


def burn(U, X, gamma, A, Ta, q, dt, nsub):
    """One operator-split source step.  Returns (U', X') as new FP64 arrays:
    X integrated by nsub backward-Euler substeps, E raised by the released
    energy; rho and momentum unchanged."""
    U = np.array(U, dtype=np.float64)
    X = np.array(X, dtype=np.float64)
    M = X.shape[0]
    k = rates(temperature(U, gamma), A, Ta)               # (M-1, ...)
    h = dt / nsub
    X0 = X.copy()
    for _ in range(nsub):
        X[0] = X[0] / (1.0 + h * k[0])
        for i in range(1, M):
            ki = k[i] if i < M - 1 else 0.0
            X[i] = (X[i] + h * k[i - 1] * X[i - 1]) / (1.0 + h * ki)
    B = np.concatenate([[0.0], np.cumsum(np.asarray(q, dtype=np.float64))])
    dE = U[0] * np.tensordot(B[:M], X - X0, axes=(0, 0))
    U[4] = U[4] + dE
    return U, X


def bateman(X00, k, t):
    """Exact solution of the chain from X_0(0) = X00 (all other species 0) at
    time t, for distinct rates k_0..k_{M-2} (the last species stable):
    X_n(t) = X00 (prod_{j<n} k_j) sum_{i<=n} exp(-k_i t) / prod_{j<=n, j!=i} (k_j - k_i),
    with k_{M-1} = 0."""
    kk = list(k) + [0.0]
    M = len(kk)
    out = np.zeros(M)
    for n in range(M):
        pre = np.prod(kk[:n])
        s = 0.0
        for i in range(n + 1):
            den = np.prod([kk[j] - kk[i] for j in range(n + 1) if j != i])
            s += np.exp(-kk[i] * t) / den
        out[n] = X00 * pre * s
    return out
