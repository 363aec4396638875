"""Helpers shared by the GPU tests (no numerics of the scheme here)."""
import sys

import numpy as np

import oracle
from paper_1510_05061_amd import hydro


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def params_of(P, nthreads=0):
    return oracle.make_params(P.shape, P.dx, P.gamma, P.cfl, P.bc, P.grav,
                              nthreads=nthreads)


def to_device(U, prec):
    t = torch()
    dt = np.float64 if prec == hydro.FP64 else np.float32
    return t.from_numpy(np.ascontiguousarray(U.astype(dt))).to("cuda:0")


def gpu_grid(P, prec=hydro.FP64, flags=hydro.FLAG_NO_TUNE, config=None, U=None):
    dev = to_device(P.U if U is None else U, prec)
    g = hydro.Grid(dev, P.dx, P.gamma, P.cfl, P.bc, P.grav, flags=flags)
    if config:
        g.config = config
    return g, dev


def host(dev):
    torch().cuda.synchronize()
    return dev.double().cpu().numpy()


def rel_err(got, want, scale=None):
    """max |got - want| / max |want| per conserved variable.  `scale` (one
    value per variable) replaces max |want| when `want` is a sampled block:
    the parity bound is relative to the variable's scale over the whole grid,
    and a block where a variable is nearly zero (m_z far from an RT
    interface) would otherwise turn round-off into a large ratio."""
    out = []
    for v in range(5):
        s = np.abs(want[v]).max() if scale is None else scale[v]
        out.append(float(np.abs(got[v] - want[v]).max() / max(s, 1e-300)))
    return out


def grid_scale(U):
    """max |q| over the whole grid, per conserved variable."""
    return [float(np.abs(U[v]).max()) for v in range(5)]


def l1_err(got, want):
    """sum |got - want| / sum |want| per conserved variable."""
    out = []
    for v in range(5):
        scale = max(np.abs(want[v]).sum(), 1e-300)
        out.append(float(np.abs(got[v] - want[v]).sum() / scale))
    return out


def l1_fp32_errors(got, want):
    """L1 error measures of an FP32 result against the FP64 oracle:
    (e_rho, e_m, e_E) with e_q = sum |q32 - q64| / sum |q64| for rho and E,
    and for the momentum the component errors summed over the three axes
    divided by sum |m|_1 (a component that is nearly zero everywhere, such as
    m_z of a KH layer after one step, would make its own ratio meaningless)."""
    e_rho = float(np.abs(got[0] - want[0]).sum() / np.abs(want[0]).sum())
    e_E = float(np.abs(got[4] - want[4]).sum() / np.abs(want[4]).sum())
    e_m = float(np.abs(got[1:4] - want[1:4]).sum() / np.abs(want[1:4]).sum())
    return e_rho, e_m, e_E


def sub_box(U, z0, y0, x0, m):
    """(5, m, m, m) block of U starting at (z0, y0, x0), wrapping periodically."""
    nz, ny, nx = U.shape[1:]
    iz = (np.arange(z0, z0 + m) % nz)[:, None, None]
    iy = (np.arange(y0, y0 + m) % ny)[None, :, None]
    ix = (np.arange(x0, x0 + m) % nx)[None, None, :]
    return np.ascontiguousarray(U[:, iz, iy, ix])


def oracle_box_step(U_in, corner, m, P, dt, step, bc_axes_periodic=(True, True, True)):
    """Oracle step of an (m+4)^3 box of the input around `corner` (the low
    corner of the m^3 output block); returns the exact m^3 centre.  Cells
    within 2 of a box face see wrong boundary data only through sweeps along
    that axis, so the centre, 2 cells in from every face, is exact."""
    import oracle
    z0, y0, x0 = corner
    box = sub_box(U_in, z0 - 2, y0 - 2, x0 - 2, m + 4)
    p = oracle.make_params(box.shape[1:], P.dx, P.gamma, P.cfl, (1,) * 6, P.grav)
    oracle.step(p, box, dt, step)
    return box[:, 2:-2, 2:-2, 2:-2]


def max_fp32_errors(got, want):
    """Per-cell (max-norm) errors of an FP32 result against the FP64 oracle:
    (e_rho, e_m, e_E) with e_q = max_i |q32 - q64| / max_i |q64| for rho and
    E, and for the momentum the largest component difference over the
    largest momentum magnitude max_i |m_i| (one scale for the three
    components, as in the L1 measure)."""
    e_rho = float(np.abs(got[0] - want[0]).max() / np.abs(want[0]).max())
    e_E = float(np.abs(got[4] - want[4]).max() / np.abs(want[4]).max())
    m_scale = float(np.sqrt((want[1:4] ** 2).sum(axis=0)).max())
    e_m = float(np.abs(got[1:4] - want[1:4]).max() / max(m_scale, 1e-300))
    return e_rho, e_m, e_E


def sub_box_dev(dev, z0, y0, x0, m):
    """sub_box of a device state tensor, gathered on the device (only the
    (5, m, m, m) block crosses to the host)."""
    t = torch()
    nz, ny, nx = dev.shape[1:]
    idx = [t.tensor(np.arange(a, a + m) % n, device=dev.device) for a, n in
           ((z0, nz), (y0, ny), (x0, nx))]
    return dev.index_select(1, idx[0]).index_select(2, idx[1]).index_select(3, idx[2])
