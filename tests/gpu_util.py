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


def rel_err(got, want):
    """max |got - want| / max |want| per conserved variable."""
    out = []
    for v in range(5):
        scale = max(np.abs(want[v]).max(), 1e-300)
        out.append(float(np.abs(got[v] - want[v]).max() / scale))
    return out


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
