"""FP64 CPU oracle for the compressible-Euler zone update.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke()
and by the cpu_baseline leg of bench.py, never by the product package.
It shares no code with the HIP path.

The scheme (primitive MC-limited MUSCL-Hancock, HLLC with Davis speeds,
x,y,z / z,y,x split sweeps, constant gravity, CFL dt) lives in oracle.c;
this module only marshals numpy arrays into it.  The exact Riemann solver
used to pin it is in oracle/exact_riemann.py.

State arrays are float64 of shape (5, nz, ny, nx), C order, holding
(rho, mx, my, mz, E).
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2
OK, EINVAL, ENOMEM, ENUMERIC = 0, 1, 2, 3


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("grav", ctypes.c_double * 3),
        ("nthreads", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("HYDRO_ORACLE_LIB", "")   # mutation tests only
    if not path:
        path = LIB
        if not os.path.exists(LIB):
            build()
    lib = ctypes.CDLL(path)
    lib.oracle_step.argtypes = [ctypes.POINTER(Params), _dp, ctypes.c_double,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_long)]
    lib.oracle_sweep.argtypes = [ctypes.POINTER(Params), _dp, ctypes.c_double,
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
    lib.oracle_sweep_flux.argtypes = [ctypes.POINTER(Params), _dp, ctypes.c_double,
                                      ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_long)]
    lib.oracle_run.argtypes = [ctypes.POINTER(Params), _dp, ctypes.c_int64,
                               ctypes.c_double, _dp,
                               ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_long)]
    lib.oracle_cfl_dt.argtypes = [ctypes.POINTER(Params), _dp, _dp]
    lib.oracle_totals.argtypes = [ctypes.POINTER(Params), _dp, _dp]
    lib.oracle_prim.argtypes = [_dp, ctypes.c_double, _dp]
    lib.oracle_prim.restype = None
    lib.oracle_mc_slope.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_mc_slope.restype = ctypes.c_double
    lib.oracle_hllc.argtypes = [_dp, _dp, ctypes.c_double, _dp]
    lib.oracle_hllc.restype = None
    lib.oracle_hancock.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.oracle_hancock.restype = None
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def make_params(shape, dx, gamma, cfl=0.8, bc=(PERIODIC,) * 6,
                grav=(0.0, 0.0, 0.0), nthreads=0):
    """shape = (nz, ny, nx); dx = (dx, dy, dz) or a scalar."""
    nz, ny, nx = shape
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    p = Params()
    p.n[:] = [nx, ny, nz]
    p.bc[:] = list(bc)
    p.dx[:] = list(dx)
    p.gamma = gamma
    p.cfl = cfl
    p.grav[:] = list(grav)
    p.nthreads = nthreads
    return p


def _arr(U):
    if U.dtype != np.float64 or not U.flags.c_contiguous or U.ndim != 4 \
            or U.shape[0] != 5:
        raise ValueError("state must be C-contiguous float64 (5, nz, ny, nx)")
    return U.ctypes.data_as(_dp)


def _check_shape(p, U):
    if tuple(U.shape[1:]) != (p.n[2], p.n[1], p.n[0]):
        raise ValueError("state shape does not match params")


def step(p, U, dt, step_index):
    """One Strang step with a given dt, in place; returns the fallback count."""
    _check_shape(p, U)
    fb = ctypes.c_long(0)
    rc = _load().oracle_step(ctypes.byref(p), _arr(U), dt, step_index,
                             ctypes.byref(fb))
    if rc != OK:
        raise OracleError(f"oracle_step failed ({rc})")
    return fb.value


def sweep(p, U, dt, axis):
    """A single directional sweep along axis (0=x, 1=y, 2=z), in place."""
    _check_shape(p, U)
    fb = ctypes.c_long(0)
    rc = _load().oracle_sweep(ctypes.byref(p), _arr(U), dt, axis,
                              ctypes.byref(fb))
    if rc != OK:
        raise OracleError(f"oracle_sweep failed ({rc})")
    return fb.value


def sweep_flux(p, U, dt, axis):
    """sweep() that also returns the face fluxes it applied: float64
    (5, ...) in lab components with n + 1 entries along `axis`, entry i
    being the face between cells i - 1 and i."""
    _check_shape(p, U)
    shape = list(U.shape)
    shape[3 - axis] += 1
    F = np.zeros(shape)
    fb = ctypes.c_long(0)
    rc = _load().oracle_sweep_flux(ctypes.byref(p), _arr(U), dt, axis,
                                   F.ctypes.data_as(_dp), ctypes.byref(fb))
    if rc != OK:
        raise OracleError(f"oracle_sweep_flux failed ({rc})")
    return F


def run(p, U, nsteps, t_end=0.0, t=0.0, step_index=0):
    """Advance with the CFL dt; returns (t, step_index, fallbacks)."""
    _check_shape(p, U)
    tt = ctypes.c_double(t)
    ss = ctypes.c_int64(step_index)
    fb = ctypes.c_long(0)
    rc = _load().oracle_run(ctypes.byref(p), _arr(U), nsteps, t_end,
                            ctypes.byref(tt), ctypes.byref(ss), ctypes.byref(fb))
    if rc != OK:
        raise OracleError(f"oracle_run failed ({rc})")
    return tt.value, ss.value, fb.value


def cfl_dt(p, U):
    _check_shape(p, U)
    dt = ctypes.c_double(0.0)
    rc = _load().oracle_cfl_dt(ctypes.byref(p), _arr(U), ctypes.byref(dt))
    if rc != OK:
        raise OracleError(f"oracle_cfl_dt failed ({rc})")
    return dt.value


def totals(p, U):
    """(rho, mx, my, mz, E, E + rho*phi) summed over cells times volume."""
    _check_shape(p, U)
    out = np.zeros(6)
    rc = _load().oracle_totals(ctypes.byref(p), _arr(U), out.ctypes.data_as(_dp))
    if rc != OK:
        raise OracleError(f"oracle_totals failed ({rc})")
    return out


def prim(U5, gamma):
    U5 = np.ascontiguousarray(U5, dtype=np.float64)
    W = np.zeros(5)
    _load().oracle_prim(U5.ctypes.data_as(_dp), gamma, W.ctypes.data_as(_dp))
    return W


def mc_slope(a, b):
    return _load().oracle_mc_slope(a, b)


def hllc(WL, WR, gamma):
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    _load().oracle_hllc(WL.ctypes.data_as(_dp), WR.ctypes.data_as(_dp), gamma,
                        F.ctypes.data_as(_dp))
    return F


def hancock(W, D, dtdx, gamma, half_dt_g=0.0, has_g=False):
    W = np.ascontiguousarray(W, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    Wm = np.zeros(5)
    Wp = np.zeros(5)
    _load().oracle_hancock(W.ctypes.data_as(_dp), D.ctypes.data_as(_dp), dtdx,
                           gamma, half_dt_g, int(has_g), Wm.ctypes.data_as(_dp),
                           Wp.ctypes.data_as(_dp))
    return Wm, Wp
