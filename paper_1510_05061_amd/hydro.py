"""ctypes binding of libhydro (include/hydro.h): argument marshalling only.

Every numerical step runs in the HIP kernels of libhydro.so.  PyTorch
supplies device memory and the stream; nothing here computes on the state.
If the library is missing this module raises on import of `lib()`: there is
no CPU fallback.

Two layers:
  * functions with the C names (hydro_init, hydro_step, ...) that take and
    return plain values and raise HydroError on a non-zero status;
  * `Grid` and `Batch`, small owners of a context plus its workspace
    tensor.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro.so")

HYDRO_OK, HYDRO_EINVAL, HYDRO_EDEVICE, HYDRO_ENUMERIC, HYDRO_ESTATE = range(5)
PERIODIC, OUTFLOW, REFLECT = 0, 1, 2
FP32, FP64 = 0, 1
Q_RHO, Q_PRESSURE, Q_SPEED, Q_MACH = 0, 1, 2, 3
FLAG_NO_GRAPH, FLAG_NO_TUNE, BATCH_PER_PATCH_DT, FLAG_FUSE_XY = 0x1, 0x2, 0x4, 0x8
DT_CFL = 0.0


class HydroDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("ng", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("grav", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 6),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


MAX_SPECIES = 20


class HydroNetwork(ctypes.Structure):
    _fields_ = [
        ("nspec", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("A", ctypes.c_double * (MAX_SPECIES - 1)),
        ("Ta", ctypes.c_double * (MAX_SPECIES - 1)),
        ("q", ctypes.c_double * (MAX_SPECIES - 1)),
    ]


def make_network(A, Ta, q):
    """hydro_network for a chain of len(A) + 1 species."""
    n = len(A) + 1
    net = HydroNetwork()
    net.nspec = n
    for i in range(min(n - 1, MAX_SPECIES - 1)):
        net.A[i], net.Ta[i], net.q[i] = float(A[i]), float(Ta[i]), float(q[i])
    return net


class HydroAmrLink(ctypes.Structure):
    _fields_ = [("fine", ctypes.c_int32), ("coarse", ctypes.c_int32), ("ox", ctypes.c_int32),
                ("oy", ctypes.c_int32), ("oz", ctypes.c_int32), ("pad", ctypes.c_int32)]


def make_links(links):
    """hydro_amr_link array from (fine, coarse, ox, oy, oz) tuples."""
    arr = (HydroAmrLink * max(1, len(links)))()
    for i, (f, c, ox, oy, oz) in enumerate(links):
        arr[i].fine, arr[i].coarse, arr[i].ox, arr[i].oy, arr[i].oz = f, c, ox, oy, oz
    return arr


class HydroPatch(ctypes.Structure):
    _fields_ = [
        ("offset_elems", ctypes.c_int64),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("ng", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("row_pitch", ctypes.c_int64), ("slab_pitch", ctypes.c_int64),
        ("plane_pitch", ctypes.c_int64), ("interior_offset", ctypes.c_int64),
    ]


class HydroError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__(f"{where}: status {status} ({detail})")


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "hydro_abi_version": ([], ctypes.c_int),
    "hydro_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "hydro_last_error": ([], ctypes.c_char_p),
    "hydro_workspace_bytes": ([ctypes.POINTER(HydroDesc), ctypes.POINTER(_sz)], ctypes.c_int),
    "hydro_init": ([ctypes.POINTER(HydroDesc), _vp, _sz, _vp, _sz, _vp,
                    ctypes.POINTER(_vp)], ctypes.c_int),
    "hydro_cfl_dt": ([_vp, _dp], ctypes.c_int),
    "hydro_step": ([_vp, ctypes.c_double], ctypes.c_int),
    "hydro_step_noalloc": ([ctypes.POINTER(HydroDesc), _vp, _sz, ctypes.c_double, ctypes.c_int64,
                            _vp, _vp], ctypes.c_int),
    "hydro_sweep": ([_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "hydro_batch_workspace_bytes": ([ctypes.POINTER(HydroPatch), ctypes.c_int32,
                                     ctypes.POINTER(HydroDesc), ctypes.POINTER(_sz)],
                                    ctypes.c_int),
    "hydro_batch_init": ([ctypes.POINTER(HydroPatch), ctypes.c_int32,
                          ctypes.POINTER(HydroDesc), _vp, _sz, _vp, _sz, _vp,
                          ctypes.POINTER(_vp)], ctypes.c_int),
    "hydro_batch_step": ([_vp, ctypes.c_double], ctypes.c_int),
    "hydro_batch_times": ([_vp, _dp, _dp], ctypes.c_int),
    "hydro_totals": ([_vp, _dp], ctypes.c_int),
    "hydro_diag_pdf": ([_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                        _vp], ctypes.c_int),
    "hydro_diag_profile": ([_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, _vp],
                           ctypes.c_int),
    "hydro_diag_spectrum": ([_vp, _vp], ctypes.c_int),
    "hydro_diag_spectrum3d_workspace_bytes": ([_vp, ctypes.POINTER(_sz),
                                               ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "hydro_diag_spectrum3d": ([_vp, _vp, _sz, _vp], ctypes.c_int),
    "hydro_fill_ghosts": ([_vp], ctypes.c_int),
    "hydro_amr_restrict": ([_vp, ctypes.POINTER(HydroAmrLink), ctypes.c_int32], ctypes.c_int),
    "hydro_amr_prolong": ([_vp, ctypes.POINTER(HydroAmrLink), ctypes.c_int32, ctypes.c_int],
                          ctypes.c_int),
    "hydro_amr_cfl_dt": ([_vp, _vp, _dp], ctypes.c_int),
    "hydro_amr_step_workspace_bytes": ([_vp, _vp, ctypes.c_int32, ctypes.POINTER(_sz)],
                                       ctypes.c_int),
    "hydro_amr_step": ([_vp, _vp, ctypes.POINTER(HydroAmrLink), ctypes.c_int32, ctypes.c_int32,
                        ctypes.c_double, ctypes.c_uint32, _vp, _sz], ctypes.c_int),
    "hydro_burn": ([_vp, _vp, _sz, ctypes.POINTER(HydroNetwork), ctypes.c_double, ctypes.c_int32],
                   ctypes.c_int),
    "hydro_get_time": ([_vp, _dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "hydro_set_time": ([_vp, ctypes.c_double, ctypes.c_int64], ctypes.c_int),
    "hydro_set_t_end": ([_vp, ctypes.c_double], ctypes.c_int),
    "hydro_state_changed": ([_vp], ctypes.c_int),
    "hydro_get_error": ([_vp], ctypes.c_int),
    "hydro_clear_error": ([_vp], ctypes.c_int),
    "hydro_get_config": ([_vp, ctypes.c_char_p, _sz], ctypes.c_int),
    "hydro_set_config": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "hydro_time_sweeps": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "hydro_profile_step": ([_vp, ctypes.c_double, _dp], ctypes.c_int),
    "hydro_stream_ceiling": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "hydro_destroy": ([_vp], ctypes.c_int),
}


def lib():
    """Load libhydro.so (built in-tree by __graft_entry__.build()).  Raises if
    it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc, where):
    if rc != HYDRO_OK:
        detail = lib().hydro_last_error().decode(errors="replace")
        raise HydroError(rc, where, detail or lib().hydro_strerror(rc).decode())
    return rc


# --------------------------------------------------------------------------
# C-named wrappers
# --------------------------------------------------------------------------

def hydro_abi_version():
    return lib().hydro_abi_version()


def hydro_workspace_bytes(desc):
    n = _sz(0)
    _check(lib().hydro_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)),
           "hydro_workspace_bytes")
    return n.value


def hydro_init(desc, state_ptr, state_bytes, ws_ptr, ws_bytes, stream_ptr):
    ctx = _vp()
    _check(lib().hydro_init(ctypes.byref(desc), state_ptr, state_bytes, ws_ptr, ws_bytes,
                            stream_ptr, ctypes.byref(ctx)), "hydro_init")
    return ctx


def hydro_batch_workspace_bytes(patches, desc):
    n = _sz(0)
    _check(lib().hydro_batch_workspace_bytes(patches, len(patches), ctypes.byref(desc),
                                             ctypes.byref(n)), "hydro_batch_workspace_bytes")
    return n.value


def hydro_batch_init(patches, desc, pool_ptr, pool_bytes, ws_ptr, ws_bytes, stream_ptr):
    ctx = _vp()
    _check(lib().hydro_batch_init(patches, len(patches), ctypes.byref(desc), pool_ptr,
                                  pool_bytes, ws_ptr, ws_bytes, stream_ptr,
                                  ctypes.byref(ctx)), "hydro_batch_init")
    return ctx


def hydro_cfl_dt(ctx):
    dt = ctypes.c_double(0.0)
    _check(lib().hydro_cfl_dt(ctx, ctypes.byref(dt)), "hydro_cfl_dt")
    return dt.value


def hydro_step(ctx, dt=DT_CFL):
    _check(lib().hydro_step(ctx, float(dt)), "hydro_step")


NOALLOC_SCRATCH_BYTES = 1 << 20


def hydro_step_noalloc(desc, state_ptr, state_bytes, dt, step, stream_ptr, out_ptr=None):
    """One step of a single grid with no context and no allocation
    (asynchronous); out_ptr: None or a device float64[9] (see hydro.h)."""
    _check(lib().hydro_step_noalloc(ctypes.byref(desc), state_ptr, state_bytes, float(dt),
                                    int(step), stream_ptr, out_ptr), "hydro_step_noalloc")


def hydro_batch_step(ctx, dt=DT_CFL):
    _check(lib().hydro_batch_step(ctx, float(dt)), "hydro_batch_step")


def hydro_batch_times(ctx, n):
    """(t, dt) lists of the n patches of a batch."""
    t = (ctypes.c_double * n)()
    dt = (ctypes.c_double * n)()
    _check(lib().hydro_batch_times(ctx, t, dt), "hydro_batch_times")
    return list(t), list(dt)


def hydro_sweep(ctx, axis, dt, fold_cfl=False):
    _check(lib().hydro_sweep(ctx, int(axis), float(dt), int(bool(fold_cfl))), "hydro_sweep")


def hydro_totals(ctx):
    out = (ctypes.c_double * 6)()
    _check(lib().hydro_totals(ctx, out), "hydro_totals")
    return list(out)


def hydro_diag_pdf(ctx, quantity, lo, hi, nbins, counts_ptr):
    """Asynchronous; counts_ptr: device int64[nbins + 2]."""
    _check(lib().hydro_diag_pdf(ctx, int(quantity), float(lo), float(hi), int(nbins),
                                counts_ptr), "hydro_diag_pdf")


def hydro_diag_profile(ctx, axis, rho_lo, rho_hi, out_ptr):
    """Asynchronous; out_ptr: device float64[5 n_axis + 2]."""
    _check(lib().hydro_diag_profile(ctx, int(axis), float(rho_lo), float(rho_hi), out_ptr),
           "hydro_diag_profile")


def hydro_diag_spectrum(ctx, out_ptr):
    """Asynchronous; out_ptr: device float64[nx // 2 + 1]."""
    _check(lib().hydro_diag_spectrum(ctx, out_ptr), "hydro_diag_spectrum")


def hydro_diag_spectrum3d_workspace_bytes(ctx):
    """(workspace bytes, number of shells) of the shell spectrum."""
    b = _sz(0)
    nb = ctypes.c_int32(0)
    _check(lib().hydro_diag_spectrum3d_workspace_bytes(ctx, ctypes.byref(b), ctypes.byref(nb)),
           "hydro_diag_spectrum3d_workspace_bytes")
    return int(b.value), int(nb.value)


def hydro_diag_spectrum3d(ctx, work_ptr, work_bytes, out_ptr):
    """Asynchronous; work_ptr: device workspace; out_ptr: device float64[nshells]."""
    _check(lib().hydro_diag_spectrum3d(ctx, work_ptr, int(work_bytes), out_ptr),
           "hydro_diag_spectrum3d")


def hydro_burn(ctx, x_ptr, x_bytes, net, dt, nsub):
    """Asynchronous; x_ptr: device composition planes (see hydro_burn)."""
    _check(lib().hydro_burn(ctx, x_ptr, int(x_bytes), ctypes.byref(net), float(dt), int(nsub)),
           "hydro_burn")


def hydro_fill_ghosts(ctx):
    _check(lib().hydro_fill_ghosts(ctx), "hydro_fill_ghosts")


def hydro_amr_restrict(ctx, links):
    arr = make_links(links)
    _check(lib().hydro_amr_restrict(ctx, arr, len(links)), "hydro_amr_restrict")


def hydro_amr_prolong(ctx, links, ghosts_only=False):
    arr = make_links(links)
    _check(lib().hydro_amr_prolong(ctx, arr, len(links), int(bool(ghosts_only))),
           "hydro_amr_prolong")


AMR_NO_REFLUX = 0x1


def hydro_amr_cfl_dt(coarse_ctx, fine_ctx):
    dt = ctypes.c_double(0.0)
    _check(lib().hydro_amr_cfl_dt(coarse_ctx, fine_ctx, ctypes.byref(dt)), "hydro_amr_cfl_dt")
    return dt.value


def hydro_amr_step_workspace_bytes(coarse_ctx, fine_ctx, fine_ng):
    n = _sz(0)
    _check(lib().hydro_amr_step_workspace_bytes(coarse_ctx, fine_ctx, fine_ng, ctypes.byref(n)),
           "hydro_amr_step_workspace_bytes")
    return n.value


def hydro_amr_step(coarse_ctx, fine_ctx, links, fine_ng, dt, flags, ws_ptr, ws_bytes):
    arr = make_links(links)
    _check(lib().hydro_amr_step(coarse_ctx, fine_ctx, arr, len(links), fine_ng, dt, flags,
                                ws_ptr, ws_bytes), "hydro_amr_step")


class AmrLevels:
    """A coarse Batch and a fine Batch of whole stored boxes (see
    hydro_amr_step) joined by (fine, coarse, ox, oy, oz) links, stepped by
    hydro_amr_step with a workspace this object owns."""

    def __init__(self, coarse, fine, links, fine_ng):
        torch = _torch()
        self.coarse, self.fine = coarse, fine
        self.links = [tuple(k) for k in links]
        self.fine_ng = int(fine_ng)
        nbytes = hydro_amr_step_workspace_bytes(coarse.ctx, fine.ctx, self.fine_ng)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=coarse.pool.device)

    def step(self, dt, reflux=True):
        hydro_amr_step(self.coarse.ctx, self.fine.ctx, self.links, self.fine_ng, dt,
                       0 if reflux else AMR_NO_REFLUX,
                       ctypes.c_void_p(self.workspace.data_ptr()),
                       self.workspace.numel())

    def cfl_dt(self):
        """Largest stable coarse dt (see hydro_amr_cfl_dt)."""
        return hydro_amr_cfl_dt(self.coarse.ctx, self.fine.ctx)


def _pdf(obj, quantity, lo, hi, nbins, out):
    torch = _torch()
    dev = obj.state.device if hasattr(obj, "state") else obj.pool.device
    if out is None:
        out = torch.empty(max(int(nbins), 0) + 2, dtype=torch.int64, device=dev)
    hydro_diag_pdf(obj.ctx, quantity, lo, hi, nbins, ctypes.c_void_p(out.data_ptr()))
    return out


def hydro_get_time(ctx):
    t = ctypes.c_double(0.0)
    s = ctypes.c_int64(0)
    _check(lib().hydro_get_time(ctx, ctypes.byref(t), ctypes.byref(s)), "hydro_get_time")
    return t.value, s.value


def hydro_set_time(ctx, t, step):
    _check(lib().hydro_set_time(ctx, float(t), int(step)), "hydro_set_time")


def hydro_set_t_end(ctx, t_end):
    _check(lib().hydro_set_t_end(ctx, float(t_end)), "hydro_set_t_end")


def hydro_state_changed(ctx):
    _check(lib().hydro_state_changed(ctx), "hydro_state_changed")


def hydro_get_error(ctx):
    """HYDRO_OK or HYDRO_ENUMERIC (returned, not raised)."""
    rc = lib().hydro_get_error(ctx)
    if rc not in (HYDRO_OK, HYDRO_ENUMERIC):
        _check(rc, "hydro_get_error")
    return rc


def hydro_clear_error(ctx):
    _check(lib().hydro_clear_error(ctx), "hydro_clear_error")


def hydro_get_config(ctx):
    buf = ctypes.create_string_buffer(256)
    _check(lib().hydro_get_config(ctx, buf, 256), "hydro_get_config")
    return buf.value.decode()


def hydro_set_config(ctx, text):
    _check(lib().hydro_set_config(ctx, text.encode()), "hydro_set_config")


def hydro_time_sweeps(ctx, reps=10):
    ms = (ctypes.c_double * 3)()
    _check(lib().hydro_time_sweeps(ctx, int(reps), ms), "hydro_time_sweeps")
    return list(ms)


def hydro_profile_step(ctx, dt=DT_CFL):
    ms = (ctypes.c_double * 4)()
    _check(lib().hydro_profile_step(ctx, float(dt), ms), "hydro_profile_step")
    return list(ms)


def hydro_stream_ceiling(ctx, reps=10):
    ms = ctypes.c_double(0.0)
    _check(lib().hydro_stream_ceiling(ctx, int(reps), ctypes.byref(ms)), "hydro_stream_ceiling")
    return ms.value


def hydro_destroy(ctx):
    if ctx:
        _check(lib().hydro_destroy(ctx), "hydro_destroy")


# --------------------------------------------------------------------------
# owners
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def make_desc(shape, dx, gamma, cfl=0.8, bc=(PERIODIC,) * 6, grav=(0.0, 0.0, 0.0),
              precision=FP32, ng=0, flags=0):
    nz, ny, nx = shape
    d = HydroDesc()
    d.nx, d.ny, d.nz, d.ng = nx, ny, nz, ng
    if not hasattr(dx, "__len__"):
        dx = (dx, dx, dx)
    d.dx, d.dy, d.dz = (float(v) for v in dx)
    d.gamma = float(gamma)
    d.cfl = float(cfl)
    d.grav[:] = [float(g) for g in grav]
    d.bc[:] = [int(b) for b in bc]
    d.precision = int(precision)
    d.flags = int(flags)
    return d


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class Grid:
    """A grid stepped by libhydro.  `state` is a CUDA tensor of shape
    (5, nz+2ng, ny+2ng, nx+2ng), float32 or float64, contiguous; it is
    updated in place."""

    def __init__(self, state, dx, gamma, cfl=0.8, bc=(PERIODIC,) * 6,
                 grav=(0.0, 0.0, 0.0), ng=0, flags=0, stream=None):
        torch = _torch()
        if not state.is_cuda or not state.is_contiguous() or state.dim() != 4 \
                or state.shape[0] != 5:
            raise ValueError("state must be a contiguous CUDA tensor (5, nz, ny, nx)")
        if state.dtype == torch.float32:
            prec = FP32
        elif state.dtype == torch.float64:
            prec = FP64
        else:
            raise ValueError("state must be float32 or float64")
        shape = tuple(int(s) - 2 * ng for s in state.shape[1:])
        self.state = state
        self.desc = make_desc(shape, dx, gamma, cfl, bc, grav, prec, ng, flags)
        nbytes = hydro_workspace_bytes(self.desc)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=state.device)
        sp, self.stream = _stream_ptr(stream)
        self.ctx = hydro_init(self.desc, ctypes.c_void_p(state.data_ptr()),
                              state.numel() * state.element_size(),
                              ctypes.c_void_p(self.workspace.data_ptr()), nbytes, sp)

    # thin method forms of the C calls
    def step(self, dt=DT_CFL):
        hydro_step(self.ctx, dt)

    def sweep(self, axis, dt, fold_cfl=False):
        hydro_sweep(self.ctx, axis, dt, fold_cfl)

    def cfl_dt(self):
        return hydro_cfl_dt(self.ctx)

    def totals(self):
        return hydro_totals(self.ctx)

    def fill_ghosts(self):
        hydro_fill_ghosts(self.ctx)

    def pdf(self, quantity, lo, hi, nbins, out=None):
        """Device int64 tensor of nbins + 2 counts (see hydro_diag_pdf)."""
        return _pdf(self, quantity, lo, hi, nbins, out)

    def profile(self, axis, rho_lo, rho_hi, out=None):
        """Device float64 tensor of 5 n_axis + 2 values (see hydro_diag_profile)."""
        torch = _torch()
        n = (self.desc.nx, self.desc.ny, self.desc.nz)[axis] if axis in (0, 1, 2) else 0
        if out is None:
            out = torch.empty(5 * n + 2, dtype=torch.float64, device=self.state.device)
        hydro_diag_profile(self.ctx, axis, rho_lo, rho_hi, ctypes.c_void_p(out.data_ptr()))
        return out

    def burn(self, X, A, Ta, q, dt, nsub):
        """Reactive-source step on the composition tensor X (nspec planes
        shaped like the state's: (nspec, nz+2ng, ny+2ng, nx+2ng), the state's
        dtype, contiguous, on the same device); updates X and the energy."""
        if (not X.is_cuda or not X.is_contiguous() or X.dtype != self.state.dtype
                or tuple(X.shape[1:]) != tuple(self.state.shape[1:])):
            raise ValueError("X must be a contiguous CUDA tensor shaped like the state's planes")
        net = make_network(A, Ta, q)
        if X.shape[0] != net.nspec:
            raise ValueError("X must hold len(A) + 1 planes")
        hydro_burn(self.ctx, ctypes.c_void_p(X.data_ptr()), X.numel() * X.element_size(), net,
                   dt, nsub)

    def spectrum(self, out=None):
        """Device float64 tensor of nx // 2 + 1 values (see hydro_diag_spectrum)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.desc.nx // 2 + 1, dtype=torch.float64,
                              device=self.state.device)
        hydro_diag_spectrum(self.ctx, ctypes.c_void_p(out.data_ptr()))
        return out

    def spectrum3d(self, out=None, work=None):
        """Device float64 tensor of the shell spectrum (see
        hydro_diag_spectrum3d).  `work` (a device uint8 tensor of at least
        spectrum3d_workspace()[0] bytes) is allocated when not given."""
        torch = _torch()
        nbytes, nb = hydro_diag_spectrum3d_workspace_bytes(self.ctx)
        if work is None:
            work = torch.empty(nbytes, dtype=torch.uint8, device=self.state.device)
        if out is None:
            out = torch.empty(nb, dtype=torch.float64, device=self.state.device)
        hydro_diag_spectrum3d(self.ctx, ctypes.c_void_p(work.data_ptr()), work.numel(),
                              ctypes.c_void_p(out.data_ptr()))
        return out

    def spectrum3d_workspace(self):
        """(bytes, shells) of the shell spectrum."""
        return hydro_diag_spectrum3d_workspace_bytes(self.ctx)

    def time(self):
        return hydro_get_time(self.ctx)

    def set_time(self, t, step):
        hydro_set_time(self.ctx, t, step)

    def set_t_end(self, t_end):
        hydro_set_t_end(self.ctx, t_end)

    def state_changed(self):
        hydro_state_changed(self.ctx)

    def error(self):
        return hydro_get_error(self.ctx)

    def clear_error(self):
        hydro_clear_error(self.ctx)

    @property
    def config(self):
        return hydro_get_config(self.ctx)

    @config.setter
    def config(self, text):
        hydro_set_config(self.ctx, text)

    def time_sweeps(self, reps=10):
        return hydro_time_sweeps(self.ctx, reps)

    def profile_step(self, dt=DT_CFL):
        return hydro_profile_step(self.ctx, dt)

    def stream_ceiling(self, reps=10):
        return hydro_stream_ceiling(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None):
            hydro_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent patches in one pool tensor, stepped by one persistent
    launch per sweep.  `patches` is a list of tuples (offset_elems, nx, ny,
    nz, ng, dx, dy, dz[, row_pitch, slab_pitch, plane_pitch,
    interior_offset]); omitted or zero pitches mean the unpadded layout."""

    def __init__(self, pool, patches, gamma, cfl=0.8, bc=(PERIODIC,) * 6,
                 grav=(0.0, 0.0, 0.0), flags=0, stream=None):
        torch = _torch()
        if not pool.is_cuda or not pool.is_contiguous():
            raise ValueError("pool must be a contiguous CUDA tensor")
        prec = FP64 if pool.dtype == torch.float64 else FP32
        if pool.dtype not in (torch.float32, torch.float64):
            raise ValueError("pool must be float32 or float64")
        arr = (HydroPatch * len(patches))()
        for i, p in enumerate(patches):
            p = tuple(p) + (0,) * (12 - len(p))
            (arr[i].offset_elems, arr[i].nx, arr[i].ny, arr[i].nz, arr[i].ng,
             arr[i].dx, arr[i].dy, arr[i].dz, arr[i].row_pitch, arr[i].slab_pitch,
             arr[i].plane_pitch, arr[i].interior_offset) = p
        self.patches = arr
        self.pool = pool
        self.desc = make_desc((1, 1, 1), 1.0, gamma, cfl, bc, grav, prec, 0, flags)
        nbytes = hydro_batch_workspace_bytes(arr, self.desc)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=pool.device)
        sp, self.stream = _stream_ptr(stream)
        self.ctx = hydro_batch_init(arr, self.desc, ctypes.c_void_p(pool.data_ptr()),
                                    pool.numel() * pool.element_size(),
                                    ctypes.c_void_p(self.workspace.data_ptr()), nbytes, sp)

    def step(self, dt=DT_CFL):
        hydro_batch_step(self.ctx, dt)

    def times(self):
        """(t, dt) lists per patch (see hydro_batch_times)."""
        return hydro_batch_times(self.ctx, len(self.patches))

    def sweep(self, axis, dt, fold_cfl=False):
        hydro_sweep(self.ctx, axis, dt, fold_cfl)

    def cfl_dt(self):
        return hydro_cfl_dt(self.ctx)

    def totals(self):
        return hydro_totals(self.ctx)

    def fill_ghosts(self):
        hydro_fill_ghosts(self.ctx)

    def restrict(self, links):
        """links: (fine, coarse, ox, oy, oz) tuples (see hydro_amr_restrict)."""
        hydro_amr_restrict(self.ctx, links)

    def prolong(self, links, ghosts_only=False):
        """links: (fine, coarse, ox, oy, oz) tuples (see hydro_amr_prolong)."""
        hydro_amr_prolong(self.ctx, links, ghosts_only)

    def pdf(self, quantity, lo, hi, nbins, out=None):
        """Device int64 tensor of nbins + 2 counts over every patch."""
        return _pdf(self, quantity, lo, hi, nbins, out)

    def time(self):
        return hydro_get_time(self.ctx)

    def set_time(self, t, step):
        hydro_set_time(self.ctx, t, step)

    def set_t_end(self, t_end):
        hydro_set_t_end(self.ctx, t_end)

    def state_changed(self):
        hydro_state_changed(self.ctx)

    def error(self):
        return hydro_get_error(self.ctx)

    @property
    def config(self):
        return hydro_get_config(self.ctx)

    @config.setter
    def config(self, text):
        hydro_set_config(self.ctx, text)

    def time_sweeps(self, reps=10):
        return hydro_time_sweeps(self.ctx, reps)

    def profile_step(self, dt=DT_CFL):
        return hydro_profile_step(self.ctx, dt)

    def stream_ceiling(self, reps=10):
        return hydro_stream_ceiling(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None):
            hydro_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
