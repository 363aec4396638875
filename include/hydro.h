/*
 * hydro.h -- C ABI of libhydro: the finite-volume compressible-Euler zone
 * update on one AMD Instinct MI355X (gfx950).
 *
 * Zingale, Calder, Malone & Timmes (arXiv:1510.05061) model an exploding
 * star as a fluid on a decomposed grid, with nearest-neighbour and global
 * communication every timestep (introduction; section "Capabilities
 * needed"), and argue for suites of independent runs (section "Increasing
 * computing power"; capacity computing under "Capabilities needed").  The
 * paper gives no numerical method.  This library implements the standard
 * one for that setting:
 *   - ideal-gas Euler equations, U = (rho, mx, my, mz, E),
 *     p = (gamma-1)(E - |m|^2/(2 rho));
 *   - primitive piecewise-linear reconstruction with the MC limiter
 *     (van Leer 1977) and the MUSCL-Hancock predictor (Toro 2009 sec. 14.4);
 *   - HLLC fluxes with Davis wave speeds (Toro, Spruce & Speares 1994;
 *     Toro 2009 sec. 10.4);
 *   - conservative, dimensionally split sweeps: x,y,z on even steps and
 *     z,y,x on odd steps (Strang 1968); a sweep along an axis with one cell
 *     is skipped;
 *   - a constant gravity source (predictor half kick, time-centred momentum
 *     source, energy source from the face mass fluxes);
 *   - dt = cfl / max over cells and active axes of (|v_d| + c) / dx_d, a
 *     global max reduction kept in FP64 on the device.
 *
 * Data layout (caller-owned device memory, never allocated or freed here):
 *   state = 5 planes (rho, mx, my, mz, E); each plane holds
 *   (nz+2ng)(ny+2ng)(nx+2ng) elements, x fastest, then y, then z; plane v
 *   starts at element v * plane_elems.  Elements are float (HYDRO_FP32) or
 *   double (HYDRO_FP64).  Interior cell (i,j,k) sits at stored index
 *   (i+ng, j+ng, k+ng).  Stored ghost layers (ng > 0) are never read or
 *   written: boundary conditions are applied on the fly.  The state pointer
 *   must be 16-byte aligned; 256-byte alignment is recommended.
 *
 * Precision: HYDRO_FP32 keeps the state and the per-zone arithmetic in FP32
 * while dt, t, the CFL maximum and the conserved totals are FP64.
 * HYDRO_FP64 runs everything in FP64.
 *
 * Streams and synchronisation: every call enqueues on the stream given at
 * init (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) and
 * returns without waiting, except the calls marked "Synchronous", which
 * wait for that stream.  A context is not thread-safe; separate contexts on
 * separate streams may run concurrently if their buffers do not overlap.
 *
 * Errors: every function returns a hydro_status; no C++ exception crosses
 * this interface.  hydro_last_error() describes the last failure of the
 * calling thread.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_ABI_VERSION 3

typedef enum hydro_status {
  HYDRO_OK = 0,
  HYDRO_EINVAL = 1,   /* bad descriptor, argument, pointer or workspace size */
  HYDRO_EDEVICE = 2,  /* a HIP runtime call failed */
  HYDRO_ENUMERIC = 3, /* sticky device flag: rho <= 0, p <= 0 or a non-finite
                         value after an update, or a zero/non-finite signal
                         speed */
  HYDRO_ESTATE = 4    /* call out of order (e.g. a batch call on a grid ctx) */
} hydro_status;

typedef enum hydro_bc {
  HYDRO_BC_PERIODIC = 0, /* wrap; must be set on both sides of an axis */
  HYDRO_BC_OUTFLOW = 1,  /* zero gradient: ghosts copy the edge cell */
  HYDRO_BC_REFLECT = 2   /* mirror: ghost -k copies cell k-1 with the normal
                            momentum negated; gravity is mirrored too */
} hydro_bc;

typedef enum hydro_precision { HYDRO_FP32 = 0, HYDRO_FP64 = 1 } hydro_precision;

/* hydro_desc.flags */
#define HYDRO_FLAG_NO_GRAPH 0x1u /* launch kernels one by one, no hipGraph */
#define HYDRO_FLAG_NO_TUNE 0x2u  /* skip the autotuner and its cache; use the
                                    built-in default configuration */
#define HYDRO_BATCH_PER_PATCH_DT 0x4u /* batches: every patch keeps its own
                                    time and steps with its own CFL dt (a
                                    suite of independent runs) instead of
                                    one dt, the minimum over patches */
#define HYDRO_FLAG_FUSE_XY 0x8u /* single grids with even x and y extents,
                                    x >= 64, y >= 64 (FP32) or 32 (FP64), and
                                    an active z axis: allow the fused x+y
                                    step, which sweeps x and y together in
                                    windows of 64 x 64 FP32 or 64 x 32 FP64
                                    cells of each z-plane held in LDS (one
                                    pass over HBM for two sweeps, the windows
                                    overlapping by two cells on each side).
                                    The windows
                                    write to a second buffer laid out like the
                                    state, which the workspace then holds
                                    (hydro_workspace_bytes grows by the
                                    state's size); a step runs x+y into it and
                                    z back, or z into it and y+x back, so the
                                    state holds the result after every step.
                                    The autotuner keeps the fused step only
                                    where whole steps run faster; the result
                                    is the same bits either way.  Ignored
                                    where it does not apply. */

/* dt argument of hydro_step / hydro_batch_step: use the CFL dt held on the
 * device (no host synchronisation). */
#define HYDRO_DT_CFL 0.0

typedef struct hydro_desc {
  int32_t nx, ny, nz;  /* interior cells per axis (>= 1; an axis with more
                          than one cell needs at least 2) */
  int32_t ng;          /* stored ghost layers per side (>= 0) */
  double dx, dy, dz;   /* cell widths (> 0) */
  double gamma;        /* ratio of specific heats (> 1) */
  double cfl;          /* Courant number in (0, 1] */
  double grav[3];      /* constant gravitational acceleration */
  int32_t bc[6];       /* hydro_bc for x-lo, x-hi, y-lo, y-hi, z-lo, z-hi */
  int32_t precision;   /* hydro_precision */
  uint32_t flags;      /* HYDRO_FLAG_* */
} hydro_desc;

/* One patch of a batch.  The patch's 5 planes start at element
 * offset_elems of the pool (16-byte aligned), x fastest.  By default a plane
 * holds (nz+2ng)(ny+2ng)(nx+2ng) elements and interior cell (0,0,0) sits at
 * stored index (ng, ng, ng).  The four pitches below (in elements, 0 = that
 * default) describe a padded layout instead, e.g. rows whose interior starts
 * on a 128-byte boundary so that every row access is whole cache lines:
 *   row_pitch        elements between y-neighbours (>= nx + 2ng)
 *   slab_pitch       elements between z-neighbours (>= row_pitch (ny + 2ng))
 *   plane_pitch      elements between variables    (>= slab_pitch (nz + 2ng))
 *   interior_offset  elements from offset_elems to interior cell (0,0,0)
 *                    (>= ng (1 + row_pitch + slab_pitch))
 * The kernels address a plane with 32-bit byte offsets: (plane_pitch +
 * slab_pitch) elements must span less than 4 GiB (HYDRO_EINVAL otherwise);
 * the same bound holds for the plane of a single grid. */
typedef struct hydro_patch {
  int64_t offset_elems;
  int32_t nx, ny, nz, ng;
  double dx, dy, dz;
  int64_t row_pitch, slab_pitch, plane_pitch, interior_offset;
} hydro_patch;

typedef struct hydro_ctx hydro_ctx;

/* ABI version of the loaded library (HYDRO_ABI_VERSION). */
int hydro_abi_version(void);

/* Human-readable name of a status code (static storage). */
const char* hydro_strerror(int status);

/* Description of the last failure on the calling thread (static storage,
 * valid until the next call on that thread). */
const char* hydro_last_error(void);

/* Bytes of device workspace hydro_init needs for this descriptor.  The
 * workspace holds the device scalars (dt, t, CFL maximum, error flag, work
 * tickets) and reduction partials (the FP64 totals of each step). */
int hydro_workspace_bytes(const hydro_desc* d, size_t* bytes);

/* The star as a fluid on a grid (paper, introduction): a context binds the
 * zone update to one grid.
 * Bind a context to caller-owned device buffers.  `state` is the grid
 * (layout above) of `state_bytes` bytes (at least 5 planes), `workspace` at
 * least hydro_workspace_bytes bytes (16-byte aligned), `stream` a
 * hipStream_t (NULL: the null stream).  Validates the
 * descriptor, picks the kernel configuration (autotuner cache, or a timing
 * search with dt = 0, which leaves the state bit for bit), captures the
 * even- and odd-step graphs, sets t = 0 and step = 0.  Synchronous.
 * On success *out owns only host objects and hipGraphExecs; free it with
 * hydro_destroy.  Errors: HYDRO_EINVAL, HYDRO_EDEVICE. */
int hydro_init(const hydro_desc* d, void* state, size_t state_bytes, void* workspace,
               size_t ws_bytes, void* stream, hydro_ctx** out);

/* The global reduction every timestep needs (paper, section "Capabilities
 * needed": global communication each timestep), here the CFL maximum.
 * Compute dt = cfl / max signal speed from the current state (capped so
 * that t does not pass t_end when a final time is set), store it on the
 * device for the next HYDRO_DT_CFL step and return it in *dt.  Synchronous.
 * Returns HYDRO_ENUMERIC (and *dt = 0) when the sticky error flag is set or
 * the state holds rho <= 0, p <= 0 or a non-finite value. */
int hydro_cfl_dt(hydro_ctx* c, double* dt);

/* The zone update of the fluid (paper, introduction), with the
 * nearest-neighbour data of every sweep and the step's global reductions
 * (section "Capabilities needed": the CFL maximum for the next dt and the
 * FP64 conserved totals, both folded into the last sweep).
 * Enqueue one full split step of the grid.  dt > 0 uses exactly that dt;
 * dt == HYDRO_DT_CFL uses the CFL dt on the device (computed from the
 * current state before the first such step, then by the last sweep of each
 * step).  Advances t by dt and the step counter by one; the counter's parity
 * sets the sweep order.  Asynchronous.  Errors: HYDRO_EINVAL (dt < 0 or not
 * finite), HYDRO_EDEVICE, HYDRO_ESTATE (batch context). */
int hydro_step(hydro_ctx* c, double dt);

/* One split step of a single grid that allocates nothing, for callers that
 * cannot allocate device memory: code under stream capture, tight serving
 * loops, harnesses that forbid allocation.  It runs exactly the step that
 * hydro_step runs for a context made by hydro_init from the same descriptor
 * with HYDRO_FLAG_NO_TUNE (the built-in kernel configuration: the same
 * bits), without a context or a workspace.  Its device scalars and totals
 * partials live in a static device array of HYDRO_NOALLOC_SCRATCH_BYTES that
 * every GPU the library runs on holds from the first call on it until the
 * process ends (its address is looked up on that first call).  All calls on
 * one GPU share the array, which keeps the last call's contents (each call
 * resets what it reads): calls that overlap in time on one GPU (other
 * streams or threads) race, and must not be made.
 *   d, state, state_bytes  as for hydro_init (d->flags is ignored);
 *   dt                     > 0: that dt; HYDRO_DT_CFL: the CFL dt of the
 *                          state, reduced on the device first;
 *   step                   >= 0; its parity sets the sweep order;
 *   stream                 a hipStream_t (NULL: the null stream);
 *   out                    NULL, or a caller-owned DEVICE array of 9 doubles
 *                          (8-byte aligned): out[0] the dt taken, out[1] the
 *                          CFL dt of the new state, out[2..7] the FP64
 *                          totals of the new state (as hydro_totals), out[8]
 *                          the step's sticky error bits (0: none).
 * Asynchronous on `stream`.  Errors: HYDRO_EINVAL (as hydro_init; dt < 0 or
 * not finite; step < 0; a grid whose totals need more partial sums than the
 * array holds, about 21 500: the z sweep of the built-in configuration takes
 * one per 64 columns, so an x-y cross-section of more than about 1.38 M
 * cells), HYDRO_EDEVICE. */
#define HYDRO_NOALLOC_SCRATCH_BYTES (1u << 20)
int hydro_step_noalloc(const hydro_desc* d, void* state, size_t state_bytes, double dt,
                       int64_t step, void* stream, double* out);

/* Enqueue a single directional sweep along `axis` (0 = x, 1 = y, 2 = z)
 * with the given dt > 0 (or HYDRO_DT_CFL), without touching t or the step
 * counter.  fold_cfl != 0 also folds the CFL maximum of the updated cells
 * (as the last sweep of a step does).  For tests and per-kernel timing.
 * Asynchronous. */
int hydro_sweep(hydro_ctx* c, int axis, double dt, int fold_cfl);

/* Bytes of device workspace hydro_batch_init needs. */
int hydro_batch_workspace_bytes(const hydro_patch* p, int32_t n, const hydro_desc* common,
                                size_t* bytes);

/* Many independent grids in one launch per sweep: the suites of runs of
 * the paper's capacity-computing argument (section "Capabilities needed";
 * section "Increasing computing power": suites of simulations), and the
 * patches of adaptively refined levels.
 * Bind a context to a batch of n independent patches stored in the
 * caller-owned `pool` of `pool_bytes` bytes (offsets in p[]; every patch
 * must lie inside the pool and patches must not overlap).  `common` gives gamma, cfl, grav,
 * bc, precision and flags (its nx..dz are ignored).  The patch table and
 * the per-axis work lists (largest patches first) are written into the
 * workspace.  Synchronous.  Errors: HYDRO_EINVAL, HYDRO_EDEVICE. */
int hydro_batch_init(const hydro_patch* p, int32_t n, const hydro_desc* common, void* pool,
                     size_t pool_bytes, void* workspace, size_t ws_bytes, void* stream,
                     hydro_ctx** out);

/* Enqueue one split step of every patch of the batch: one persistent
 * launch per sweep direction over the whole work list.  By default with one
 * global dt, the minimum over patches (an AMR level without subcycling);
 * with HYDRO_BATCH_PER_PATCH_DT each patch with its own dt, patch p
 * advancing its own time by its own CFL dt (the suites of independent runs
 * of the paper's section "Capabilities needed"; each patch then takes the
 * steps it would take as a single grid, bit for bit).  dt > 0: that dt for
 * every patch; HYDRO_DT_CFL: the CFL dt on the device (per patch with the
 * flag).  The step counter, and so the sweep order, is shared.
 * Asynchronous. */
int hydro_batch_step(hydro_ctx* c, double dt);

/* Time and next dt of every patch of a batch (host arrays of n doubles;
 * without HYDRO_BATCH_PER_PATCH_DT every entry holds the batch's one t and
 * dt).  With the flag, hydro_get_time reports the earliest patch time and
 * hydro_cfl_dt the smallest patch dt, hydro_set_time sets every patch's
 * time, and hydro_set_t_end caps each patch's dt so that its own time lands
 * on t_end.  Synchronous.  Errors: HYDRO_EINVAL, HYDRO_ESTATE (single-grid
 * context), HYDRO_EDEVICE. */
int hydro_batch_times(hydro_ctx* c, double* t, double* dt);

/* The conserved totals, a global reduction of every timestep (paper,
 * section "Capabilities needed"), kept in FP64.
 * FP64 totals of the current state: sum over cells of (rho, mx, my, mz, E,
 * E + rho*phi) times the cell volume, phi = -(g . x) at cell centres with
 * the origin at the low corner of the grid (of each patch).  Every step
 * folds them into its last sweep: each workgroup (or batch work item) sums
 * the cells it updates and a final kernel adds those partial sums in a
 * fixed order, so the result is bitwise reproducible for a configuration.
 * After a step this returns the folded totals; after anything else that may
 * change the state (hydro_state_changed, hydro_sweep, hydro_set_time,
 * hydro_burn, AMR operators) it recomputes them with the same partition (the
 * last sweep of the previous step's order, run with dt = 0 and nothing
 * stored), so both give the same bits.  Synchronous. */
int hydro_totals(hydro_ctx* c, double out[6]);

/* In-situ diagnostics.  Large runs need their analysis done in situ (the
 * paper's discussion of the capabilities needed at the exascale); these are
 * standard diagnostics of stratified and shear-layer flows, each one pass
 * over the interior cells of the current state.  Cell quantities are
 * computed in FP64 with IEEE operations in this order (an FP32 state is
 * widened first, exactly):
 *   m2 = mx*mx + my*my + mz*mz,  ke = (0.5*m2)/rho,  p = (gamma-1)*(E - ke),
 *   speed = sqrt(m2)/rho,        mach = speed/sqrt((gamma*p)/rho). */
typedef enum hydro_quantity {
  HYDRO_Q_RHO = 0,       /* density */
  HYDRO_Q_PRESSURE = 1,  /* p */
  HYDRO_Q_SPEED = 2,     /* |v| */
  HYDRO_Q_MACH = 3       /* |v| / c */
} hydro_quantity;

/* PDF (histogram) of a hydro_quantity over every interior cell (of every
 * patch of a batch).  `counts` is a caller-owned DEVICE array of nbins + 2
 * int64 (8-byte aligned): with w = nbins / (hi - lo) (computed in FP64),
 *   counts[0]          cells with !(q >= lo)  (below the range, or NaN)
 *   counts[1 + b]      cells with b = floor((q - lo) * w), 0 <= b < nbins
 *   counts[nbins + 1]  cells at or above hi.
 * Counts are exact.  1 <= nbins <= 2^24; lo, hi finite with hi > lo.
 * Asynchronous on the context's stream (the array is overwritten).
 * Errors: HYDRO_EINVAL, HYDRO_EDEVICE. */
int hydro_diag_pdf(hydro_ctx* c, int quantity, double lo, double hi, int32_t nbins,
                   int64_t* counts);

/* Slab profiles of a single grid along `axis` (0 x, 1 y, 2 z): for each
 * slab s (cells of equal index along the axis) the means of rho, p, ke, f
 * and f(1-f), with the heavy-fluid fraction of a layer between densities
 * rho_lo < rho_hi f = min(max((rho - rho_lo)/(rho_hi - rho_lo), 0), 1).
 * `out` is a caller-owned DEVICE array of 5 n_axis + 2 doubles (8-byte
 * aligned): out[5 s + k] for the five fields, then
 *   out[5 n_axis]      mixing width W = dx_axis sum_s 4 <f>_s (1 - <f>_s)
 *   out[5 n_axis + 1]  mixedness Theta = sum_s <f(1-f)>_s / sum_s <f>_s (1 - <f>_s)
 *                      (0 when the denominator is 0).
 * Sums run in FP64 in a fixed order: bitwise reproducible for a shape.
 * Asynchronous on the context's stream.  Errors: HYDRO_EINVAL, HYDRO_ESTATE
 * (batch context), HYDRO_EDEVICE. */
int hydro_diag_profile(hydro_ctx* c, int axis, double rho_lo, double rho_hi, double* out);

/* One-dimensional kinetic-energy spectrum along x of a single grid's
 * velocity u = m/rho: with P[k] the mean over the x-lines of the power
 * |DFT_x(u_c)[k]|^2 summed over the three components (unnormalised DFT of
 * length N = nx, in FP64), `out` (a caller-owned DEVICE array of N/2 + 1
 * doubles, 8-byte aligned) receives
 *   out[0] = P[0]/(2N^2),  out[k] = P[k]/N^2 (0 < k < N/2),
 *   out[N/2] = P[N/2]/(2N^2) for even N,
 * so that sum_k out[k] = <|u|^2>/2 (Parseval).  nx must be 2^a 3^b with
 * 2 <= nx <= 1024 (HYDRO_EINVAL otherwise).  Partial sums run in a fixed
 * order: bitwise reproducible for a shape.  Asynchronous on the context's
 * stream.  Errors: HYDRO_EINVAL, HYDRO_ESTATE (batch context), HYDRO_EDEVICE. */
int hydro_diag_spectrum(hydro_ctx* c, double* out);

/* Shell kinetic-energy spectrum of a single grid (in-situ analysis, the
 * paper's discussion of the capabilities needed at the exascale; the shells
 * are those of the turbulence initial data's spectrum).  With u_hat_c the
 * unnormalised three-dimensional DFT of the velocity component u_c = m_c/rho
 * over the grid (N = nx ny nz cells, FP64) and k the signed integer
 * wavevector of each coefficient (k_i in (-n_i/2, n_i/2]), `out` (a
 * caller-owned DEVICE array of nshells doubles, 8-byte aligned) receives
 *   out[K] = sum over k with round(|k|) = K of sum_c |u_hat_c(k)|^2 / (2 N^2),
 * K = 0 .. nshells - 1, where nshells - 1 is the shell of the corner
 * wavevector (nx/2, ny/2, nz/2) (integer halves); sum_K out[K] = <|u|^2>/2
 * (Parseval).  Every extent must be 2^a 3^b with 1 <= n <= 1024
 * (HYDRO_EINVAL otherwise).  `work` is a caller-owned DEVICE buffer of at
 * least the bytes hydro_diag_spectrum3d_workspace_bytes reports (256-byte
 * aligned; about 28 bytes per cell: the three half spectra, their power and
 * the partial spectra); its contents are overwritten and need not be kept
 * between calls.  Sums run in a fixed order: bitwise reproducible for a
 * shape.  Asynchronous on the context's stream (the state and `work` must
 * stay valid until it completes).  Errors: HYDRO_EINVAL, HYDRO_ESTATE
 * (batch context), HYDRO_EDEVICE. */
int hydro_diag_spectrum3d_workspace_bytes(hydro_ctx* c, size_t* bytes, int32_t* nshells);
int hydro_diag_spectrum3d(hydro_ctx* c, void* work, size_t work_bytes, double* out);

/* Operator-split reactive source: a self-contained toy network.  The
 * paper's explosion models carry nuclear networks of 10-20 nuclei without
 * rates; this chain has the same shape of work, a stiff ODE per zone.
 * Species 0 -> 1 -> ... -> nspec-1 (the last stable); link i converts
 * species i to i+1 at k_i = A[i] exp(-Ta[i] / T), T = p/rho of the zone
 * (code units, held fixed over the step), releasing q[i] per unit mass.
 * The step integrates the mass fractions over dt with nsub backward-Euler
 * substeps (exact forward substitution; L-stable; sum of X conserved) in
 * FP64 and raises the total energy by rho sum_s B_s (X_s - X_s^0),
 * B_s = q[0] + ... + q[s-1]. */
#define HYDRO_MAX_SPECIES 20
typedef struct hydro_network {
  int32_t nspec;                     /* 2 .. HYDRO_MAX_SPECIES */
  int32_t pad;
  double A[HYDRO_MAX_SPECIES - 1];   /* link rate prefactors, >= 0, finite */
  double Ta[HYDRO_MAX_SPECIES - 1];  /* link activation temperatures, finite */
  double q[HYDRO_MAX_SPECIES - 1];   /* link specific energy releases, finite */
} hydro_network;

/* One reactive-source step of a single grid.  `X` is a caller-owned DEVICE
 * array of nspec composition planes, each laid out exactly like one plane
 * of the state (same element type, plane size, pitches and ghost layers;
 * plane s starts s * plane-size elements after X), `x_bytes` its size.  X
 * and the energy plane are updated in place; rho and momentum unchanged.
 * dt >= 0 finite, 1 <= nsub <= 1000000.  Asynchronous on the context's
 * stream.  Errors: HYDRO_EINVAL, HYDRO_ESTATE (batch context), HYDRO_EDEVICE. */
int hydro_burn(hydro_ctx* c, void* X, size_t x_bytes, const hydro_network* net, double dt,
               int32_t nsub);

/* AMR operators around the batched patches (refinement ratio 2).  The
 * paper's codes run the hydrodynamics on adaptively refined grids; these are
 * the standard conservative operators between levels.  The sweeps apply
 * the physical boundary conditions on the fly and never read stored
 * ghosts: these serve the layers around the step (regridding, coarse-fine
 * exchange, output, checkpoints).  All are asynchronous on the context's
 * stream and reproduce their definitions' operations in order (results
 * bitwise equal to a plain FP64 evaluation, rounded once to the state's
 * precision). */

/* The stored ghost layers of a single grid (ng > 0) or of every patch, from
 * the interior under the context's boundary conditions, axis by axis:
 * periodic wraps, outflow copies the edge cell, reflect mirrors (ghost -k
 * copies cell k-1, with period 2n beyond the interior) and negates the
 * momentum normal to the reflecting side.  Errors: HYDRO_EINVAL,
 * HYDRO_EDEVICE. */
int hydro_fill_ghosts(hydro_ctx* c);

/* A fine patch inside a coarse one of the same batch: fine interior cell
 * (0,0,0) is the first child of coarse interior cell (ox, oy, oz); the fine
 * cells are half as wide.  Fine interior extents must be even. */
typedef struct hydro_amr_link {
  int32_t fine, coarse;  /* patch indices */
  int32_t ox, oy, oz;
  int32_t pad;
} hydro_amr_link;

/* Restriction: every coarse cell covered by a fine patch becomes the mean
 * of its 2x2x2 children (summed in (dz, dy, dx) order, times 1/8).  The
 * covered cells must lie in the coarse interior.  Links of one call must not
 * write overlapping cells, nor read cells another link writes.  Errors:
 * HYDRO_EINVAL, HYDRO_ESTATE (single-grid context), HYDRO_EDEVICE. */
int hydro_amr_restrict(hydro_ctx* c, const hydro_amr_link* links, int32_t n);

/* Prolongation: fine cells from the coarse patch by MC-limited linear
 * reconstruction, conservative (the eight children average to the parent):
 *   child = ((U + s_x D_x) + s_y D_y) + s_z D_z,  s = -1/4 or +1/4,
 * D = sign(a) min(2|a|, 2|b|, |a+b|/2) when the coarse one-sided
 * differences a, b have a positive product, else 0.  ghosts_only = 0 fills
 * the fine interior; 1 fills only the fine ghost shell (coarse-fine ghost
 * exchange).  The coarse cells used (parents and their neighbours, coarse
 * ghosts included: fill them first) must lie in the coarse patch's stored
 * region.  Same independence rule and errors as hydro_amr_restrict. */
int hydro_amr_prolong(hydro_ctx* c, const hydro_amr_link* links, int32_t n, int ghosts_only);

/* One subcycled step of a two-level hierarchy with refluxing (Berger &
 * Colella 1989; the paper's codes refine adaptively without fixing these
 * operators).  `coarse` is a batch of coarse patches stepped with its own
 * boundary conditions.  `fine` is a batch whose patch i is the whole stored
 * box of fine patch i described without ghosts: extents n + 2 fine_ng and
 * ng = 0, so its outer fine_ng layers (fine_ng >= 2) are the patch's ghost
 * shell and are swept with it (the boundary conditions of `fine` act only
 * on that shell's outer edge).  links[i].fine indexes `fine`,
 * links[i].coarse indexes `coarse`; fine interior cell (0,0,0) is the first
 * child of coarse interior cell (ox, oy, oz).  n must equal the number of
 * fine patches, each linked once.  The step, on the stream both contexts
 * share:
 *   1. the coarse batch takes one Strang step of dt (sweep order by its
 *      step counter), each sweep preceded by a flux register of the coarse
 *      faces on every fine patch's boundary (R_c = dt F);
 *   2. the fine batch takes two steps of dt/2 (orders by its counter); before
 *      substep s its ghost shells are prolonged (as hydro_amr_prolong) from
 *      the coarse data interpolated in time, U_old + (s/2)(U - U_old) (U_old
 *      itself for s = 0), and
 *      each sweep registers the mean over the 2x2 fine faces of every coarse
 *      face, summed in (t2, t1) order, times dt/2 (R_f);
 *   3. restriction of every fine interior onto the coarse cells it covers;
 *   4. refluxing (unless HYDRO_AMR_NO_REFLUX): the uncovered coarse cell
 *      across each coarse-fine face gains (R_c - R_f)/dx on a patch's low
 *      side and (R_f - R_c)/dx on its high side, per axis x, y, z, low sides
 *      before high sides.
 * Both levels need every axis > 1 cell, equal precision, gamma and gravity,
 * fine cells exactly half as wide, even fine interior extents, each patch
 * at least ceil(fine_ng/2) + 1 coarse cells inside the coarse interior, and
 * patches on one coarse patch at least one coarse cell apart along some
 * axis.  dt > 0 (for example min(coarse CFL dt, 2 x fine CFL dt)).  Both
 * step counters advance (by 1 and 2) and the device dt of each context is
 * recomputed before its next HYDRO_DT_CFL step.  The workspace (256-byte
 * aligned, hydro_amr_step_workspace_bytes) holds the start-of-step copy of
 * the coarse cells that prolongation reads (at the coarse pool's offsets, so
 * it is as large as the pool), the registers and the link table.  Asynchronous.  Errors: HYDRO_EINVAL, HYDRO_ESTATE
 * (not batches, work lists out of date), HYDRO_EDEVICE. */
#define HYDRO_AMR_NO_REFLUX 0x1u

/* The largest stable coarse dt of the two-level step: min(coarse CFL dt,
 * 2 x fine CFL dt), each the CFL dt of its batch's current state (as
 * hydro_cfl_dt, which it also stores on each context's device), since the
 * fine level takes two substeps of dt/2.  Synchronous.  Errors:
 * HYDRO_EINVAL, HYDRO_ESTATE (not batches), HYDRO_ENUMERIC, HYDRO_EDEVICE. */
int hydro_amr_cfl_dt(hydro_ctx* coarse, hydro_ctx* fine, double* dt);

int hydro_amr_step_workspace_bytes(const hydro_ctx* coarse, const hydro_ctx* fine,
                                   int32_t fine_ng, size_t* bytes);
int hydro_amr_step(hydro_ctx* coarse, hydro_ctx* fine, const hydro_amr_link* links, int32_t n,
                   int32_t fine_ng, double dt, uint32_t flags, void* workspace,
                   size_t ws_bytes);

/* Simulated time and step counter (Synchronous).  hydro_set_time restores a
 * checkpoint: the counter's parity selects the next sweep order, and the
 * device dt is recomputed before the next HYDRO_DT_CFL step. */
int hydro_get_time(hydro_ctx* c, double* t, int64_t* step);
int hydro_set_time(hydro_ctx* c, double t, int64_t step);

/* Final time: HYDRO_DT_CFL steps are shortened so that t lands on t_end,
 * and become empty afterwards.  t_end <= 0 removes the cap. */
int hydro_set_t_end(hydro_ctx* c, double t_end);

/* Declare that the caller changed the state behind the library's back (the
 * device dt is then recomputed before the next HYDRO_DT_CFL step). */
int hydro_state_changed(hydro_ctx* c);

/* Sticky device error flag, read synchronously: HYDRO_OK or HYDRO_ENUMERIC.
 * hydro_clear_error resets it. */
int hydro_get_error(hydro_ctx* c);
int hydro_clear_error(hydro_ctx* c);

/* Kernel configuration as text, parts separated by ';' (any subset may be
 * given to hydro_set_config; the rest keeps its value):
 *   x:v=V,b=B[,m=1[,g=G]]  x sweep: V cells per lane (1, 2, 4), B threads
 *                          per workgroup; m=1 selects the chunked march (one
 *                          pencil per wave), G caps its grid (0: none);
 *                          without m the lane-run sweep;
 *   y:q=Q,s=S  z:q=Q,s=S   column marches: Q columns per tile, S segments;
 *   p:g=G,d=D,f=F          batch: G persistent workgroups, D = 1 ticket or
 *                          0 round-robin work items, F = 1 fuses the x and
 *                          y sweeps per patch z-plane;
 *   w:v=V,b=B              batch, fused plane kernel: V cells per lane, B
 *                          threads per workgroup.
 * hydro_get_config writes at most len bytes including the NUL.
 * hydro_set_config replaces it (validated: HYDRO_EINVAL for a shape the
 * kernels do not support, e.g. f=1 when a patch plane exceeds 80 KiB; work
 * lists are rebuilt and graphs re-captured).  Every valid configuration
 * gives the same bits. */
int hydro_get_config(hydro_ctx* c, char* buf, size_t len);
int hydro_set_config(hydro_ctx* c, const char* cfg);

/* Mean device time in milliseconds of each sweep kernel (x, y, z) over
 * `reps` launches, measured with hipEvents on the context's stream with
 * dt = 0 (the state is unchanged bit for bit).  An inactive axis reports 0.
 * Synchronous. */
int hydro_time_sweeps(hydro_ctx* c, int reps, double ms[3]);

/* One full split step like hydro_step / hydro_batch_step, launched kernel
 * by kernel with a hipEvent pair around each sweep on the context's stream;
 * ms[0..2] receive the device time of the x, y and z sweep kernels (0 for
 * an inactive axis; with the fused batch plane sweeps ms[0] holds the fused
 * x and y launch and ms[1] is 0) and ms[3] their sum.  For measurement; it
 * waits after each sweep, so the step as a whole runs slower than
 * hydro_step.  Synchronous. */
int hydro_profile_step(hydro_ctx* c, double dt, double ms[4]);

/* Mean device time in milliseconds of one in-place streaming pass over the
 * context's whole state (or pool) buffer: every 16-byte word read and
 * written back unchanged, with no arithmetic.  The memory-only ceiling a
 * sweep kernel over the same bytes can approach.  The state is unchanged.
 * Synchronous. */
int hydro_stream_ceiling(hydro_ctx* c, int reps, double* ms);

/* Release the host objects of a context (device buffers stay with the
 * caller).  Waits for the context's stream. */
int hydro_destroy(hydro_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H */
