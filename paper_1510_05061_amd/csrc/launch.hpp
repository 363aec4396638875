// launch.hpp -- launch descriptors passed from the host runtime (capi.cpp)
// to the kernel launchers (kernels.hip), and the launcher entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace hydro {

// Which kernel a sweep launch runs.
constexpr int kPlaneNone = 0;  // one sweep along `axis`
constexpr int kPlaneXY = 1;    // fused x then y sweeps of patch z-planes
constexpr int kPlaneYX = 2;    // fused y then x sweeps of patch z-planes
constexpr int kWinXY = 3;      // fused x then y sweeps of single-grid windows
constexpr int kWinYX = 4;      // fused y then x sweeps of single-grid windows
constexpr int kZPlane = 5;     // z sweep of patch x-z planes in LDS (batches)

struct LaunchSweep {
  // pool: state or patch pool; patches/items: device tables (persistent)
  void* pool;
  const PatchDev* patches;
  PatchDev single;
  const WorkItem* items;
  int32_t nitems;
  int32_t nblocks;     // persistent: workgroups launched
  int32_t axis;
  int32_t bc_lo, bc_hi;
  int32_t do_cfl;
  double grav;
  double gamma;
  DevScalars* scal;
  SweepCfg cfg;
  int32_t persistent;
  int32_t fp64;
  int32_t xmode;       // x sweep: kXPacked, kXMulti or kXMarch
  int32_t dyn;         // persistent: ticket (1) or static round-robin (0) items
  int32_t plane;       // kPlaneNone, kPlaneXY or kPlaneYX
  int32_t plane_lds;   // fused plane sweeps: LDS bytes of the largest plane
  int32_t bc_lo_y, bc_hi_y;  // fused plane sweeps: boundary conditions along y
  double grav_y;             // fused plane sweeps: gravity along y
  // FP64 conserved totals of the updated cells (the last sweep of a step):
  // 6 sums per workgroup (direct launches) or per work item (persistent),
  // at tpart + 6 * index; null: none
  double* tpart;
  double gvec[3];            // gravity vector (totals: phi = -g . x)
  int32_t totals_only;       // dt = 0 and nothing stored: totals of the current state
  int32_t tot_cap;           // direct x launches with totals: at most this many
                             // workgroups, striding over the tiles (0: no cap)
  // persistent launches with a dt per patch (null: one dt in DevScalars):
  // patch p steps by pdt[p] and folds its CFL maximum into psmax[p]
  const double* pdt;
  unsigned long long* psmax;
  // out-of-place sweeps (single grid, fused x+y step): results go to dst,
  // laid out like pool (null: in place); only the z march and the window
  // sweeps take one
  void* dst;
  const WinDev* wins;  // window sweeps: the windows of a z-plane
  int32_t nwin;
};

// Partial sums a sweep launch writes (grid size or work items).
int64_t sweep_parts(const LaunchSweep& L);

// Sums n partials (6 doubles each) in a fixed order into scal->totals, using
// `slice` (6 * kTotalsSlices doubles) for the first level; with finish set it
// then ends a step (t += dt, next dt from the folded CFL maximum).  Always
// resets the persistent-sweep tickets.
constexpr int kTotalsSlices = 256;
hipError_t launch_totals_finish(const double* part, int64_t n, double* slice, DevScalars* s,
                                int finish, hipStream_t st);

struct LaunchReduce {
  const void* pool;
  const PatchDev* patches;
  PatchDev single;
  int32_t npatch;
  int32_t chunks;
  double gamma;
  double grav[3];
  DevScalars* scal;
  double* partials;
  int32_t fp64;
  unsigned long long* psmax;  // CFL maximum per patch (null: one in DevScalars)
  int32_t fold_only;          // CFL: leave the maximum folded (no dt from it yet)
};

// In-situ diagnostics (diag.hip).
constexpr int kQRho = 0, kQPressure = 1, kQSpeed = 2, kQMach = 3;  // hydro_quantity
constexpr int kPdfLdsBins = 8192;       // counters (bins + 2) kept in LDS up to this
constexpr int kPdfMaxBins = 1 << 24;
constexpr int kPdfMaxBlocks = 4096;     // single grid
constexpr int kPdfPatchBlocks = 4;      // batch: workgroups per patch
constexpr int kProfileChunksX = 256;    // partial sums per slab, slabs normal to x
constexpr int kProfileChunksYZ = 16;    // partial sums per slab, slabs normal to y or z
constexpr int kSpecBlocks = 2048;       // spectrum: workgroups (partial spectra)
constexpr int kSpecMaxLen = 1024;       // spectrum: longest x-line

struct LaunchDiag {
  const void* pool;
  const PatchDev* patches;  // batch: device patch table (PDF only); null: single grid
  PatchDev single;
  int32_t npatch;
  int32_t fp64;
  double gamma;
  // PDF
  int32_t quantity;
  int32_t nbins;
  double lo, w;                   // w = nbins / (hi - lo)
  unsigned long long* counts;     // device, nbins + 2
  // slab profiles (single grid)
  int32_t axis;
  int32_t chunks;                 // partial sums per slab
  double rho_lo, drho;            // f = clip((rho - rho_lo) / drho, 0, 1)
  double dx_axis;
  double* partials;               // device, n_axis * chunks * 5
  double* out;                    // device, n_axis * 5 + 2
};

// Operator-split reactive source (burn.hip).
constexpr int kBurnMaxSpecies = 20;

struct LaunchBurn {
  void* pool;                      // state (5 planes)
  void* X;                         // composition (nspec planes, laid out like the state's)
  PatchDev single;
  int32_t fp64;
  int32_t nspec;
  int32_t nsub;
  double gamma;
  double h;                        // dt / nsub
  double A[kBurnMaxSpecies - 1];   // link rate prefactors
  double Ta[kBurnMaxSpecies - 1];  // link activation temperatures
  double B[kBurnMaxSpecies];       // energy released in making species s from species 0
};

// AMR operators (amr.hip).
constexpr int kAmrFill = 0, kAmrRestrict = 1, kAmrProlong = 2, kAmrFlux = 3, kAmrReflux = 4,
              kAmrSnapshot = 5;
constexpr int kAmrLinksPerLaunch = 128;  // links passed by value in the kernel arguments
constexpr int kAmrMaxBlocks = 4096;

// A fine patch inside a coarse one (refinement ratio 2): fine cell (0,0,0)
// is the first child of coarse cell (ox, oy, oz).
struct AmrLink {
  int32_t fine, coarse;
  int32_t ox, oy, oz;
  int32_t pad;
};

struct LaunchAmr {
  int32_t op;                        // kAmrFill ... kAmrReflux
  int32_t fp64;
  void* pool;                        // coarse patches (fill: the patches)
  const PatchDev* patches;           // batch: device patch table; null: single grid
  PatchDev single;
  int32_t npatch;
  int32_t ng;                        // single grid: stored ghost layers
  int32_t bc[6];
  AmrLink links[kAmrLinksPerLaunch];
  int32_t nlinks;
  int32_t ghosts_only;               // prolongation: the fine ghost shell only
  int32_t shell;                     // ghost prolongation: walk the shell's parents only
                                     // (a thin shell), a variable per grid layer
  int64_t cells;                     // most cells one workgroup row walks (grid sizing)
  // Fine side of the links (null: the coarse pool and table).  finset > 0:
  // each fine table entry is a whole stored box without ghosts whose outer
  // finset layers are the ghost shell of the patch inside.
  void* fpool;
  const PatchDev* fpatches;
  int32_t finset;
  // prolongation: coarse data at theta in [0, 1] between cold (a copy of
  // the coarse cells it reads, taken at the start of the step at their pool
  // offsets) and the pool; cold null: pool.  kAmrSnapshot writes that copy
  // (cells within `margin` coarse cells of each link's covered box).
  const void* cold;
  int32_t margin;
  double theta;
  // flux registers (kAmrFlux, kAmrReflux): register of (link, axis, side,
  // coarse face, variable) at reg + ((((link0 + l) * 3 + axis) * 2 + side) *
  // maxface + face) * 5 + v, the fine registers nreg doubles further on
  double* reg;
  int64_t nreg;
  int32_t link0, maxface;
  int32_t axis, side;                // side: reflux only (flux does both)
  int32_t fine;                      // kAmrFlux: 1 fine faces, 0 coarse faces
  double dt;                         // kAmrFlux: sweep length
  double weight;                     // kAmrFlux: register += weight * flux
  double gamma, grav;                // kAmrFlux: sweep constants (gravity along axis)
  // device link table (null: `links`); with it one launch takes nlinks links
  // and link l of the launch is table entry l
  const AmrLink* dlinks;
};

// Writes n links into a device table, from kernel arguments (no host copy).
hipError_t launch_amr_upload(AmrLink* dst, const AmrLink* src, int32_t n, hipStream_t st);

hipError_t launch_sweep(const LaunchSweep& L, hipStream_t st);
hipError_t launch_amr(const LaunchAmr& L, hipStream_t st);
hipError_t launch_burn(const LaunchBurn& L, hipStream_t st);
hipError_t launch_diag_pdf(const LaunchDiag& L, hipStream_t st);
hipError_t launch_diag_profile(const LaunchDiag& L, hipStream_t st);
hipError_t launch_diag_spectrum(const LaunchDiag& L, hipStream_t st);

// Shell kinetic-energy spectrum of a single grid (spec3.hip).
constexpr int kSpec3BinBlocks = 2048;  // binning workgroups (partial spectra)
struct LaunchSpec3 {
  const void* pool;
  PatchDev single;
  int32_t fp64;
  int32_t cu_count;
  void* work;   // spec3_workspace_bytes(single) bytes, 256-byte aligned
  double* out;  // device, one value per shell
};
// every extent 2^a 3^b, from 1 to 1024
bool spec3_shape_ok(const PatchDev& P);
// workspace bytes; *nb receives the number of shells
size_t spec3_workspace_bytes(const PatchDev& P, int* nb);
hipError_t launch_diag_spectrum3d(const LaunchSpec3& L, hipStream_t st);
hipError_t launch_cfl(const LaunchReduce& L, hipStream_t st);
hipError_t launch_totals(const LaunchReduce& L, hipStream_t st);
hipError_t launch_finish_step(DevScalars* s, hipStream_t st);
hipError_t launch_finish_cfl(DevScalars* s, hipStream_t st);
hipError_t launch_init_scalars(DevScalars* s, double cfl, double t, double t_end,
                               hipStream_t st);
hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t st);
hipError_t launch_step_results(const DevScalars* s, double* out, hipStream_t st);
// Per-patch time steps: with advance, t[p] += dt[p] first; then dt[p] =
// cfl / psmax[p] capped by t_end - t[p] (DevScalars), and psmax[p] = 0.
hipError_t launch_patch_dt(double* t, double* dt, unsigned long long* psmax, int32_t n,
                           DevScalars* s, int advance, hipStream_t st);
// a[0..n) = v (a fill kernel: safe to capture in a graph)
hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t st);
hipError_t launch_set_time(DevScalars* s, double t, double t_end, hipStream_t st);
hipError_t launch_clear_error(DevScalars* s, hipStream_t st);
hipError_t launch_timing_begin(DevScalars* s, hipStream_t st);
hipError_t launch_timing_end(DevScalars* s, hipStream_t st);
hipError_t launch_reset_tickets(DevScalars* s, hipStream_t st);
hipError_t launch_stream(void* p, int64_t bytes, hipStream_t st);
int64_t x_tiles(const PatchDev& P, const SweepCfg& c);
int64_t x_grid(const PatchDev& P, const SweepCfg& c);
int64_t col_tiles(const PatchDev& P, int axis, const SweepCfg& c);
bool x_wave_ok(int n, int v);
int64_t x_pencils_per_tile(const PatchDev& P, const SweepCfg& c);
int plane_lds_bytes(const PatchDev& P, int fp64, int axis2 = 1);

}  // namespace hydro
