// layout.hpp -- structures shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace hydro {

constexpr int kBcPeriodic = 0;
constexpr int kBcOutflow = 1;
constexpr int kBcReflect = 2;

// Geometry of one grid or patch inside the caller's state buffer.  The
// state is 5 planes (rho, mx, my, mz, E); plane v of the patch starts at
// element base0 + v * plane, x is contiguous, y has stride sy, z stride sz.
// base0 points at interior cell (0,0,0).
struct PatchDev {
  int64_t base0;   // element offset of interior cell (0,0,0) of plane 0
  int64_t plane;   // elements per plane of this patch
  int32_t n[3];    // interior cells along x, y, z
  int32_t sy, sz;  // element strides along y and z
  int32_t ng;      // stored ghost layers on every side
  double dx[3];    // cell widths
  double idx[3];   // 1 / dx per axis, 0 along an axis with one cell
};

// Device-resident scalars at the start of the workspace.
struct DevScalars {
  double dt;                     // dt of the next step
  double t;                      // simulated time
  double t_end;                  // final time (<= 0: none)
  double cfl;                    // Courant number
  unsigned long long smax_bits;  // running max of signal speed / dx (FP64 bits)
  unsigned int error;            // sticky error bits (kErr*)
  unsigned int tdone;            // totals reduction: workgroups finished
  unsigned int tickets[4];       // persistent-sweep work tickets
  double saved[2];               // dt, t saved around timing runs
  double totals[6];              // last FP64 totals
  double pad1[2];
};

constexpr unsigned kErrState = 1u;   // rho <= 0, p <= 0 or non-finite after an update
constexpr unsigned kErrSpeed = 2u;   // max signal speed zero or non-finite

// A unit of work of a persistent sweep: tile `tile` of patch `patch`.
struct WorkItem {
  int32_t patch;
  int32_t tile;
};

// A window of the fused x+y sweeps of a single grid: kWinEdge cells along
// x by win_rows() rows along y of a z-plane, whose inner part is written
// (64 x 64 FP32 cells or 64 x 32 FP64 cells: 80 KiB of LDS either way).
// The sweeps need two cells on each side of a written cell, so a window
// reaches two cells past its written part, except where it meets a domain
// edge that is not periodic (there the pencil ends apply that boundary
// condition).
constexpr int kWinEdge = 64;
constexpr int kWinHalo = 2;
constexpr int win_rows(bool fp64) { return fp64 ? 32 : 64; }
struct WinDev {
  int32_t x0, y0;          // cell (0, 0) of the window in the grid (wrapped on
                           // periodic axes: x0 may be -2)
  int32_t ox0, ox1;        // written columns [ox0, ox1), window-relative
  int32_t oy0, oy1;        // written rows [oy0, oy1)
  int32_t bx_lo, bx_hi;    // pencil-end conditions along x (hydro_bc; periodic
  int32_t by_lo, by_hi;    // where the window's end is not a domain edge)
};

// Kinds of sweep kernel (SweepCfg::kind).
constexpr int kLaneRunKind = 0;   // x: lane runs, whole pencils per workgroup
constexpr int kColumnKind = 1;    // y, z: column march
constexpr int kXMarchKind = 2;    // x: one pencil per wave, marched in chunks

// Shapes of the x lane-run launch.
constexpr int kXPacked = 0;  // every pencil inside one wave
constexpr int kXMulti = 1;   // a pencil spans several waves of a workgroup
constexpr int kXMarch = 2;   // chunked march (kXMarchKind)

// Kernel configuration of one sweep axis.
struct SweepCfg {
  int32_t kind;    // kLaneRunKind, kColumnKind or kXMarchKind
  int32_t v;       // lane runs: cells per lane (1, 2, 4)
  int32_t block;   // threads per workgroup
  int32_t q;       // column march: columns per tile; x march: workgroup cap (0: none)
  int32_t s;       // column march: segments per column
  int32_t pad;
};

}  // namespace hydro
