// kernels.hip -- HIP kernels (gfx950, wave64) of the split compressible-Euler
// zone update: directional sweeps, CFL reduction, FP64 totals, step
// bookkeeping.  The per-zone arithmetic is in euler.hpp.
//
// Two sweep shapes, both in place and race-free:
//  * lane runs (x, the contiguous axis): a workgroup owns whole x-pencils;
//    lane l of a pencil holds V consecutive cells, loads them coalesced, and
//    trades its edge primitives, its last face state and its first face flux
//    with its neighbours through LDS.  Every load of a pencil happens before
//    the first barrier and every store after the last, so no other lane can
//    see a half-updated pencil.
//  * column marches (y and z, strided axes): lanes sit on consecutive
//    columns (consecutive x), so every row access of a wave is one coalesced
//    segment; each column is cut into S segments owned by S waves of the
//    same workgroup.  A thread loads the two halo cells on each side of its
//    segment, the workgroup barriers, then each thread marches through its
//    own cells keeping a three-cell window in registers.  A cell is written
//    only by its owner and only after every thread has taken its halo copy.
// Boundary conditions are applied on the fly (wrap, copy, mirror); stored
// ghost layers are never read.
//
// The last sweep of a step also folds max_d (|v_d| + c) / dx_d of every
// updated cell into one FP64 atomic max (on the bit pattern of a
// non-negative double, which orders like the value), the "global
// communication each timestep" of the paper's section "Capabilities needed".
#include <hip/hip_runtime.h>

#include "euler.hpp"
#include "launch.hpp"
#include "layout.hpp"

namespace hydro {

template <class T>
struct SweepArgs {
  T* pool;                   // state buffer (single grid) or patch pool
  const PatchDev* patches;   // patch table (persistent launches)
  PatchDev single;           // the grid (direct launches)
  const WorkItem* items;     // work list (persistent launches)
  int32_t nitems;
  int32_t bc_lo, bc_hi;      // boundary conditions along the sweep axis
  int32_t do_cfl;            // fold the CFL maximum of the updated cells
  int32_t q, s;              // column march: columns per tile, segments
  int32_t dyn;               // persistent launches: 1 ticket scheduling, 0 static
  int32_t bc_lo_y, bc_hi_y;  // fused plane sweeps: boundary conditions along y
  double grav;               // gravity along the sweep axis (plane sweeps: x)
  double grav_y;             // fused plane sweeps: gravity along y
  double gamma;
  DevScalars* scal;
  double* tpart;             // totals partials (null: no totals)
  double gvec[3];            // gravity vector (totals: phi = -g . x)
  int32_t tonly;             // totals of the current state: dt = 0, no stores
  const double* pdt;         // persistent: dt per patch (null: scal->dt)
  unsigned long long* psmax; // persistent: CFL maximum per patch
  T* dst;                    // out-of-place result (null: pool, in place)
  const WinDev* wins;        // window sweeps: the windows of a z-plane
  int32_t nwin;
};

// plane indices of (normal, transverse 1, transverse 2) momenta per axis
template <int AXIS> struct Rot;
template <> struct Rot<0> { static constexpr int n = 1, t1 = 2, t2 = 3; };
template <> struct Rot<1> { static constexpr int n = 2, t1 = 1, t2 = 3; };
template <> struct Rot<2> { static constexpr int n = 3, t1 = 1, t2 = 2; };

// The five planes of a grid or patch as uniform base pointers, addressed by
// a 32-bit byte offset inside a plane (one address VGPR shared by the five
// loads or stores of a cell; the runtime guarantees planes below 4 GiB).
template <class T, int AXIS>
struct Planes {
  char* r;
  char* n;
  char* t1;
  char* t2;
  char* e;
  __device__ __forceinline__ Planes(T* pool, const PatchDev& P) {
    T* p0 = pool + P.base0;
    const int64_t pl = P.plane;
    r = reinterpret_cast<char*>(p0);
    n = reinterpret_cast<char*>(p0 + Rot<AXIS>::n * pl);
    t1 = reinterpret_cast<char*>(p0 + Rot<AXIS>::t1 * pl);
    t2 = reinterpret_cast<char*>(p0 + Rot<AXIS>::t2 * pl);
    e = reinterpret_cast<char*>(p0 + 4 * pl);
  }
  __device__ __forceinline__ Cons<T> load(uint32_t b) const {
    Cons<T> U;
    U.r = *reinterpret_cast<const T*>(r + b);
    U.mn = *reinterpret_cast<const T*>(n + b);
    U.mt1 = *reinterpret_cast<const T*>(t1 + b);
    U.mt2 = *reinterpret_cast<const T*>(t2 + b);
    U.e = *reinterpret_cast<const T*>(e + b);
    return U;
  }
  __device__ __forceinline__ void store(uint32_t b, const Cons<T>& U) const {
    *reinterpret_cast<T*>(r + b) = U.r;
    *reinterpret_cast<T*>(n + b) = U.mn;
    *reinterpret_cast<T*>(t1 + b) = U.mt1;
    *reinterpret_cast<T*>(t2 + b) = U.mt2;
    *reinterpret_cast<T*>(e + b) = U.e;
  }
};

// V consecutive elements of one plane at byte offset b (aligned to the
// vector width; the runtime only picks V > 1 where rows are aligned).
template <class T, int V>
__device__ __forceinline__ void load_run(const char* base, uint32_t b, T (&o)[V]) {
  if constexpr (V == 1) {
    o[0] = *reinterpret_cast<const T*>(base + b);
  } else if constexpr (sizeof(T) * V <= 16) {
    typedef T vec __attribute__((ext_vector_type(V)));
    vec t = *reinterpret_cast<const vec*>(base + b);
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = t[i];
  } else {
    constexpr int H = 16 / sizeof(T);
    typedef T vec __attribute__((ext_vector_type(H)));
#pragma unroll
    for (int h = 0; h < V / H; ++h) {
      vec t = *reinterpret_cast<const vec*>(base + b + h * 16);
#pragma unroll
      for (int i = 0; i < H; ++i) o[h * H + i] = t[i];
    }
  }
}

template <class T, int V>
__device__ __forceinline__ void store_run(char* base, uint32_t b, const T (&o)[V]) {
  if constexpr (V == 1) {
    *reinterpret_cast<T*>(base + b) = o[0];
  } else if constexpr (sizeof(T) * V <= 16) {
    typedef T vec __attribute__((ext_vector_type(V)));
    vec t;
#pragma unroll
    for (int i = 0; i < V; ++i) t[i] = o[i];
    *reinterpret_cast<vec*>(base + b) = t;
  } else {
    constexpr int H = 16 / sizeof(T);
    typedef T vec __attribute__((ext_vector_type(H)));
#pragma unroll
    for (int h = 0; h < V / H; ++h) {
      vec t;
#pragma unroll
      for (int i = 0; i < H; ++i) t[i] = o[h * H + i];
      *reinterpret_cast<vec*>(base + b + h * 16) = t;
    }
  }
}

// Signal speed over the cell width, maxed over the active axes, of an
// updated cell, and its health.  U is rotated back to the physical frame
// (rho, mx, my, mz, E) first so that the result does not depend on which
// sweep computed it: the folded maximum of a step and a standalone
// reduction of the same state give the same bits.  id[] is 1/dx per
// physical axis, zero for an inactive axis.
template <class T, int AXIS>
__device__ __forceinline__ T cell_speed(const Cons<T>& S, const SweepConst<T>& k,
                                        const T id[3], bool& bad) {
  Cons<T> U;  // physical frame: mn holds mx, mt1 my, mt2 mz
  U.r = S.r;
  U.e = S.e;
  if (AXIS == 0) { U.mn = S.mn; U.mt1 = S.mt1; U.mt2 = S.mt2; }
  if (AXIS == 1) { U.mn = S.mt1; U.mt1 = S.mn; U.mt2 = S.mt2; }
  if (AXIS == 2) { U.mn = S.mt1; U.mt1 = S.mt2; U.mt2 = S.mn; }
  Prim<T> W = to_prim(U, k);
  bad |= !cell_ok(U, W);
  T c = sound(k.gamma, W.p, W.r);
  T s = (fabs_(W.u) + c) * id[0];
  s = fmax_(s, (fabs_(W.t1) + c) * id[1]);
  s = fmax_(s, (fabs_(W.t2) + c) * id[2]);
  return s;
}

template <class T>
__device__ __forceinline__ void inv_widths(const PatchDev& P, T id[3]) {
  for (int a = 0; a < 3; ++a) id[a] = T(P.idx[a]);  // 1/dx, made on the host
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax_(v, __shfl_xor(v, off));
  return v;
}

// Workgroup max of smax folded into the FP64 atomic at `dst` (the bit
// pattern of a non-negative double orders like the value; NaN propagates as
// the largest bits).  Every thread calls this; `red` holds one T per wave.
template <class T>
__device__ void block_max_fold(T smax, unsigned long long* dst, T* red) {
  T m = wave_max(smax);
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    T b = red[0];
    for (int i = 1; i < nw; ++i) b = fmax_(b, red[i]);
    double d = double(b);
    if (!(d >= 0.0)) d = __builtin_nan("");
    unsigned long long bits = (unsigned long long)__double_as_longlong(d);
    atomicMax(dst, bits);
  }
}

// The end of a persistent work item with a dt per patch: the item's CFL
// maximum into its patch's slot (smax restarts at 0); `red` is free again
// on return.
template <class T>
__device__ __forceinline__ void item_cfl(const SweepArgs<T>& a, int patch, T& smax, T* red) {
  if (a.pdt && a.do_cfl) {
    block_max_fold(smax, &a.psmax[patch], red);
    __syncthreads();
    smax = T(0);
  }
}

// dt of a persistent work item on `patch`
template <class T>
__device__ __forceinline__ double item_dt(const SweepArgs<T>& a, int patch, double dt) {
  return a.pdt && !a.tonly ? a.pdt[patch] : dt;
}

// Workgroup max of smax folded into the step's FP64 atomic (unless the
// launch folds it per patch), and the sticky error (one atomic per wave
// that saw a bad cell: a wave vote, no LDS).  `red` holds one T per wave.
template <class T>
__device__ void finish_block(DevScalars* scal, T smax, bool bad, bool do_cfl, T* red,
                             unsigned long long* dst = nullptr) {
  const bool wbad = __any(bad);
  if (wbad && (threadIdx.x & 63) == 0) atomicOr(&scal->error, kErrState);
  if (!do_cfl) return;
  block_max_fold(smax, dst ? dst : &scal->smax_bits, red);
}

// --------------------------------------------------------------------------
// FP64 conserved totals folded into the last sweep of a step
// --------------------------------------------------------------------------
//
// Each thread sums, in the order it updates its cells, the lab-frame
// rho, mx, my, mz, E and E + rho phi of every updated cell times the cell
// volume, phi = -(g . x) at the cell centre (origin at the low corner of the
// grid or patch).  A workgroup then reduces its threads' sums in a fixed
// tree into one partial per workgroup (direct launches) or per work item
// (persistent launches), so the summation order depends only on the launch
// configuration, never on scheduling: the totals are bitwise reproducible.

// Per-thread sums in registers.
struct TotR {
  double s[6];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int v = 0; v < 6; ++v) s[v] = 0.0;
  }
  __device__ __forceinline__ void add(int v, double x) { s[v] += x; }
  __device__ __forceinline__ double get(int v) const { return s[v]; }
};

// Per-thread sums in LDS, for kernels whose registers are spoken for: the
// six sums of thread t at p[kTotStride t + v].  One address register and an
// immediate offset per slot; a stride of 7 doubles (14 banks) puts the 64-bit
// slots of 16 consecutive lanes on 32 distinct banks.  Each thread adds only
// into its own slots, with LDS atomic adds that return nothing: no
// registers are held and the wave does not wait.
constexpr int kTotStride = 7;
struct TotL {
  double* p;
  __device__ __forceinline__ double* slot() const { return p + kTotStride * threadIdx.x; }
  __device__ __forceinline__ void zero() {
    double* q = slot();
#pragma unroll
    for (int v = 0; v < 6; ++v) q[v] = 0.0;
  }
  __device__ __forceinline__ void add(int v, double x) { atomicAdd(slot() + v, x); }
  __device__ __forceinline__ double get(int v) const { return slot()[v]; }
};

__device__ __forceinline__ double cell_volume(const PatchDev& P) {
  return P.dx[0] * P.dx[1] * P.dx[2];
}

__device__ __forceinline__ bool has_grav(const double g[3]) {
  return g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0;
}

// Cell (i, j, k) of patch P (interior indices along x, y, z) with its
// updated state S in the frame of sweep axis AXIS: adds q for q = rho, mx,
// my, mz, E and, with gravity, E + rho phi (the cell volume multiplies each
// thread's sums once, in tot_block).
template <class T, int AXIS, class Acc>
__device__ __forceinline__ void tot_add(Acc& t, const Cons<T>& S, const PatchDev& P,
                                        const double g[3], int i, int j, int k) {
  constexpr int vn = AXIS + 1, vt1 = AXIS == 0 ? 2 : 1, vt2 = AXIS == 2 ? 2 : 3;
  t.add(0, double(S.r));
  t.add(vn, double(S.mn));
  t.add(vt1, double(S.mt1));
  t.add(vt2, double(S.mt2));
  t.add(4, double(S.e));
  if (has_grav(g)) {  // else E + rho phi = E (tot_block)
    const double xc = (double(i) + 0.5) * P.dx[0];
    const double yc = (double(j) + 0.5) * P.dx[1];
    const double zc = (double(k) + 0.5) * P.dx[2];
    const double phi = -(g[0] * xc + g[1] * yc + g[2] * zc);
    t.add(5, double(S.e) + double(S.r) * phi);
  }
}

// v of every lane moved by the DPP pattern CTRL (one row of 16 lanes; every
// source lane lies in the destination's row), as two 32-bit moves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, 0xF, 0xF, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, 0xF, 0xF, false));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), lane));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a full wave, in a fixed tree: within each row of
// 16 lanes by register moves across lanes (pairs, quads, halves of a row,
// rows: each step adds a lane and its mirror, so every lane of a row ends
// with the same row sum), then the four row sums as (r0 + r1) + (r2 + r3).
// No LDS round trips: the reduction is four dependent adds and a few moves.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// The workgroup's sums, each thread's times the cell volume `vol`, in a
// fixed tree (lanes, then waves in order), into out[0..5]; every thread of
// the workgroup calls this.  `red` holds 6 doubles per wave (LDS).  The
// sums are cleared for the next work item.
template <class Acc>
__device__ void tot_block(Acc& t, double vol, double* out, double* red, bool grav) {
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const double w = wave_sum(t.get(grav || v < 5 ? v : 4) * vol);  // phi = 0: E + rho phi is E
    if ((threadIdx.x & 63) == 0) red[wid * 6 + v] = w;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double a = red[threadIdx.x];
    for (int w = 1; w < nw; ++w) a += red[w * 6 + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
  t.zero();
}

// LDS bytes per thread that tot_block_wide needs
constexpr int kTotWideBytes = 48;

// tot_block for kernels that reduce once per work item and have a large LDS
// area free at that point: every thread stores its six sums (times `vol`)
// at red[v B + t] (B threads); wave w then adds variable v = w, w + nw, ...
// over the threads in a fixed order (lane l takes t = l, l + 64, ...) and
// reduces its lanes with wave_sum.  About a quarter of tot_block's
// instructions per item, since only six waves reduce and each reduces one
// value.  `red` holds kTotWideBytes per thread.
template <class Acc>
__device__ void tot_block_wide(Acc& t, double vol, double* out, double* red, bool grav) {
  const int B = blockDim.x, nw = B >> 6;
  const int wid = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 6; ++v) red[v * B + threadIdx.x] = t.get(grav || v < 5 ? v : 4) * vol;
  __syncthreads();
  for (int v = wid; v < 6; v += nw) {  // wave-uniform
    double a = 0.0;
    for (int j = l; j < B; j += 64) a += red[v * B + j];
    a = wave_sum(a);
    if (l == 0) out[v] = a;
  }
  __syncthreads();
  t.zero();
}

template <class T>
__device__ __forceinline__ Prim<T> shfl_prim(const Prim<T>& W, int src) {
  Prim<T> r;
  r.r = __shfl(W.r, src);
  r.u = __shfl(W.u, src);
  r.t1 = __shfl(W.t1, src);
  r.t2 = __shfl(W.t2, src);
  r.p = __shfl(W.p, src);
  r.ri = __shfl(W.ri, src);
  return r;
}

template <class T>
__device__ __forceinline__ Cons<T> shfl_cons(const Cons<T>& F, int src) {
  Cons<T> r;
  r.r = __shfl(F.r, src);
  r.mn = __shfl(F.mn, src);
  r.mt1 = __shfl(F.mt1, src);
  r.mt2 = __shfl(F.mt2, src);
  r.e = __shfl(F.e, src);
  return r;
}

// --------------------------------------------------------------------------
// Lane runs along x
// --------------------------------------------------------------------------

// Values a wave hands to its neighbour waves of the same pencil (MULTI
// variant): the edge primitives, the last face state and the first flux.
template <class T>
struct EdgeSlots {
  T wf[6];   // W of the wave's first cell
  T wl[6];   // W of the wave's last active cell
  T wp[6];   // W+ face state of the last active cell
  T f[5];    // flux on the left face of the first cell
};

template <class T>
__device__ __forceinline__ void put_prim(T* s, const Prim<T>& W) {
  s[0] = W.r; s[1] = W.u; s[2] = W.t1; s[3] = W.t2; s[4] = W.p; s[5] = W.ri;
}
template <class T>
__device__ __forceinline__ Prim<T> get_prim(const T* s) {
  Prim<T> W;
  W.r = s[0]; W.u = s[1]; W.t1 = s[2]; W.t2 = s[3]; W.p = s[4]; W.ri = s[5];
  return W;
}

// Lane-run update of a pencil that lies inside one wave.  This lane holds V
// consecutive cells U (rotated frame: mn is the momentum along the sweep
// axis, AXIS); gl is its place in the pencil (0 .. last), srcL and srcR the
// lanes holding the neighbouring runs (a periodic pencil's ends are each
// other's neighbours).  Values cross lanes by shuffles only; the ends of a
// non-periodic pencil build their ghost cells from their own cells.  U is
// replaced by the updated state; lanes with `act` fold their cells into the
// CFL maximum when do_cfl.  Every lane of the wave must call this together.
template <class T, int V, int AXIS>
__device__ __forceinline__ void lanerun_update(Cons<T> (&U)[V], int gl, int last, int srcL,
                                               int srcR, int bc_lo, int bc_hi,
                                               const SweepConst<T>& k, const T id[3], bool act,
                                               bool do_cfl, T& smax, bool& bad) {
  Prim<T> W[V];
#pragma unroll
  for (int c = 0; c < V; ++c) W[c] = to_prim(U[c], k);

  Prim<T> Wl = shfl_prim(W[V - 1], srcL);
  Prim<T> Wr = shfl_prim(W[0], srcR);
  if (gl == 0 && bc_lo != kBcPeriodic) Wl = bc_lo == kBcOutflow ? W[0] : mirror(W[0]);
  if (gl == last && bc_hi != kBcPeriodic) Wr = bc_hi == kBcOutflow ? W[V - 1] : mirror(W[V - 1]);

  Prim<T> Wm[V], Wp[V];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    const Prim<T>& L = c == 0 ? Wl : W[c - 1];
    const Prim<T>& R = c == V - 1 ? Wr : W[c + 1];
    face_states(L, W[c], R, k, k.kick, Wm[c], Wp[c]);
  }

  Prim<T> WpL = shfl_prim(Wp[V - 1], srcL);  // face state W+ of the cell left of the first
  if (gl == 0 && bc_lo != kBcPeriodic) {
    // ghost cell -1 with ghost -2 behind it
    Prim<T> g1, g2, dummy;
    T kick = k.kick;
    if (bc_lo == kBcOutflow) {
      g1 = W[0];
      g2 = W[0];
    } else {
      const Prim<T>& W1 = V >= 2 ? W[V >= 2 ? 1 : 0] : Wr;
      g1 = mirror(W[0]);
      g2 = mirror(W1);
      kick = -k.kick;
    }
    face_states(g2, g1, W[0], k, kick, dummy, WpL);
  }

  Cons<T> F[V];
#pragma unroll
  for (int c = 0; c < V; ++c) F[c] = hllc(c == 0 ? WpL : Wp[c - 1], Wm[c], k);

  Cons<T> FR = shfl_cons(F[0], srcR);  // flux at the right face of the last cell
  if (gl == last && bc_hi != kBcPeriodic) {
    // ghost cell N with ghost N+1 beyond it
    Prim<T> g1, g2, WmR, dummy;
    T kick = k.kick;
    if (bc_hi == kBcOutflow) {
      g1 = W[V - 1];
      g2 = W[V - 1];
    } else {
      const Prim<T>& Wn2 = V >= 2 ? W[V >= 2 ? V - 2 : 0] : Wl;
      g1 = mirror(W[V - 1]);
      g2 = mirror(Wn2);
      kick = -k.kick;
    }
    face_states(W[V - 1], g1, g2, k, kick, WmR, dummy);
    FR = hllc(Wp[V - 1], WmR, k);
  }

#pragma unroll
  for (int c = 0; c < V; ++c) {
    update(U[c], F[c], c == V - 1 ? FR : F[c + 1], k);
    if (act && do_cfl) smax = fmax_(smax, cell_speed<T, AXIS>(U[c], k, id, bad));
  }
}

// One tile of x-pencils.  Lane l of a pencil holds cells [lV, lV+V).  Values
// cross lane boundaries by cross-lane shuffles.
//  * MULTI = false: a pencil has at most 64 lanes (n/V <= 64); floor(64/(n/V))
//    pencils share a wave and a pencil's periodic neighbour is its own far
//    end, also a shuffle.  No LDS, no barrier: every load of a pencil comes
//    before its first shuffle and every store after its last.
//  * MULTI = true: a pencil spans S = ceil((n/V)/64) consecutive waves of the
//    workgroup.  Inside a wave values move by shuffles; across a wave edge
//    the edge lanes pass them through small LDS slots between barriers.  All
//    loads precede the first barrier and all stores follow the last, so the
//    in-place update is race-free.
// Outflow and reflecting ends build their ghost cells from the edge lanes'
// own cells.
template <class T, int V, bool MULTI, bool TOT>
__device__ void xsweep_tile(const SweepArgs<T>& a, const PatchDev& P, int64_t tile,
                            const SweepConst<T>& k, EdgeSlots<T>* slots, T& smax,
                            bool& bad, TotL& tot) {
  const bool store = !(TOT && a.tonly);
  const int N = P.n[0];
  const int LPP = N / V;                 // lanes per pencil
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int l = tid & 63;
  const int nwaves = blockDim.x >> 6;
  int gl, last, pw, seg = 0, S = 1;      // lane in pencil, its last lane, pencil in tile
  bool act;
  int64_t q;
  if (!MULTI) {
    const int gpw = 64 / LPP;            // pencils per wave
    const int grp = l / LPP;
    gl = l - grp * LPP;
    last = LPP - 1;
    pw = wave * gpw + grp;
    q = tile * int64_t(nwaves * gpw) + pw;
    act = grp < gpw;
  } else {
    S = (LPP + 63) >> 6;
    pw = wave / S;
    seg = wave - pw * S;
    gl = seg * 64 + l;
    last = LPP - 1;
    q = tile * int64_t(nwaves / S) + pw;
    act = pw < nwaves / S && gl < LPP;
  }
  const int64_t npen = int64_t(P.n[1]) * P.n[2];
  act = act && q < npen;
  const Planes<T, 0> pl(a.pool, P);
  uint32_t off = 0;  // byte offset of this lane's first cell inside a plane
  unsigned y = 0, z = 0;
  if (act) {
    z = unsigned(q) / unsigned(P.n[1]);
    y = unsigned(q) - z * unsigned(P.n[1]);
    off = uint32_t((int64_t(y) * P.sy + int64_t(z) * P.sz + gl * V) * int64_t(sizeof(T)));
  }

  Cons<T> U[V];
  {
    T r[V], mn[V], mt1[V], mt2[V], e[V];
    if (act) {
      load_run<T, V>(pl.r, off, r);
      load_run<T, V>(pl.n, off, mn);
      load_run<T, V>(pl.t1, off, mt1);
      load_run<T, V>(pl.t2, off, mt2);
      load_run<T, V>(pl.e, off, e);
    } else {
#pragma unroll
      for (int c = 0; c < V; ++c) {  // a benign state for idle lanes
        r[c] = T(1); mn[c] = mt1[c] = mt2[c] = T(0); e[c] = T(1);
      }
    }
#pragma unroll
    for (int c = 0; c < V; ++c) U[c] = Cons<T>{r[c], mn[c], mt1[c], mt2[c], e[c]};
  }

  if constexpr (!MULTI) {
    const int srcL = gl > 0 ? l - 1 : l + last;
    const int srcR = gl < last ? l + 1 : l - last;
    T id[3];
    inv_widths<T>(P, id);
    lanerun_update<T, V, 0>(U, gl, last, srcL, srcR, a.bc_lo, a.bc_hi, k, id, act,
                            a.do_cfl != 0, smax, bad);
    if (TOT && act) {
#pragma unroll
      for (int c = 0; c < V; ++c) tot_add<T, 0>(tot, U[c], P, a.gvec, gl * V + c, y, z);
    }
    if (act && store) {
      T r[V], mn[V], mt1[V], mt2[V], e[V];
#pragma unroll
      for (int c = 0; c < V; ++c) {
        r[c] = U[c].r; mn[c] = U[c].mn; mt1[c] = U[c].mt1; mt2[c] = U[c].mt2; e[c] = U[c].e;
      }
      store_run<T, V>(pl.r, off, r);
      store_run<T, V>(pl.n, off, mn);
      store_run<T, V>(pl.t1, off, mt1);
      store_run<T, V>(pl.t2, off, mt2);
      store_run<T, V>(pl.e, off, e);
    }
    return;
  }

  Prim<T> W[V];
#pragma unroll
  for (int c = 0; c < V; ++c) W[c] = to_prim(U[c], k);

  // lane-level neighbours inside a wave (a wave-edge lane takes the value it
  // gets here only when the neighbour lives in the same wave)
  const int srcL = MULTI ? ((l + 63) & 63) : (gl > 0 ? l - 1 : l + last);
  const int srcR = MULTI ? ((l + 1) & 63) : (gl < last ? l + 1 : l - last);
  const bool firstw = MULTI && l == 0;                               // left neighbour in LDS
  const bool lastw = MULTI && (l == 63 || gl == last) && gl <= last;  // right neighbour in LDS
  const int wfirst = wave - seg;          // first wave of this pencil (MULTI)
  const int wlast = wfirst + S - 1;

  Prim<T> Wl = shfl_prim(W[V - 1], srcL);
  Prim<T> Wr = shfl_prim(W[0], srcR);
  if (MULTI) {
    if (act && firstw) put_prim(slots[wave].wf, W[0]);
    if (act && lastw) put_prim(slots[wave].wl, W[V - 1]);
    __syncthreads();
    if (act && firstw) {
      if (gl > 0) Wl = get_prim(slots[wave - 1].wl);
      else if (a.bc_lo == kBcPeriodic) Wl = get_prim(slots[wlast].wl);
    }
    if (act && lastw) {
      if (gl < last) Wr = get_prim(slots[wave + 1].wf);
      else if (a.bc_hi == kBcPeriodic) Wr = get_prim(slots[wfirst].wf);
    }
  }
  if (gl == 0 && a.bc_lo != kBcPeriodic) Wl = a.bc_lo == kBcOutflow ? W[0] : mirror(W[0]);
  if (gl == last && a.bc_hi != kBcPeriodic)
    Wr = a.bc_hi == kBcOutflow ? W[V - 1] : mirror(W[V - 1]);

  Prim<T> Wm[V], Wp[V];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    const Prim<T>& L = c == 0 ? Wl : W[c - 1];
    const Prim<T>& R = c == V - 1 ? Wr : W[c + 1];
    face_states(L, W[c], R, k, k.kick, Wm[c], Wp[c]);
  }

  Prim<T> WpL = shfl_prim(Wp[V - 1], srcL);  // face state W+ of the cell left of the first
  if (MULTI) {
    if (act && lastw) put_prim(slots[wave].wp, Wp[V - 1]);
    __syncthreads();
    if (act && firstw) {
      if (gl > 0) WpL = get_prim(slots[wave - 1].wp);
      else if (a.bc_lo == kBcPeriodic) WpL = get_prim(slots[wlast].wp);
    }
  }
  if (gl == 0 && a.bc_lo != kBcPeriodic) {
    // ghost cell -1 with ghost -2 behind it
    Prim<T> g1, g2, dummy;
    T kick = k.kick;
    if (a.bc_lo == kBcOutflow) {
      g1 = W[0];
      g2 = W[0];
    } else {
      const Prim<T>& W1 = V >= 2 ? W[V >= 2 ? 1 : 0] : Wr;
      g1 = mirror(W[0]);
      g2 = mirror(W1);
      kick = -k.kick;
    }
    face_states(g2, g1, W[0], k, kick, dummy, WpL);
  }

  Cons<T> F[V];
#pragma unroll
  for (int c = 0; c < V; ++c) F[c] = hllc(c == 0 ? WpL : Wp[c - 1], Wm[c], k);

  Cons<T> FR = shfl_cons(F[0], srcR);  // flux at the right face of the last cell
  if (MULTI) {
    if (act && firstw) {
      T* s = slots[wave].f;
      s[0] = F[0].r; s[1] = F[0].mn; s[2] = F[0].mt1; s[3] = F[0].mt2; s[4] = F[0].e;
    }
    __syncthreads();
    if (act && lastw) {
      const T* s = nullptr;
      if (gl < last) s = slots[wave + 1].f;
      else if (a.bc_hi == kBcPeriodic) s = slots[wfirst].f;
      if (s) FR = Cons<T>{s[0], s[1], s[2], s[3], s[4]};
    }
  }
  if (gl == last && a.bc_hi != kBcPeriodic) {
    // ghost cell N with ghost N+1 beyond it
    Prim<T> g1, g2, WmR, dummy;
    T kick = k.kick;
    if (a.bc_hi == kBcOutflow) {
      g1 = W[V - 1];
      g2 = W[V - 1];
    } else {
      const Prim<T>& Wn2 = V >= 2 ? W[V >= 2 ? V - 2 : 0] : Wl;
      g1 = mirror(W[V - 1]);
      g2 = mirror(Wn2);
      kick = -k.kick;
    }
    face_states(W[V - 1], g1, g2, k, kick, WmR, dummy);
    FR = hllc(Wp[V - 1], WmR, k);
  }

  if (act) {
    T id[3];
    inv_widths<T>(P, id);
    T r[V], mn[V], mt1[V], mt2[V], e[V];
#pragma unroll
    for (int c = 0; c < V; ++c) {
      update(U[c], F[c], c == V - 1 ? FR : F[c + 1], k);
      r[c] = U[c].r; mn[c] = U[c].mn; mt1[c] = U[c].mt1; mt2[c] = U[c].mt2; e[c] = U[c].e;
      if (a.do_cfl) smax = fmax_(smax, cell_speed<T, 0>(U[c], k, id, bad));
      if (TOT) tot_add<T, 0>(tot, U[c], P, a.gvec, gl * V + c, y, z);
    }
    if (store) {
      store_run<T, V>(pl.r, off, r);
      store_run<T, V>(pl.n, off, mn);
      store_run<T, V>(pl.t1, off, mt1);
      store_run<T, V>(pl.t2, off, mt2);
      store_run<T, V>(pl.e, off, e);
    }
  }
}

// Work item of a persistent launch, made wave-uniform so that the item,
// the patch record and the plane pointers live in scalar registers.
__device__ __forceinline__ int next_item(unsigned int* ticket, int* slot) {
  if (threadIdx.x == 0) *slot = int(atomicAdd(ticket, 1u));
  __syncthreads();
  const int it = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();
  return it;
}

// The i-th work item of this workgroup: pulled from the ticket (dynamic
// scheduling), or item blockIdx.x + i gridDim.x (static round robin over the
// largest-first list: no atomic and no barrier per item).
template <class T>
__device__ __forceinline__ int item_at(const SweepArgs<T>& a, int i, unsigned int* ticket,
                                       int* slot) {
  if (a.dyn) return next_item(ticket, slot);
  return int(blockIdx.x) + i * int(gridDim.x);
}

// Direct FP32 totals instantiation with whole pencils per wave: four waves per
// SIMD (128 registers), which it would otherwise miss by two registers.
template <class T, int V, bool MULTI, bool PERSIST, bool TOT>
__global__ void __launch_bounds__(512, sizeof(T) == 4 && TOT && !MULTI && !PERSIST ? 4 : 1)
    sweep_x_kernel(SweepArgs<T> a) {
  __shared__ EdgeSlots<T> slots[MULTI ? 8 : 1];
  __shared__ int item_s;
  __shared__ T red[8];
  __shared__ double tred[TOT ? 48 : 1];
  extern __shared__ __align__(16) unsigned char dyn_lds[];  // TOT: per-thread totals (TotL)
  const double dt = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool grav = has_grav(a.gvec);
  T smax = T(0);
  bool bad = false;
  TotL tot{reinterpret_cast<double*>(dyn_lds)};
  if (TOT) tot.zero();
  if (!PERSIST) {
    SweepConst<T> k = make_const<T>(dt, a.single.dx[0], a.gamma, a.grav);
    if (!TOT) {
      xsweep_tile<T, V, MULTI, TOT>(a, a.single, blockIdx.x, k, slots, smax, bad, tot);
    } else {
      // a capped grid strides over the a.nitems tiles: the totals partial
      // of a workgroup covers many pencils
      for (int64_t tile = blockIdx.x; tile < a.nitems; tile += gridDim.x) {
        xsweep_tile<T, V, MULTI, TOT>(a, a.single, tile, k, slots, smax, bad, tot);
        if (MULTI) __syncthreads();
      }
      tot_block(tot, cell_volume(a.single), a.tpart + 6 * int64_t(blockIdx.x), tred, grav);
    }
  } else {
    for (int i = 0;; ++i) {
      const int it = item_at(a, i, &a.scal->tickets[0], &item_s);
      if (it >= a.nitems) break;
      const WorkItem w = a.items[it];
      const PatchDev P = a.patches[w.patch];
      SweepConst<T> k = make_const<T>(item_dt(a, w.patch, dt), P.dx[0], a.gamma, a.grav);
      xsweep_tile<T, V, MULTI, TOT>(a, P, w.tile, k, slots, smax, bad, tot);
      if (TOT) tot_block(tot, cell_volume(P), a.tpart + 6 * int64_t(it), tred, grav);
      if (MULTI) __syncthreads();
      item_cfl(a, w.patch, smax, red);
    }
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0 && !a.pdt, red);
}

// --------------------------------------------------------------------------
// Chunked x march: one pencil per wave
// --------------------------------------------------------------------------

// Value of lane `lane` (wave-uniform) of x, as a wave-uniform value.
__device__ __forceinline__ float lane_val(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double lane_val(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), lane));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class T>
__device__ __forceinline__ Prim<T> lane_prim(const Prim<T>& W, int lane) {
  Prim<T> r;
  r.r = lane_val(W.r, lane); r.u = lane_val(W.u, lane); r.t1 = lane_val(W.t1, lane);
  r.t2 = lane_val(W.t2, lane); r.p = lane_val(W.p, lane); r.ri = lane_val(W.ri, lane);
  return r;
}
template <class T>
__device__ __forceinline__ Cons<T> lane_cons(const Cons<T>& U, int lane) {
  return Cons<T>{lane_val(U.r, lane), lane_val(U.mn, lane), lane_val(U.mt1, lane),
                 lane_val(U.mt2, lane), lane_val(U.e, lane)};
}

// The five planes of one lane run.
template <class T, int V>
struct Run {
  T r[V], n[V], t1[V], t2[V], e[V];
};

template <class T, int V>
__device__ __forceinline__ void load_runs(const Planes<T, 0>& pl, uint32_t off, bool act,
                                          Run<T, V>& R) {
  if (act) {
    load_run<T, V>(pl.r, off, R.r);
    load_run<T, V>(pl.n, off, R.n);
    load_run<T, V>(pl.t1, off, R.t1);
    load_run<T, V>(pl.t2, off, R.t2);
    load_run<T, V>(pl.e, off, R.e);
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) {  // a benign state for idle lanes
      R.r[c] = T(1); R.n[c] = R.t1[c] = R.t2[c] = T(0); R.e[c] = T(1);
    }
  }
}

// The last 128-byte line of a chunk's runs is written to memory by the next
// chunk, in one piece, rather than in two pieces at different times (the
// line holds the run whose last cell waits for the next chunk).  Until then
// it waits in a per-wave LDS buffer of kLineBytes per plane: slot i, plane v
// at elements [v kLineBytes/sizeof(T) + i V, + V).
constexpr int kLineBytes = 128;

// Orders this wave's LDS accesses across lanes: the hardware runs a wave's
// LDS instructions in order, and the fences keep the compiler from moving
// them across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T, int V>
__device__ __forceinline__ void put_run(T* line, int slot, const Run<T, V>& R) {
  constexpr int PL = kLineBytes / int(sizeof(T));
  T* b = line + slot * V;
#pragma unroll
  for (int c = 0; c < V; ++c) {
    b[c] = R.r[c]; b[PL + c] = R.n[c]; b[2 * PL + c] = R.t1[c]; b[3 * PL + c] = R.t2[c];
    b[4 * PL + c] = R.e[c];
  }
}

template <class T, int V>
__device__ __forceinline__ void get_run(const T* line, int slot, Run<T, V>& R) {
  constexpr int PL = kLineBytes / int(sizeof(T));
  const T* b = line + slot * V;
#pragma unroll
  for (int c = 0; c < V; ++c) {
    R.r[c] = b[c]; R.n[c] = b[PL + c]; R.t1[c] = b[2 * PL + c]; R.t2[c] = b[3 * PL + c];
    R.e[c] = b[4 * PL + c];
  }
}

// x-pencils q0, q0 + qs, ... (below qend) marched one after another by one
// wave, each in chunks of 64 lane runs (64 V cells); lane l of chunk j holds
// cells [(64 j + l) V, (64 j + l + 1) V).  Inside a chunk values cross lanes
// by shuffles.  Across a chunk edge:
//  * the next chunk is loaded (prefetched) before the current one is
//    stored, so its first cell is still the original state; lane 63 takes
//    that cell's primitives as its right neighbour;
//  * the flux through the chunk edge needs the next chunk's face states, so
//    the update of the chunk's last cell waits one chunk: lane 63 keeps its
//    run, and lane 0 of the next chunk finishes the held cell from the
//    carried (original) state, its left flux and the edge flux (which that
//    lane computes anyway as its own left-face flux), then stores the whole
//    run, so that no run is ever written in pieces;
//  * the carried values (primitives and W+ face state of the held cell, its
//    state and left flux, the updated head of the run) are wave-uniform.
// The last chunk of a pencil prefetches the first chunk of the next one.
// A periodic pencil reads its last two cells before anything is stored (for
// the wrap face at the low end) and keeps the first cell's primitives and
// the wrap flux of the first chunk for its high end.  Every value of a
// pencil is loaded before the wave stores over it, and no other wave touches
// the pencil, so the update is in place without barriers.
template <class T, int V, bool TOT>
__device__ void xmarch_pencils(const SweepArgs<T>& a, const PatchDev& P, int q0, int qs,
                               int qend, const SweepConst<T>& k, const T id[3], T* line,
                               T& smax, bool& bad, TotL& tot) {
  if (q0 >= qend) return;
  const bool store = !(TOT && a.tonly);
  const int N = P.n[0];
  const int LPP = N / V;
  const int C = (LPP + 63) >> 6;
  const int l = threadIdx.x & 63;
  const Planes<T, 0> pl(a.pool, P);
  const uint32_t runb = uint32_t(V * sizeof(T));
  constexpr int LPL = int(kLineBytes / (V * sizeof(T)));  // lane runs per 128-byte line
  const bool per = a.bc_lo == kBcPeriodic;  // periodic is set on both ends or neither
  const unsigned ny = unsigned(P.n[1]);
  auto row_of = [&](int q) {
    const unsigned z = unsigned(q) / ny, y = unsigned(q) - z * ny;
    return uint32_t((int64_t(y) * P.sy + int64_t(z) * P.sz) * int64_t(sizeof(T)));
  };

  Run<T, V> nxt;
  load_runs<T, V>(pl, row_of(q0) + uint32_t(l) * runb, l < LPP, nxt);
  for (int q = q0; q < qend; q += qs) {
    const uint32_t row = row_of(q);
    const int qz = int(unsigned(q) / ny), qy = q - qz * int(ny);  // the pencil's (y, z)
    const int qn = q + qs;  // next pencil of this wave
    Prim<T> Wt1, Wt2;  // original cells N-1 and N-2 (periodic low end)
    if (per) {
      Wt1 = to_prim(pl.load(row + uint32_t((N - 1) * sizeof(T))), k);
      Wt2 = to_prim(pl.load(row + uint32_t((N - 2) * sizeof(T))), k);
    }

    Prim<T> W0, Wprev, WpPrev;  // carried, wave-uniform
    Cons<T> Fwrap, Uheld, Fheld;
    for (int j = 0; j < C; ++j) {
      const int gl = j * 64 + l;
      const bool act = gl < LPP;
      const bool lastc = j == C - 1;
      const int hi = lastc ? LPP - 1 - j * 64 : 63;  // last active lane of the chunk
      const uint32_t off = row + uint32_t(gl) * runb;
      Cons<T> U[V];
      Prim<T> W[V];
#pragma unroll
      for (int c = 0; c < V; ++c) {
        U[c] = Cons<T>{nxt.r[c], nxt.n[c], nxt.t1[c], nxt.t2[c], nxt.e[c]};
        W[c] = to_prim(U[c], k);
      }
      if (!lastc) load_runs<T, V>(pl, off + 64 * runb, gl + 64 < LPP, nxt);
      else if (qn < qend) load_runs<T, V>(pl, row_of(qn) + uint32_t(l) * runb, l < LPP, nxt);
      if (j == 0 && per) W0 = lane_prim(W[0], 0);

      const int srcL = (l + 63) & 63, srcR = (l + 1) & 63;
      Prim<T> Wl = shfl_prim(W[V - 1], srcL);
      Prim<T> Wr = shfl_prim(W[0], srcR);
      if (l == 0) {
        if (j > 0) Wl = Wprev;
        else if (per) Wl = Wt1;
        else Wl = a.bc_lo == kBcOutflow ? W[0] : mirror(W[0]);
      }
      if (!lastc) {
        const Cons<T> un{lane_val(nxt.r[0], 0), lane_val(nxt.n[0], 0), lane_val(nxt.t1[0], 0),
                         lane_val(nxt.t2[0], 0), lane_val(nxt.e[0], 0)};
        const Prim<T> Wn = to_prim(un, k);
        if (l == 63) Wr = Wn;
      } else if (l == hi) {
        if (per) Wr = W0;
        else Wr = a.bc_hi == kBcOutflow ? W[V - 1] : mirror(W[V - 1]);
      }

      Prim<T> Wm[V], Wp[V];
#pragma unroll
      for (int c = 0; c < V; ++c) {
        const Prim<T>& L = c == 0 ? Wl : W[c - 1];
        const Prim<T>& R = c == V - 1 ? Wr : W[c + 1];
        face_states(L, W[c], R, k, k.kick, Wm[c], Wp[c]);
      }

      Prim<T> WpL = shfl_prim(Wp[V - 1], srcL);
      if (l == 0) {
        if (j > 0) {
          WpL = WpPrev;
        } else if (per) {
          Prim<T> dummy;
          face_states(Wt2, Wt1, W[0], k, k.kick, dummy, WpL);
        } else {
          // ghost cell -1 with ghost -2 behind it
          Prim<T> g1, g2, dummy;
          T kick = k.kick;
          if (a.bc_lo == kBcOutflow) {
            g1 = W[0];
            g2 = W[0];
          } else {
            const Prim<T>& W1 = V >= 2 ? W[V >= 2 ? 1 : 0] : Wr;
            g1 = mirror(W[0]);
            g2 = mirror(W1);
            kick = -k.kick;
          }
          face_states(g2, g1, W[0], k, kick, dummy, WpL);
        }
      }

      Cons<T> F[V];
#pragma unroll
      for (int c = 0; c < V; ++c) F[c] = hllc(c == 0 ? WpL : Wp[c - 1], Wm[c], k);
      if (j == 0 && per) Fwrap = lane_cons(F[0], 0);

      Cons<T> FR = shfl_cons(F[0], srcR);  // flux at the right face of the lane's last cell
      if (lastc && l == hi) {
        if (per) {
          FR = Fwrap;
        } else {
          // ghost cell N with ghost N+1 beyond it
          Prim<T> g1, g2, WmR, dummy;
          T kick = k.kick;
          if (a.bc_hi == kBcOutflow) {
            g1 = W[V - 1];
            g2 = W[V - 1];
          } else {
            const Prim<T>& Wn2 = V >= 2 ? W[V >= 2 ? V - 2 : 0] : Wl;
            g1 = mirror(W[V - 1]);
            g2 = mirror(Wn2);
            kick = -k.kick;
          }
          face_states(W[V - 1], g1, g2, k, kick, WmR, dummy);
          FR = hllc(Wp[V - 1], WmR, k);
        }
      }

      // the last line of the previous chunk: its held cell takes lane 0's
      // left-face flux as its right-face flux; lanes 0..LPL-1 store the
      // line's runs, kept in LDS since that chunk, as whole vectors
      wave_sync();  // the line written by other lanes of this wave
      if (j > 0) {
        Cons<T> Ud = Uheld;
        update(Ud, Fheld, lane_cons(F[0], 0), k);
        if (a.do_cfl && l == 0) smax = fmax_(smax, cell_speed<T, 0>(Ud, k, id, bad));
        if (TOT && l == 0) tot_add<T, 0>(tot, Ud, P, a.gvec, j * 64 * V - 1, qy, qz);
        if (l < LPL && store) {
          Run<T, V> o;
          get_run<T, V>(line, l, o);
          if (l == LPL - 1) {
            o.r[V - 1] = Ud.r; o.n[V - 1] = Ud.mn; o.t1[V - 1] = Ud.mt1;
            o.t2[V - 1] = Ud.mt2; o.e[V - 1] = Ud.e;
          }
          const uint32_t ho = off - uint32_t(LPL) * runb;
          store_run<T, V>(pl.r, ho, o.r);
          store_run<T, V>(pl.n, ho, o.n);
          store_run<T, V>(pl.t1, ho, o.t1);
          store_run<T, V>(pl.t2, ho, o.t2);
          store_run<T, V>(pl.e, ho, o.e);
        }
      }
      wave_sync();  // every lane has read the line before it is refilled
      const bool hold = !lastc && l == 63;  // its last cell waits for the next chunk
      if (!lastc) {
        Wprev = lane_prim(W[V - 1], 63);
        WpPrev = lane_prim(Wp[V - 1], 63);
        Uheld = lane_cons(U[V - 1], 63);
        Fheld = lane_cons(F[V - 1], 63);
      }

      if (act) {
#pragma unroll
        for (int c = 0; c < V; ++c) {
          update(U[c], F[c], c == V - 1 ? FR : F[c + 1], k);
          if (a.do_cfl && !(hold && c == V - 1))
            smax = fmax_(smax, cell_speed<T, 0>(U[c], k, id, bad));
          if (TOT && !(hold && c == V - 1))
            tot_add<T, 0>(tot, U[c], P, a.gvec, gl * V + c, qy, qz);
        }
        Run<T, V> o;
#pragma unroll
        for (int c = 0; c < V; ++c) {
          o.r[c] = U[c].r; o.n[c] = U[c].mn; o.t1[c] = U[c].mt1; o.t2[c] = U[c].mt2;
          o.e[c] = U[c].e;
        }
        if (!store) {
          // totals of the current state: nothing is written
        } else if (lastc || l < 64 - LPL) {
          store_run<T, V>(pl.r, off, o.r);
          store_run<T, V>(pl.n, off, o.n);
          store_run<T, V>(pl.t1, off, o.t1);
          store_run<T, V>(pl.t2, off, o.t2);
          store_run<T, V>(pl.e, off, o.e);
        } else {
          put_run<T, V>(line, l - (64 - LPL), o);  // the next chunk stores it
        }
      }
    }
  }
}

// Direct FP32 launches: at least three waves per SIMD (168 registers),
// which the totals instantiation would otherwise miss by one register.
template <class T, int V, bool PERSIST, bool TOT>
__global__ void __launch_bounds__(512, sizeof(T) == 4 && !PERSIST ? 3 : 1)
    sweep_xm_kernel(SweepArgs<T> a) {
  __shared__ int item_s;
  __shared__ T red[8];
  __shared__ T lines[8][5 * kLineBytes / sizeof(T)];  // per wave
  __shared__ double tred[TOT ? 48 : 1];
  extern __shared__ __align__(16) unsigned char dyn_lds[];  // TOT: per-thread totals (TotL)
  const double dt = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool grav = has_grav(a.gvec);
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T smax = T(0);
  bool bad = false;
  TotL tot{reinterpret_cast<double*>(dyn_lds)};
  if (TOT) tot.zero();
  if (!PERSIST) {
    const PatchDev& P = a.single;
    SweepConst<T> k = make_const<T>(dt, P.dx[0], a.gamma, a.grav);
    T id[3];
    inv_widths<T>(P, id);
    // grid-stride over pencils: wave w of workgroup b takes pencils
    // b nw + w, (b + G) nw + w, ... for a grid of G workgroups
    xmarch_pencils<T, V, TOT>(a, P, int(blockIdx.x) * nw + wave, int(gridDim.x) * nw,
                              P.n[1] * P.n[2], k, id, lines[wave], smax, bad, tot);
    if (TOT)
      tot_block(tot, cell_volume(a.single), a.tpart + 6 * int64_t(blockIdx.x), tred, grav);
  } else {
    for (int i = 0;; ++i) {
      const int it = item_at(a, i, &a.scal->tickets[0], &item_s);
      if (it >= a.nitems) break;
      const WorkItem w = a.items[it];
      const PatchDev P = a.patches[w.patch];
      SweepConst<T> k = make_const<T>(item_dt(a, w.patch, dt), P.dx[0], a.gamma, a.grav);
      T id[3];
      inv_widths<T>(P, id);
      const int npen = P.n[1] * P.n[2];
      xmarch_pencils<T, V, TOT>(a, P, w.tile * nw + wave, npen, npen, k, id, lines[wave], smax,
                                bad, tot);
      if (TOT) tot_block(tot, cell_volume(P), a.tpart + 6 * int64_t(it), tred, grav);
      item_cfl(a, w.patch, smax, red);
    }
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0 && !a.pdt, red);
}

// --------------------------------------------------------------------------
// Fused x and y sweeps of one z-plane of a patch, held in LDS (batches)
// --------------------------------------------------------------------------
//
// A work item is one z-plane of one patch.  The workgroup copies the plane
// (5 variables) into LDS, runs the first sweep, then the second, on the
// plane in LDS, and copies it back: one pass over HBM for two sweeps.  The x
// and y sweeps of a plane touch no other plane, so planes are independent
// and the update is in place.  Both sweeps are lane runs (lanerun_update):
// along x a lane holds V consecutive cells of a row, along y V consecutive
// cells of a column, and a pencil's lanes trade values by shuffles.
//
// LDS layout: rows of a fixed pitch of kPlanePitch elements, the five
// variables of one y interleaved row by row.  Variable v (physical order) of
// cell (x, y) sits at
//   (5 y + v) kPlanePitch + ((x + s(y)) mod kPlanePitch),  s(y) = V floor(y / V).
// With the pitch a compile-time power of two, every access of a run (V cells
// of the five variables) is one base address plus immediate offsets, and
// the rotation is a mask.  The rotation keeps every aligned run of V cells
// of a row contiguous and aligned, and spreads the V-cell column runs that
// the lanes of one y access read over different LDS banks.

// Row pitch (elements) of a plane in LDS, and the largest plane a
// workgroup holds: two such workgroups fit in the 160 KiB LDS of a CU.
constexpr int kPlanePitch = 64;
constexpr int kPlaneLdsBytes = 81920;

// Element offset of run start x (a multiple of V) in LDS row y.
template <int V>
__device__ __forceinline__ int plane_col(int x, int y) {
  return (x + (y & ~(V - 1))) & (kPlanePitch - 1);
}

// V consecutive elements between memory and LDS (both aligned to the run).
template <class T, int V>
__device__ __forceinline__ void copy_run(T* dst, const T* src) {
  constexpr int H = (sizeof(T) * V <= 16) ? V : int(16 / sizeof(T));
  typedef T vec __attribute__((ext_vector_type(H)));
#pragma unroll
  for (int h = 0; h < V / H; ++h)
    *reinterpret_cast<vec*>(dst + h * H) = *reinterpret_cast<const vec*>(src + h * H);
}

// The five plane bases of a grid or patch (wave-uniform) for row runs
// addressed by one 32-bit byte offset (planes stay below 4 GiB).
template <class T>
struct RowBases {
  char* p[5];
};

template <class T>
__device__ __forceinline__ RowBases<T> row_bases(T* buf, int64_t base0, int64_t plane) {
  RowBases<T> b;
  char* p0 = reinterpret_cast<char*>(buf + base0);
#pragma unroll
  for (int v = 0; v < 5; ++v) b.p[v] = p0 + v * plane * int64_t(sizeof(T));
  return b;
}

// A row run: V consecutive elements of each of the five variables at
// B.p[v] + off, rotated into the x frame, between registers and memory: a
// wave-uniform base and one offset register per run, no 64-bit address
// arithmetic per run.
template <class T, int V, bool WRITE>
__device__ __forceinline__ void row_run_off(const RowBases<T>& B, uint32_t off,
                                            Cons<T> (&U)[V]) {
  T r[V], mn[V], mt1[V], mt2[V], e[V];
  auto at = [&](int v) { return reinterpret_cast<T*>(B.p[v] + off); };
  if (WRITE) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      r[c] = U[c].r; mn[c] = U[c].mn; mt1[c] = U[c].mt1; mt2[c] = U[c].mt2; e[c] = U[c].e;
    }
    copy_run<T, V>(at(0), r); copy_run<T, V>(at(1), mn); copy_run<T, V>(at(2), mt1);
    copy_run<T, V>(at(3), mt2); copy_run<T, V>(at(4), e);
  } else {
    copy_run<T, V>(r, at(0)); copy_run<T, V>(mn, at(1)); copy_run<T, V>(mt1, at(2));
    copy_run<T, V>(mt2, at(3)); copy_run<T, V>(e, at(4));
#pragma unroll
    for (int c = 0; c < V; ++c) U[c] = Cons<T>{r[c], mn[c], mt1[c], mt2[c], e[c]};
  }
}

// Where the pencils of a plane sweep live in memory, as the plane functions
// below see them: a rectangle of n(0) x n(1) cells of one plane whose part
// [lo(0), hi(0)) x [lo(1), hi(1)) is written.  at(base, x, y) is cell (x, y)
// of variable 0 in a buffer laid out like the state; cell(x, y) gives its
// grid coordinates (totals).
//  * PatchPlane: the whole z-plane of a batch patch, read and written in
//    place, with the launch's boundary conditions at the pencil ends.
//  * PatchZPlane: an x-z plane of a batch patch (below).
//  * WindowPlane: a window of a single grid's z-plane (WinDev), read from
//    the pool and written to a.dst, wrapped around periodic axes.
template <class T>
struct PatchPlane {
  const SweepArgs<T>& a;
  const PatchDev& P;
  int z;
  __device__ int n(int axis) const { return P.n[axis]; }
  __device__ int bc_lo(int axis) const { return axis == 0 ? a.bc_lo : a.bc_lo_y; }
  __device__ int bc_hi(int axis) const { return axis == 0 ? a.bc_hi : a.bc_hi_y; }
  __device__ int lo(int) const { return 0; }
  __device__ int hi(int axis) const { return P.n[axis]; }
  __device__ int3 cell(int x, int y) const { return make_int3(x, y, z); }
  __device__ T* src() const { return a.pool; }
  __device__ T* dst() const { return a.pool; }
  __device__ int64_t plane() const { return P.plane; }
  __device__ T* at(T* base, int x, int y) const {
    return base + P.base0 + int64_t(z) * P.sz + int64_t(y) * P.sy + x;
  }
  __device__ RowBases<T> bases(T* buf) const { return row_bases(buf, P.base0, P.plane); }
  __device__ uint32_t off(int x, int y) const {
    return uint32_t(z * P.sz + y * P.sy + x) * uint32_t(sizeof(T));
  }
};

// The x-z plane y = yr of a batch patch: the plane's second axis is z (the
// z march of a batch as lane runs in LDS), with the launch's z boundary
// conditions in bc_lo_y / bc_hi_y.
template <class T>
struct PatchZPlane {
  const SweepArgs<T>& a;
  const PatchDev& P;
  int yr;
  __device__ int n(int axis) const { return P.n[axis == 0 ? 0 : 2]; }
  __device__ int bc_lo(int axis) const { return axis == 0 ? a.bc_lo : a.bc_lo_y; }
  __device__ int bc_hi(int axis) const { return axis == 0 ? a.bc_hi : a.bc_hi_y; }
  __device__ int lo(int) const { return 0; }
  __device__ int hi(int axis) const { return n(axis); }
  __device__ int3 cell(int x, int y) const { return make_int3(x, yr, y); }
  __device__ T* src() const { return a.pool; }
  __device__ T* dst() const { return a.pool; }
  __device__ int64_t plane() const { return P.plane; }
  __device__ T* at(T* base, int x, int y) const {
    return base + P.base0 + int64_t(y) * P.sz + int64_t(yr) * P.sy + x;
  }
  __device__ RowBases<T> bases(T* buf) const { return row_bases(buf, P.base0, P.plane); }
  __device__ uint32_t off(int x, int y) const {
    return uint32_t(y * P.sz + yr * P.sy + x) * uint32_t(sizeof(T));
  }
};

template <class T>
struct WindowPlane {
  const SweepArgs<T>& a;
  const PatchDev& G;
  const WinDev& w;
  int z;
  __device__ static int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
  __device__ int n(int axis) const { return axis == 0 ? kWinEdge : win_rows(sizeof(T) == 8); }
  __device__ int bc_lo(int axis) const { return axis == 0 ? w.bx_lo : w.by_lo; }
  __device__ int bc_hi(int axis) const { return axis == 0 ? w.bx_hi : w.by_hi; }
  __device__ int lo(int axis) const { return axis == 0 ? w.ox0 : w.oy0; }
  __device__ int hi(int axis) const { return axis == 0 ? w.ox1 : w.oy1; }
  __device__ int gx(int x) const { return wrap(w.x0 + x, G.n[0]); }
  __device__ int gy(int y) const { return wrap(w.y0 + y, G.n[1]); }
  __device__ int3 cell(int x, int y) const { return make_int3(gx(x), gy(y), z); }
  __device__ T* src() const { return a.pool; }
  __device__ T* dst() const { return a.dst; }
  __device__ int64_t plane() const { return G.plane; }
  __device__ T* at(T* base, int x, int y) const {
    return base + G.base0 + int64_t(z) * G.sz + int64_t(gy(y)) * G.sy + gx(x);
  }
  __device__ RowBases<T> bases(T* buf) const { return row_bases(buf, G.base0, G.plane); }
  __device__ uint32_t off(int x, int y) const {
    return uint32_t(z * G.sz + gy(y) * G.sy + gx(x)) * uint32_t(sizeof(T));
  }
};

// The plane between memory and LDS (LOAD: every cell from m.src(), else the
// written part to m.dst()).  LDS row r holds variable r mod 5 of y = r / 5.
template <class T, int V, bool LOAD, class M>
__device__ void plane_copy(const M& m, T* lds) {
  const int nx = m.n(0), ny = m.n(1);
  const int nq = nx / V;    // runs per row (<= 64)
  const int rpw = 64 / nq;  // rows per wave
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = l / nq, q = l - r * nq;
  if (r >= rpw) return;
  const int64_t pl = m.plane();
  const int step = nw * rpw;
  auto laddr = [&](int row) { return lds + row * kPlanePitch + plane_col<V>(q * V, row / 5); };
  if (LOAD) {
    T* base = m.src();
    const int rows = 5 * ny;
    // B runs in flight per lane before the first LDS write
    constexpr int B = int(128 / (V * sizeof(T))) < 8 ? int(128 / (V * sizeof(T))) : 8;
    for (int row0 = wave * rpw + r; row0 < rows; row0 += B * step) {
      T buf[B][V];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int row = row0 + b * step, y = row / 5;
        if (row < rows) copy_run<T, V>(buf[b], m.at(base, q * V, y) + int64_t(row - 5 * y) * pl);
      }
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (row0 + b * step < rows) copy_run<T, V>(laddr(row0 + b * step), buf[b]);
    }
  } else {
    T* base = m.dst();
    if (q * V < m.lo(0) || q * V >= m.hi(0)) return;
    for (int row = 5 * m.lo(1) + wave * rpw + r; row < 5 * m.hi(1); row += step) {
      const int y = row / 5;
      copy_run<T, V>(m.at(base, q * V, y) + int64_t(row - 5 * y) * pl, laddr(row));
    }
  }
}

// Reads (write = false) or writes the V cells of a run in LDS: the cells at
// (x0 + c dx, y0 + c dy), c < V, of the five variables, rotated into the
// frame of the sweep axis AXIS (0: x, along the plane's first axis; 1 or 2:
// y or z, along its second axis).
template <class T, int V, int AXIS, bool WRITE>
__device__ __forceinline__ void plane_run(T* lds, int x0, int y0, Cons<T> (&U)[V]) {
  constexpr int vn = Rot<AXIS>::n, vt1 = Rot<AXIS>::t1, vt2 = Rot<AXIS>::t2;
  constexpr int P = kPlanePitch;
  // x0 and y0 are multiples of V, so the whole run shares one rotation and
  // a run of a row stays contiguous
  T* base = lds + 5 * y0 * P + plane_col<V>(x0, y0);
#pragma unroll
  for (int c = 0; c < V; ++c) {
    T* p = AXIS == 0 ? base + c : base + 5 * c * P;
    if (WRITE) {
      p[0] = U[c].r; p[vn * P] = U[c].mn; p[vt1 * P] = U[c].mt1; p[vt2 * P] = U[c].mt2;
      p[4 * P] = U[c].e;
    } else {
      U[c] = Cons<T>{p[0], p[vn * P], p[vt1 * P], p[vt2 * P], p[4 * P]};
    }
  }
}

// One sweep along AXIS (0: x, 1: y, 2: z) of the pencils [p0, p1) of the
// plane (rows for AXIS 0, columns of the plane's second axis for AXIS 1 or
// 2; the launch puts that axis's gravity in grav_y).  Pencils of n cells
// take n/V lanes; a wave holds 64/(n/V) pencils, laid out so that the lanes
// of equal place in their pencils sit together (along the second axis they
// then read consecutive x).  The input comes from LDS, or for the x sweep of an x-first step
// straight from memory (GSRC); the result goes to LDS, or for the x sweep of
// a y-first step straight to memory (GDST, the written part only): a row
// run is a coalesced vector access, so those two sweeps skip a copy through
// LDS.  Only runs in the written part fold the CFL maximum and the totals.
template <class T, int V, int AXIS, bool GSRC, bool GDST, bool TOT = false, class M>
__device__ void plane_sweep(const SweepArgs<T>& a, const M& m, const PatchDev& P, int p0, int p1,
                            T* lds, bool do_cfl, double dt, T& smax, bool& bad,
                            TotR* tot = nullptr) {
  constexpr int LA = AXIS == 0 ? 0 : 1;   // the plane axis the pencils run along
  const int n = m.n(LA);                  // pencil length
  const int LPP = n / V, ppw = 64 / LPP;  // lanes per pencil, pencils per wave
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int gl = l / ppw, col = l - gl * ppw, last = LPP - 1;
  const int srcL = gl > 0 ? l - ppw : l + last * ppw;
  const int srcR = gl < last ? l + ppw : l - last * ppw;
  const SweepConst<T> k = make_const<T>(dt, P.dx[AXIS], a.gamma, AXIS == 0 ? a.grav : a.grav_y);
  T id[3];
  inv_widths<T>(P, id);
  const int blo = m.bc_lo(LA), bhi = m.bc_hi(LA);
  const int mstep = nw * ppw;
  // the written part: runs along the pencil, and pencils
  const int rlo = m.lo(LA), rhi = m.hi(LA), plo = m.lo(1 - LA), phi = m.hi(1 - LA);
  // rows in memory: wave-uniform plane bases and one byte offset per run
  const RowBases<T> sb = m.bases(m.src());
  Cons<T> Un[V];  // GSRC: the next pass's runs, loaded one pass ahead
#pragma unroll
  for (int c = 0; c < V; ++c) Un[c] = Cons<T>{T(1), T(0), T(0), T(0), T(1)};
  // lanes past the pencils (pen >= p1, or gl >= LPP when n/V does not divide
  // 64) work on a valid clamped run: their results are neither stored nor
  // folded, and shuffles never cross from them into an active pencil
  const int glr = gl < LPP ? gl : LPP - 1;
  if (GSRC && gl < LPP && p0 + wave * ppw + col < p1)
    row_run_off<T, V, false>(sb, m.off(gl * V, p0 + wave * ppw + col), Un);
  for (int m0 = p0 + wave * ppw; m0 < p1; m0 += mstep) {  // wave-uniform
    const int pen = m0 + col;
    const bool act = gl < LPP && pen < p1;
    const bool wr = act && gl * V >= rlo && gl * V < rhi && pen >= plo && pen < phi;
    Cons<T> U[V];
    if (GSRC) {
#pragma unroll
      for (int c = 0; c < V; ++c) U[c] = Un[c];
    } else {
      const int penr = pen < p1 ? pen : p1 - 1;
      plane_run<T, V, AXIS, false>(lds, AXIS == 0 ? glr * V : penr, AXIS == 0 ? penr : glr * V, U);
    }
    if (GSRC && gl < LPP && pen + mstep < p1)
      row_run_off<T, V, false>(sb, m.off(gl * V, pen + mstep), Un);
    lanerun_update<T, V, AXIS>(U, act ? gl : 0, last, srcL, srcR, blo, bhi, k, id, wr, do_cfl,
                               smax, bad);
    if (TOT && wr) {
#pragma unroll
      for (int c = 0; c < V; ++c) {
        const int3 q = m.cell(LA == 0 ? gl * V + c : pen, LA == 0 ? pen : gl * V + c);
        tot_add<T, AXIS>(*tot, U[c], P, a.gvec, q.x, q.y, q.z);
      }
    }
    if (GDST) {
      if (wr && !(TOT && a.tonly)) row_run_off<T, V, true>(m.bases(m.dst()), m.off(gl * V, pen), U);
    } else if (act) {
      plane_run<T, V, AXIS, true>(lds, AXIS == 0 ? gl * V : pen, AXIS == 0 ? pen : gl * V, U);
    }
  }
}

// The FP64 totals of the written part of the plane, held in LDS after its
// last sweep: thread t takes the cells t, t + blockDim.x, ... (x fastest).
template <class T, int V, class M>
__device__ void plane_totals(const SweepArgs<T>& a, const M& m, const PatchDev& P, const T* lds,
                             TotR& tot) {
  constexpr int PP = kPlanePitch;
  const int x0 = m.lo(0), y0 = m.lo(1), wx = m.hi(0) - x0;
  const int cells = wx * (m.hi(1) - y0);
  for (int c = threadIdx.x; c < cells; c += blockDim.x) {
    const int yy = c / wx, x = x0 + c - yy * wx, y = y0 + yy;
    const T* p = lds + 5 * y * PP + plane_col<V>(x, y);
    const Cons<T> U{p[0], p[PP], p[2 * PP], p[3 * PP], p[4 * PP]};  // x frame: lab order
    const int3 q = m.cell(x, y);
    tot_add<T, 0>(tot, U, P, a.gvec, q.x, q.y, q.z);
  }
}

// One plane of a fused step: XFIRST, x then y (even steps); else y then x
// (odd steps).  The second sweep runs only on the pencils of the written
// part; the first on all of them (the second needs its halo).  TOT (the
// last launch of a step): y then x adds each written cell to the totals as
// it stores it; x then y adds the written part in LDS with plane_totals
// before copying it out.  `P` gives the cell widths and gravity frame.
template <class T, int V, bool XFIRST, bool TOT, class M>
__device__ __forceinline__ void plane_item(const SweepArgs<T>& a, const M& m, const PatchDev& P,
                                           T* lds, double dt, T& smax, bool& bad, TotR& tot) {
  const bool store = !(TOT && a.tonly);
  if (XFIRST) {
    // x: memory -> registers -> LDS; y: LDS -> LDS; then LDS -> memory
    plane_sweep<T, V, 0, true, false>(a, m, P, 0, m.n(1), lds, false, dt, smax, bad);
    __syncthreads();
    plane_sweep<T, V, 1, false, false>(a, m, P, m.lo(0), m.hi(0), lds, a.do_cfl != 0, dt, smax,
                                       bad);
    __syncthreads();
    if (TOT) plane_totals<T, V>(a, m, P, lds, tot);
    if (store) plane_copy<T, V, false>(m, lds);
  } else {
    // memory -> LDS; y: LDS -> LDS; x: LDS -> registers -> memory
    plane_copy<T, V, true>(m, lds);
    __syncthreads();
    plane_sweep<T, V, 1, false, false>(a, m, P, 0, m.n(0), lds, false, dt, smax, bad);
    __syncthreads();
    // (with TOT adding each written cell to the totals)
    plane_sweep<T, V, 0, false, true, TOT>(a, m, P, m.lo(1), m.hi(1), lds, a.do_cfl != 0, dt,
                                           smax, bad, &tot);
  }
  __syncthreads();  // the LDS is free again
}

// The fused x and y sweeps of batch patch z-planes (persistent; XFIRST as
// in plane_item).  The plane takes up to half the LDS of a CU, so two
// workgroups share one: no static LDS beside it (the totals reduction and
// the next ticket use the plane's LDS once the plane has been copied out).
template <class T, int V, bool XFIRST, bool TOT>
__global__ void __launch_bounds__(512) sweep_plane_kernel(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* lds = reinterpret_cast<T*>(dyn_lds);
  int* slot = reinterpret_cast<int*>(dyn_lds);  // free between items
  const double dt0 = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool grav = has_grav(a.gvec);
  T smax = T(0);
  bool bad = false;
  TotR tot;
  tot.zero();
  for (int i = 0;; ++i) {
    const int it = item_at(a, i, &a.scal->tickets[3], slot);
    if (it >= a.nitems) break;
    const WorkItem w = a.items[it];
    const PatchDev P = a.patches[w.patch];
    const PatchPlane<T> m{a, P, w.tile};
    plane_item<T, V, XFIRST, TOT>(a, m, P, lds, item_dt(a, w.patch, dt0), smax, bad, tot);
    if (TOT)
      tot_block_wide(tot, cell_volume(P), a.tpart + 6 * int64_t(it),
                     reinterpret_cast<double*>(dyn_lds), grav);
    item_cfl(a, w.patch, smax, lds);
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0 && !a.pdt, lds);
}

// Item i of n, remapped so that neighbouring items run on one XCD: the
// dispatcher places workgroup b on XCD b mod 8, and round robin over a grid
// of a multiple of 8 workgroups hands item i to XCD i mod 8, so XCD x gets
// the contiguous items x q + min(x, r) .. (n = 8 q + r).  Neighbouring
// windows share the cache lines of their overlap.
__device__ __forceinline__ int xcd_item(int i, int n) {
  const int q = n >> 3, r = n & 7, x = i & 7, k = i >> 3;
  return x * q + (x < r ? x : r) + k;
}

// The z sweep of a batch as lane runs in LDS: a work item is one x-z plane
// (y = tile) of one patch (nx <= 64; <= 80 KiB), loaded whole (rows of x,
// coalesced), swept along z (the column pencils of the plane), and stored
// back.  Unlike the column march it recomputes nothing at segment edges
// (patches are 16-64 cells along z).  Persistent like the plane kernel; TOT
// adds the plane in LDS before copying it out.
template <class T, int V, bool TOT>
__global__ void __launch_bounds__(512) sweep_zplane_kernel(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* lds = reinterpret_cast<T*>(dyn_lds);
  int* slot = reinterpret_cast<int*>(dyn_lds);  // free between items
  const double dt0 = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool store = !(TOT && a.tonly);
  const bool grav = has_grav(a.gvec);
  T smax = T(0);
  bool bad = false;
  TotR tot;
  tot.zero();
  for (int i = 0;; ++i) {
    const int it = item_at(a, i, &a.scal->tickets[2], slot);
    if (it >= a.nitems) break;
    const WorkItem w = a.items[it];
    const PatchDev P = a.patches[w.patch];
    const PatchZPlane<T> m{a, P, w.tile};
    plane_copy<T, V, true>(m, lds);
    __syncthreads();
    plane_sweep<T, V, 2, false, false>(a, m, P, 0, m.n(0), lds, a.do_cfl != 0,
                                       item_dt(a, w.patch, dt0), smax, bad);
    __syncthreads();
    if (TOT) plane_totals<T, V>(a, m, P, lds, tot);
    if (store) plane_copy<T, V, false>(m, lds);
    __syncthreads();  // the LDS is free again
    if (TOT)
      tot_block_wide(tot, cell_volume(P), a.tpart + 6 * int64_t(it),
                     reinterpret_cast<double*>(dyn_lds), grav);
    item_cfl(a, w.patch, smax, lds);
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0 && !a.pdt, lds);
}

// The fused x and y sweeps of a single grid, window by window (WinDev):
// work item it is window it mod nwin of z-plane it / nwin, taken round
// robin (xcd_item order) by a grid of resident workgroups (every item
// costs the same); with TOT each workgroup sums its items in registers and
// writes one partial.  The
// windows overlap (each reads two cells past its written part), so the
// result goes to a.dst, a buffer laid out like the state.  Four waves per
// SIMD (at most 128 registers): the LDS holds two workgroups of eight waves
// per CU.
template <class T, int V, bool XFIRST, bool TOT>
__global__ void __launch_bounds__(512, sizeof(T) == 4 ? 4 : 2) sweep_window_kernel(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* lds = reinterpret_cast<T*>(dyn_lds);
  const double dt = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool grav = has_grav(a.gvec);
  T smax = T(0);
  bool bad = false;
  TotR tot;
  tot.zero();
  for (int i = blockIdx.x; i < a.nitems; i += gridDim.x) {
    const int it = xcd_item(i, a.nitems);
    const int z = it / a.nwin;
    const WinDev w = a.wins[it - z * a.nwin];
    const WindowPlane<T> m{a, a.single, w, z};
    plane_item<T, V, XFIRST, TOT>(a, m, a.single, lds, dt, smax, bad, tot);
  }
  // the items of a workgroup are fixed by the grid size (round robin), so
  // one partial per workgroup has a fixed summation order
  if (TOT)
    tot_block_wide(tot, cell_volume(a.single), a.tpart + 6 * int64_t(blockIdx.x),
                   reinterpret_cast<double*>(dyn_lds), grav);
  finish_block(a.scal, smax, bad, a.do_cfl != 0, lds);
}

// --------------------------------------------------------------------------
// Column marches along y (AXIS 1) or z (AXIS 2)
// --------------------------------------------------------------------------

// Column march prefetch depth (cells in flight ahead of the update).
#ifndef HYDRO_MARCH_AHEAD
#define HYDRO_MARCH_AHEAD 3
#endif
constexpr int kMarchAhead = HYDRO_MARCH_AHEAD;

// Cell c of a column, as (a) the owning segment's index s' = c / L and
// (b) that segment's edge slot: its first two cells are slots 0, 1 and its
// last two slots 2, 3 (a segment shorter than four cells repeats cells).
// Only cells within two of a segment edge are ever looked up.
__device__ __forceinline__ int edge_slot(int c, int L, int N, int* seg) {
  const int s = c / L;
  const int ja = s * L, jb = min(N, ja + L);
  *seg = s;
  return c - ja < 2 ? c - ja : 2 + (c - (jb - 2));
}

// One tile of a column march: Q consecutive columns, each cut into S
// segments of L cells owned by S threads.
//  * LDSH = true (halos through LDS): every thread loads its segment's
//    first two and last two cells once, writes their primitives to an LDS
//    table (tab: [segment][slot][component][Q]) and keeps the last two
//    states in registers for the end of its march; after the barrier each
//    thread reads its four halo cells from the table.  Every cell is then
//    read from memory once.
//  * LDSH = false: each thread loads its halo cells from memory before the
//    barrier (the owner loads them again when it marches there).
template <class T, int AXIS, bool LDSH, bool TOT>
__device__ void colsweep_tile(const SweepArgs<T>& a, const PatchDev& P, int64_t tile,
                              const SweepConst<T>& k, T* tab, T& smax, bool& bad, TotL& tot) {
  const bool store = !(TOT && a.tonly);
  constexpr int TA = AXIS == 1 ? 2 : 1;   // the other transverse axis
  const int N = P.n[AXIS];
  const int nx = P.n[0];
  const int ncol = nx * P.n[TA];
  const uint32_t sd = uint32_t((AXIS == 1 ? P.sy : P.sz) * int64_t(sizeof(T)));  // bytes
  const int64_t st = AXIS == 1 ? P.sz : P.sy;
  const int Q = a.q, S = a.s;
  const int l = threadIdx.x % Q;
  const int seg = threadIdx.x / Q;
  const int col = int(tile) * Q + l;
  const int L = (N + S - 1) / S;
  const int ja = seg * L;
  const int jb = min(N, ja + L);
  const bool act = (seg < S) && (col < ncol) && (ja < jb);
  const Planes<T, AXIS> pl(a.pool, P);
  const Planes<T, AXIS> pd(a.dst ? a.dst : a.pool, P);  // the result (out of place: a.dst)
  uint32_t cb = 0;  // byte offset of the column's cell 0 inside a plane
  int cx = 0, ct = 0;  // the column's x and its index along the other transverse axis
  if (act) {
    const unsigned t = unsigned(col) / unsigned(nx), x = unsigned(col) - t * unsigned(nx);
    cb = uint32_t((int64_t(x) + int64_t(t) * st) * int64_t(sizeof(T)));
    cx = int(x);
    ct = int(t);
  }
  // the updated cell c of the column into the totals
  auto total = [&](const Cons<T>& U, int c) {
    if (AXIS == 1) tot_add<T, 1>(tot, U, P, a.gvec, cx, c, ct);
    else tot_add<T, 2>(tot, U, P, a.gvec, cx, ct, c);
  };

  // halo cell h (ja-2, ja-1, jb, jb+1) after the boundary conditions: the
  // interior cell it copies, and whether it is mirrored
  auto halo_cell = [&](int h, bool& mir) {
    int j = h < 2 ? ja - 2 + h : jb + h - 2;
    mir = false;
    if (j < 0) {
      if (a.bc_lo == kBcPeriodic) j += N;
      else if (a.bc_lo == kBcOutflow) j = 0;
      else { j = -j - 1; mir = true; }
    } else if (j >= N) {
      if (a.bc_hi == kBcPeriodic) j -= N;
      else if (a.bc_hi == kBcOutflow) j = N - 1;
      else { j = 2 * N - 1 - j; mir = true; }
    }
    return j;
  };

  // halo h from the LDSH table (primitives of segment edge cells)
  auto table_halo = [&](int h) {
    bool mir;
    int os;
    const int e = edge_slot(halo_cell(h, mir), L, N, &os);
    const T* t = tab + ((os * 4 + e) * 5) * Q + l;
    Prim<T> W;
    W.r = t[0]; W.u = t[Q]; W.t1 = t[2 * Q]; W.t2 = t[3 * Q]; W.p = t[4 * Q];
    W.ri = rcp(W.r);  // as to_prim computes it
    return mir ? mirror(W) : W;
  };

  Prim<T> H[4];
  Cons<T> E[4];  // LDSH: own cells ja, ja+1, jb-2, jb-1 (clamped into the segment)
  if (LDSH) {
    if (act) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = e < 2 ? min(ja + e, jb - 1) : max(jb - 4 + e, ja);
        E[e] = pl.load(cb + uint32_t(c) * sd);
        const Prim<T> W = to_prim(E[e], k);
        T* t = tab + ((seg * 4 + e) * 5) * Q + l;
        t[0] = W.r; t[Q] = W.u; t[2 * Q] = W.t1; t[3 * Q] = W.t2; t[4 * Q] = W.p;
      }
    }
    __syncthreads();  // the table is full, and no cell has been written
    if (!act) return;
    // the halos before the segment now; those after it are read from the
    // table again at the end of the march (the table stays intact until the
    // tile ends), so they hold no registers during the march
    H[0] = table_halo(0);
    H[1] = table_halo(1);
  } else {
    if (act) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        bool mir;
        const int j = halo_cell(h, mir);
        Prim<T> W = to_prim(pl.load(cb + uint32_t(j) * sd), k);
        H[h] = mir ? mirror(W) : W;
      }
    }
    __syncthreads();  // every halo copy is taken before any cell is written
    if (!act) return;
  }

  T id[3];
  inv_widths<T>(P, id);
  const T kick_lo = (ja == 0 && a.bc_lo == kBcReflect) ? -k.kick : k.kick;
  const T kick_hi = (jb == N && a.bc_hi == kBcReflect) ? -k.kick : k.kick;

  // March: cell j is updated from the flux on its left face (carried) and
  // the flux on its right face, which needs the face states of cell j+1,
  // hence the primitives of j, j+1, j+2.  The body of the main loop has no
  // branch on the position: cells are prefetched three iterations ahead,
  // clamped to the last cell read from memory (an own cell ahead of the
  // march, not yet written); with LDSH the last two cells come from
  // registers; the last two updates, whose j+2 neighbour is a halo copy,
  // run in the tail loop.
  uint32_t b = cb + uint32_t(ja) * sd;    // byte offset of cell j
  Cons<T> U0 = LDSH ? E[0] : pl.load(b);
  Prim<T> W0 = to_prim(U0, k);
  Cons<T> U1;
  Prim<T> W1;
  if (ja + 1 < jb) {
    U1 = LDSH ? E[1] : pl.load(b + sd);
    W1 = to_prim(U1, k);
  } else {
    W1 = LDSH ? table_halo(2) : H[2];
  }
  Prim<T> WpPrev, WmC, WpC, dummy;
  face_states(H[0], H[1], W0, k, kick_lo, dummy, WpPrev);   // cell ja-1
  face_states(H[1], W0, W1, k, k.kick, WmC, WpC);           // cell ja
  Cons<T> Fl = hllc(WpPrev, WmC, k);
  WpPrev = WpC;

  // one step of the march with cell j+2 in U2 (cell j updated)
  auto advance = [&](const Cons<T>& U2, int j) {
    const Prim<T> W2 = to_prim(U2, k);
    Prim<T> Wm1, Wp1;
    face_states(W0, W1, W2, k, k.kick, Wm1, Wp1);  // cell j+1
    const Cons<T> Fr = hllc(WpPrev, Wm1, k);
    update(U0, Fl, Fr, k);
    if (store) pd.store(b, U0);
    if (a.do_cfl) smax = fmax_(smax, cell_speed<T, AXIS>(U0, k, id, bad));
    if (TOT) total(U0, j);
    b += sd;
    U0 = U1;
    U1 = U2;
    W0 = W1;
    W1 = W2;
    WpPrev = Wp1;
    Fl = Fr;
  };

  int j = ja;
  const int jm = LDSH ? jb - 4 : jb - 2;  // main loop: cell j+2 read from memory
  if (jm > ja) {
    // cells j+3 .. j+2+D are in flight while cell j is updated (clamped to
    // the last cell read from memory)
    // The offset of the newest prefetched cell runs in 32 bits, clamped to
    // bmax, so every access is a scalar base plus one 32-bit offset (the
    // host keeps every offset up to one layer past a plane's last cell
    // below 4 GiB, so oa + sd cannot wrap).
    constexpr int D = kMarchAhead;
    const uint32_t bmax = cb + uint32_t(jm + 1) * sd;
    uint32_t oa = b + 2 * sd;  // cell ja+2 <= jm+1
    Cons<T> Pq[D];
    Pq[0] = pl.load(oa);
#pragma unroll
    for (int d = 1; d < D; ++d) {
      oa = min(oa + sd, bmax);
      Pq[d] = pl.load(oa);
    }
    // unrolled 6 times: the carried cells rotate with period 3, the carried
    // face state and flux with period 2 and the prefetch queue with period
    // D (a divisor of 6), so the copies vanish
#pragma unroll 6
    for (; j < jm; ++j) {
      const Cons<T> U2 = Pq[0];
#pragma unroll
      for (int d = 0; d + 1 < D; ++d) Pq[d] = Pq[d + 1];
      oa = min(oa + sd, bmax);  // cell j+2+D, clamped
      Pq[D - 1] = pl.load(oa);
      advance(U2, j);
    }
  }
  if (LDSH) {
    for (; j < jb - 2; ++j) advance(j + 2 == jb - 2 ? E[2] : E[3], j);
    H[2] = table_halo(2);
    H[3] = table_halo(3);
  }
  for (; j < jb; ++j) {
    const Prim<T> W2 = (j + 2 == jb) ? H[2] : H[3];
    Prim<T> Wm1, Wp1;
    face_states(W0, W1, W2, k, (j + 1 == jb) ? kick_hi : k.kick, Wm1, Wp1);  // cell j+1
    const Cons<T> Fr = hllc(WpPrev, Wm1, k);
    update(U0, Fl, Fr, k);
    if (store) pd.store(b, U0);
    if (a.do_cfl) smax = fmax_(smax, cell_speed<T, AXIS>(U0, k, id, bad));
    if (TOT) total(U0, j);
    b += sd;
    U0 = U1;
    W0 = W1;
    W1 = W2;
    WpPrev = Wp1;
    Fl = Fr;
  }
}

// FP32: at least kColWaves waves per SIMD, the occupancy the march needs to
// cover memory latency.
#ifndef HYDRO_COL_WAVES
#define HYDRO_COL_WAVES 4
#endif
constexpr int kColWaves = HYDRO_COL_WAVES;
// Dynamic LDS: with TOT the per-thread totals (kTotStride doubles a
// thread) first, then with LDSH the halo table.
// FP32: kColWaves waves per SIMD; the persistent totals instantiation (the
// batch's last z sweep) takes three, whose registers hold it without spills.
template <class T, int AXIS, bool PERSIST, bool LDSH, bool TOT>
__global__ void __launch_bounds__(512, sizeof(T) == 4 ? (PERSIST && TOT ? 3 : kColWaves) : 1)
    sweep_col_kernel(SweepArgs<T> a) {
  __shared__ int item_s;
  __shared__ T red[8];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ double tred[TOT ? 48 : 1];
  TotL tot{reinterpret_cast<double*>(dyn_lds)};
  T* tab = reinterpret_cast<T*>(dyn_lds + (TOT ? 8 * kTotStride * blockDim.x : 0));
  const double dt = (TOT && a.tonly) ? 0.0 : a.scal->dt;
  const bool grav = has_grav(a.gvec);
  T smax = T(0);
  bool bad = false;
  if (TOT) tot.zero();
  if (!PERSIST) {
    SweepConst<T> k = make_const<T>(dt, a.single.dx[AXIS], a.gamma, a.grav);
    colsweep_tile<T, AXIS, LDSH, TOT>(a, a.single, blockIdx.x, k, tab, smax, bad, tot);
    if (TOT)
      tot_block(tot, cell_volume(a.single), a.tpart + 6 * int64_t(blockIdx.x), tred, grav);
  } else {
    for (int i = 0;; ++i) {
      const int it = item_at(a, i, &a.scal->tickets[AXIS], &item_s);
      if (it >= a.nitems) break;
      const WorkItem w = a.items[it];
      const PatchDev P = a.patches[w.patch];
      SweepConst<T> k = make_const<T>(item_dt(a, w.patch, dt), P.dx[AXIS], a.gamma, a.grav);
      colsweep_tile<T, AXIS, LDSH, TOT>(a, P, w.tile, k, tab, smax, bad, tot);
      __syncthreads();
      if (TOT) tot_block(tot, cell_volume(P), a.tpart + 6 * int64_t(it), tred, grav);
      item_cfl(a, w.patch, smax, red);
    }
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0 && !a.pdt, red);
}

// --------------------------------------------------------------------------
// Standalone CFL reduction and FP64 totals (grid: x = chunks, y = patch)
// --------------------------------------------------------------------------

template <class T>
struct ReduceArgs {
  const T* pool;
  const PatchDev* patches;  // null: single grid
  PatchDev single;
  double gamma;
  double grav[3];
  DevScalars* scal;
  double* partials;         // totals: [patch][chunk][6]
  unsigned long long* psmax;  // CFL maximum per patch (null: scal->smax_bits)
};

template <class T>
__global__ void __launch_bounds__(256) cfl_kernel(ReduceArgs<T> a) {
  __shared__ T red[16];
  const PatchDev P = a.patches ? a.patches[blockIdx.y] : a.single;
  const int64_t cells = int64_t(P.n[0]) * P.n[1] * P.n[2];
  SweepConst<T> k = make_const<T>(0.0, 1.0, a.gamma, 0.0);
  T id[3];
  inv_widths<T>(P, id);
  const Planes<T, 0> pl(const_cast<T*>(a.pool), P);
  T smax = T(0);
  bool bad = false;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cells;
       c += int64_t(gridDim.x) * blockDim.x) {
    int x = int(c % P.n[0]);
    int64_t r = c / P.n[0];
    int y = int(r % P.n[1]);
    int z = int(r / P.n[1]);
    uint32_t off = uint32_t((x + int64_t(y) * P.sy + int64_t(z) * P.sz) * int64_t(sizeof(T)));
    Cons<T> U = pl.load(off);
    smax = fmax_(smax, cell_speed<T, 0>(U, k, id, bad));
  }
  finish_block(a.scal, smax, bad, true, red, a.psmax ? &a.psmax[blockIdx.y] : nullptr);
}

// Partial sums of rho, mx, my, mz, E and E + rho*phi (phi = -g.x at cell
// centres, origin at the low corner of the patch), times the cell volume,
// accumulated in FP64 in a fixed order: per thread in a fixed stride, then
// a fixed wave and workgroup tree.  One partial per (patch, chunk).
template <class T>
__global__ void __launch_bounds__(256) totals_kernel(ReduceArgs<T> a) {
  __shared__ double red[4][6];
  const PatchDev P = a.patches ? a.patches[blockIdx.y] : a.single;
  const int64_t cells = int64_t(P.n[0]) * P.n[1] * P.n[2];
  const double vol = P.dx[0] * P.dx[1] * P.dx[2];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cells;
       c += int64_t(gridDim.x) * blockDim.x) {
    int x = int(c % P.n[0]);
    int64_t r = c / P.n[0];
    int y = int(r % P.n[1]);
    int z = int(r / P.n[1]);
    const T* p = a.pool + P.base0 + x + int64_t(y) * P.sy + int64_t(z) * P.sz;
    double rho = double(p[0]);
    double e = double(p[4 * P.plane]);
    acc[0] += rho * vol;
    acc[1] += double(p[P.plane]) * vol;
    acc[2] += double(p[2 * P.plane]) * vol;
    acc[3] += double(p[3 * P.plane]) * vol;
    acc[4] += e * vol;
    double phi = -(a.grav[0] * ((x + 0.5) * P.dx[0]) + a.grav[1] * ((y + 0.5) * P.dx[1]) +
                   a.grav[2] * ((z + 0.5) * P.dx[2]));
    acc[5] += (e + rho * phi) * vol;
  }
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    double s = wave_sum(acc[v]);
    if ((threadIdx.x & 63) == 0) red[wid][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
    a.partials[(int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = s;
  }
}

// Sum of n partials (each 6 doubles) in a fixed order into scal->totals.
__global__ void __launch_bounds__(256) totals_final_kernel(const double* partials, int64_t n,
                                                           DevScalars* scal) {
  __shared__ double red[4][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
    for (int v = 0; v < 6; ++v) acc[v] += partials[i * 6 + v];
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    double s = wave_sum(acc[v]);
    if ((threadIdx.x & 63) == 0) red[wid][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
    scal->totals[threadIdx.x] = s;
  }
}

// --------------------------------------------------------------------------
// Step bookkeeping (one thread)
// --------------------------------------------------------------------------

__device__ void next_dt(DevScalars* s) {
  double smax = __longlong_as_double((long long)s->smax_bits);
  double dt = s->cfl / smax;
  if (!(smax > 0.0) || !(smax < __builtin_huge_val())) {
    s->error |= kErrSpeed;
    dt = 0.0;
  }
  if (s->t_end > 0.0) dt = fmin(dt, fmax(0.0, s->t_end - s->t));
  s->dt = dt;
  s->smax_bits = 0ull;
}

// after a step: t += dt, then dt of the next step from the folded maximum
__global__ void finish_step_kernel(DevScalars* s) {
  s->t += s->dt;
  next_dt(s);
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
}

// The FP64 totals from n per-workgroup partials, in a fixed order: workgroup
// b of R sums the partials [b n / R, (b + 1) n / R) (thread-strided, then a
// fixed wave and workgroup tree) into slice b; the last workgroup to finish
// (counted in s->tdone) sums the R slices in order into s->totals.  With
// `finish` it then ends the step: t += dt and the next dt from the folded
// CFL maximum.  The tickets are reset either way.
__global__ void __launch_bounds__(256) totals_finish_kernel(const double* part, int64_t n,
                                                            double* slice, DevScalars* s,
                                                            int finish) {
  __shared__ double red[4 * 6];
  __shared__ int last;
  const int R = int(gridDim.x), b = int(blockIdx.x);
  const int64_t lo = n * b / R, hi = n * (b + 1) / R;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
#pragma unroll
    for (int v = 0; v < 6; ++v) acc[v] += part[i * 6 + v];
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const double w = wave_sum(acc[v]);
    if ((threadIdx.x & 63) == 0) red[wid * 6 + v] = w;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double a = red[threadIdx.x];
    for (int w = 1; w < int(blockDim.x >> 6); ++w) a += red[w * 6 + threadIdx.x];
    slice[b * 6 + threadIdx.x] = a;
  }
  __threadfence();  // the slice is visible device-wide before the count
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&s->tdone, 1u) == unsigned(R - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();  // every other slice is visible to this workgroup
  if (threadIdx.x < 6) {
    double a = slice[threadIdx.x];
    for (int r = 1; r < R; ++r) a += slice[r * 6 + threadIdx.x];
    s->totals[threadIdx.x] = a;
  }
  if (threadIdx.x == 0) {
    s->tdone = 0u;
    if (finish) {
      s->t += s->dt;
      next_dt(s);
    }
    s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
  }
}

// after a standalone CFL reduction: dt from the current state
__global__ void finish_cfl_kernel(DevScalars* s) {
  next_dt(s);
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
}

__global__ void init_scalars_kernel(DevScalars* s, double cfl, double t, double t_end) {
  s->dt = 0.0;
  s->t = t;
  s->t_end = t_end;
  s->cfl = cfl;
  s->smax_bits = 0ull;
  s->error = 0u;
  s->tdone = 0u;
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
  s->saved[0] = s->saved[1] = 0.0;
  for (int v = 0; v < 6; ++v) s->totals[v] = 0.0;
}

__global__ void set_dt_kernel(DevScalars* s, double dt) { s->dt = dt; }

// after a step that started at t = 0: the dt it took (its t), the next CFL
// dt, the six totals and the sticky error bits into out[0..8]
__global__ void step_results_kernel(const DevScalars* s, double* out) {
  out[0] = s->t;
  out[1] = s->dt;
  for (int v = 0; v < 6; ++v) out[2 + v] = s->totals[v];
  out[8] = double(s->error);
}
__global__ void set_time_kernel(DevScalars* s, double t, double t_end) {
  s->t = t;
  s->t_end = t_end;
}
__global__ void clear_error_kernel(DevScalars* s) { s->error = 0u; }

// save dt and t, set dt = 0 (timing runs leave the state bit for bit)
__global__ void timing_begin_kernel(DevScalars* s) {
  s->saved[0] = s->dt;
  s->saved[1] = s->t;
  s->dt = 0.0;
}
__global__ void timing_end_kernel(DevScalars* s) {
  s->dt = s->saved[0];
  s->t = s->saved[1];
  s->smax_bits = 0ull;
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
}
__global__ void reset_tickets_kernel(DevScalars* s) {
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
}

// --------------------------------------------------------------------------
// Host-side launchers
// --------------------------------------------------------------------------


template <class T>
static SweepArgs<T> to_args(const LaunchSweep& L) {
  SweepArgs<T> a;
  a.pool = static_cast<T*>(L.pool);
  a.patches = L.patches;
  a.single = L.single;
  a.items = L.items;
  a.nitems = L.nitems;
  a.bc_lo = L.bc_lo;
  a.bc_hi = L.bc_hi;
  a.do_cfl = L.do_cfl;
  a.q = L.cfg.q;
  a.s = L.cfg.s;
  a.dyn = L.dyn;
  a.bc_lo_y = L.bc_lo_y;
  a.bc_hi_y = L.bc_hi_y;
  a.grav = L.grav;
  a.grav_y = L.grav_y;
  a.gamma = L.gamma;
  a.scal = L.scal;
  a.tpart = L.tpart;
  for (int i = 0; i < 3; ++i) a.gvec[i] = L.gvec[i];
  a.tonly = L.totals_only;
  a.pdt = L.pdt;
  a.psmax = L.psmax;
  a.dst = static_cast<T*>(L.dst);
  a.wins = L.wins;
  a.nwin = L.nwin;
  return a;
}

// pencils of a patch processed by one workgroup of the x sweep
int64_t x_pencils_per_tile(const PatchDev& P, const SweepCfg& c) {
  const int lpp = P.n[0] / c.v;
  const int nw = c.block / 64;
  if (c.kind == kXMarchKind) return nw;  // one pencil per wave
  if (lpp <= 64) return int64_t(nw) * (64 / lpp);
  const int s = (lpp + 63) / 64;
  return nw / s;
}

int64_t x_tiles(const PatchDev& P, const SweepCfg& c) {
  const int64_t ppw = x_pencils_per_tile(P, c);
  const int64_t npen = int64_t(P.n[1]) * P.n[2];
  return (npen + ppw - 1) / ppw;
}

// workgroups of a direct x launch: one per tile, or for the march at most
// c.q (its grid-stride cap; 0 = no cap)
int64_t x_grid(const PatchDev& P, const SweepCfg& c) {
  const int64_t t = x_tiles(P, c);
  return c.kind == kXMarchKind && c.q > 0 ? std::min<int64_t>(t, c.q) : t;
}

int64_t col_tiles(const PatchDev& P, int axis, const SweepCfg& c) {
  int64_t ncol = int64_t(P.n[0]) * P.n[axis == 1 ? 2 : 1];
  return (ncol + c.q - 1) / c.q;
}

template <class T, int V, bool MULTI, bool PERSIST, bool TOT>
static hipError_t launch_x_vw(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  const size_t tl = TOT ? size_t(L.cfg.block) * kTotStride * sizeof(double) : 0;
  hipLaunchKernelGGL((sweep_x_kernel<T, V, MULTI, PERSIST, TOT>), grid, dim3(L.cfg.block), tl,
                     st, to_args<T>(L));
  return hipGetLastError();
}

template <class T, int V, bool PERSIST, bool TOT>
static hipError_t launch_x_v(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  if (L.xmode == kXMarch) {
    if constexpr (sizeof(T) == 8 && V == 4) {
      return hipErrorInvalidValue;  // not built: the FP64 V=4 march spills registers
    } else {
      const size_t tl = TOT ? size_t(L.cfg.block) * kTotStride * sizeof(double) : 0;
      hipLaunchKernelGGL((sweep_xm_kernel<T, V, PERSIST, TOT>), grid, dim3(L.cfg.block), tl, st,
                         to_args<T>(L));
      return hipGetLastError();
    }
  }
  return L.xmode == kXPacked ? launch_x_vw<T, V, false, PERSIST, TOT>(L, st, grid)
                             : launch_x_vw<T, V, true, PERSIST, TOT>(L, st, grid);
}

template <class T, bool PERSIST, bool TOT>
static hipError_t launch_x(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  switch (L.cfg.v) {
    case 1: return launch_x_v<T, 1, PERSIST, TOT>(L, st, grid);
    case 2: return launch_x_v<T, 2, PERSIST, TOT>(L, st, grid);
    case 4: return launch_x_v<T, 4, PERSIST, TOT>(L, st, grid);
    default: return hipErrorInvalidValue;
  }
}

template <class T, bool PERSIST, bool TOT>
static hipError_t launch_col(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  int s = L.cfg.s;
  // the persistent FP32 totals instantiation holds three waves per SIMD
  // (its register bound): workgroups of at most 256 threads, so that three
  // of them share a CU (fewer segments per column; the same work items and
  // the same state bits)
  if (TOT && PERSIST && sizeof(T) == 4)
    while (L.cfg.q * s > 256 && s % 2 == 0) s /= 2;
  const int threads = L.cfg.q * s;
  dim3 block(threads);
  // halos through LDS while the table (20 values per thread) fits in 64 KiB
  const size_t tab = size_t(threads) * 20 * sizeof(T);
  const bool ldsh = tab <= 65536;
  const size_t tl = TOT ? size_t(threads) * kTotStride * sizeof(double) : 0;  // totals (TotL)
  SweepArgs<T> a = to_args<T>(L);
  a.s = s;
  if (L.axis == 1) {
    if (ldsh)
      hipLaunchKernelGGL((sweep_col_kernel<T, 1, PERSIST, true, TOT>), grid, block, tl + tab, st,
                         a);
    else
      hipLaunchKernelGGL((sweep_col_kernel<T, 1, PERSIST, false, TOT>), grid, block, tl, st, a);
  } else {
    if (ldsh)
      hipLaunchKernelGGL((sweep_col_kernel<T, 2, PERSIST, true, TOT>), grid, block, tl + tab, st,
                         a);
    else
      hipLaunchKernelGGL((sweep_col_kernel<T, 2, PERSIST, false, TOT>), grid, block, tl, st, a);
  }
  return hipGetLastError();
}

template <class T, int V, bool TOT>
static hipError_t launch_plane_v(const LaunchSweep& L, hipStream_t st) {
  const SweepArgs<T> a = to_args<T>(L);
  // with totals the plane's LDS also takes the per-item reduction
  const size_t lds = std::max(size_t(L.plane_lds), TOT ? size_t(kTotWideBytes) * L.cfg.block : 0);
  if (L.plane == kPlaneXY)
    hipLaunchKernelGGL((sweep_plane_kernel<T, V, true, TOT>), dim3(L.nblocks),
                       dim3(L.cfg.block), lds, st, a);
  else
    hipLaunchKernelGGL((sweep_plane_kernel<T, V, false, TOT>), dim3(L.nblocks),
                       dim3(L.cfg.block), lds, st, a);
  return hipGetLastError();
}

template <class T, bool TOT>
static hipError_t launch_plane(const LaunchSweep& L, hipStream_t st) {
  if (L.plane_lds <= 0 || L.plane_lds > kPlaneLdsBytes || !L.persistent)
    return hipErrorInvalidValue;
  switch (L.cfg.v) {
    case 1: return launch_plane_v<T, 1, TOT>(L, st);
    case 2: return launch_plane_v<T, 2, TOT>(L, st);
    case 4: return launch_plane_v<T, 4, TOT>(L, st);
    default: return hipErrorInvalidValue;
  }
}

template <class T, int V, bool TOT>
static hipError_t launch_window_v(const LaunchSweep& L, hipStream_t st) {
  const SweepArgs<T> a = to_args<T>(L);
  const size_t lds = std::max(size_t(kPlaneLdsBytes), TOT ? size_t(kTotWideBytes) * L.cfg.block : 0);
  if (L.plane == kWinXY)
    hipLaunchKernelGGL((sweep_window_kernel<T, V, true, TOT>), dim3(L.nblocks),
                       dim3(L.cfg.block), lds, st, a);
  else
    hipLaunchKernelGGL((sweep_window_kernel<T, V, false, TOT>), dim3(L.nblocks),
                       dim3(L.cfg.block), lds, st, a);
  return hipGetLastError();
}

template <class T, int V, bool TOT>
static hipError_t launch_zplane_v(const LaunchSweep& L, hipStream_t st) {
  const SweepArgs<T> a = to_args<T>(L);
  const size_t lds = std::max(size_t(L.plane_lds), TOT ? size_t(kTotWideBytes) * L.cfg.block : 0);
  hipLaunchKernelGGL((sweep_zplane_kernel<T, V, TOT>), dim3(L.nblocks), dim3(L.cfg.block), lds,
                     st, a);
  return hipGetLastError();
}

template <class T, bool TOT>
static hipError_t launch_zplane(const LaunchSweep& L, hipStream_t st) {
  if (L.plane_lds <= 0 || L.plane_lds > kPlaneLdsBytes || !L.persistent)
    return hipErrorInvalidValue;
  switch (L.cfg.v) {
    case 1: return launch_zplane_v<T, 1, TOT>(L, st);
    case 2: return launch_zplane_v<T, 2, TOT>(L, st);
    case 4: return launch_zplane_v<T, 4, TOT>(L, st);
    default: return hipErrorInvalidValue;
  }
}

// Window sweeps (a 64 x 64 FP32 or 64 x 32 FP64 plane is the LDS share of a
// workgroup), V = 1 or 2 (window origins are even cells).
template <class T, bool TOT>
static hipError_t launch_window(const LaunchSweep& L, hipStream_t st) {
  if (!L.wins || !L.dst || L.nwin < 1 || L.nblocks < 1 || L.nitems % L.nwin)
    return hipErrorInvalidValue;
  switch (L.cfg.v) {
    case 1: return launch_window_v<T, 1, TOT>(L, st);
    case 2: return launch_window_v<T, 2, TOT>(L, st);
    default: return hipErrorInvalidValue;
  }
}

// TOT: the launch also folds the FP64 totals of the cells it updates (the
// last sweep of a step), a separate instantiation of each kernel so that the
// other sweeps keep their registers.
template <class T, bool TOT>
static hipError_t launch_sweep_tt(const LaunchSweep& L, hipStream_t st) {
  if (L.plane == kWinXY || L.plane == kWinYX) return launch_window<T, TOT>(L, st);
  if (L.plane == kZPlane) return launch_zplane<T, TOT>(L, st);
  if (L.plane != kPlaneNone) return launch_plane<T, TOT>(L, st);
  if (L.persistent) {
    dim3 grid(L.nblocks);
    return L.axis == 0 ? launch_x<T, true, TOT>(L, st, grid)
                       : launch_col<T, true, TOT>(L, st, grid);
  }
  if (L.axis == 0) {
    if (!TOT) return launch_x<T, false, TOT>(L, st, dim3(unsigned(x_grid(L.single, L.cfg))));
    LaunchSweep M = L;
    M.nitems = int32_t(x_tiles(L.single, L.cfg));  // the tiles the capped grid strides over
    return launch_x<T, false, TOT>(M, st, dim3(unsigned(sweep_parts(L))));
  }
  return launch_col<T, false, TOT>(L, st, dim3(unsigned(col_tiles(L.single, L.axis, L.cfg))));
}

template <class T>
static hipError_t launch_sweep_t(const LaunchSweep& L, hipStream_t st) {
  if (L.totals_only && !L.tpart) return hipErrorInvalidValue;
  return L.tpart ? launch_sweep_tt<T, true>(L, st) : launch_sweep_tt<T, false>(L, st);
}

hipError_t launch_sweep(const LaunchSweep& L, hipStream_t st) {
  return L.fp64 ? launch_sweep_t<double>(L, st) : launch_sweep_t<float>(L, st);
}

int64_t sweep_parts(const LaunchSweep& L) {
  if (L.plane == kWinXY || L.plane == kWinYX) return L.nblocks;  // one per workgroup
  if (L.plane != kPlaneNone || L.persistent) return L.nitems;
  if (L.axis == 0) {
    const int64_t g = x_grid(L.single, L.cfg);
    return L.tpart && L.tot_cap > 0 ? std::min<int64_t>(g, L.tot_cap) : g;
  }
  return col_tiles(L.single, L.axis, L.cfg);
}

hipError_t launch_totals_finish(const double* part, int64_t n, double* slice, DevScalars* s,
                                int finish, hipStream_t st) {
  // about 8 partials per thread in each slice, at most kTotalsSlices slices
  int64_t R = (n + 2047) / 2048;
  R = R < 1 ? 1 : (R > kTotalsSlices ? kTotalsSlices : R);
  hipLaunchKernelGGL(totals_finish_kernel, dim3(unsigned(R)), dim3(256), 0, st, part, n, slice,
                     s, finish);
  return hipGetLastError();
}


template <class T>
static ReduceArgs<T> to_rargs(const LaunchReduce& L) {
  ReduceArgs<T> a;
  a.pool = static_cast<const T*>(L.pool);
  a.patches = L.patches;
  a.single = L.single;
  a.gamma = L.gamma;
  for (int i = 0; i < 3; ++i) a.grav[i] = L.grav[i];
  a.scal = L.scal;
  a.partials = L.partials;
  a.psmax = L.psmax;
  return a;
}

// The CFL maximum of the state: with L.psmax one per patch (turned into dt
// per patch by launch_patch_dt), else one, turned into scal->dt here unless
// L.fold_only (a step without sweeps: its bookkeeping takes the maximum).
hipError_t launch_cfl(const LaunchReduce& L, hipStream_t st) {
  dim3 grid(L.chunks, L.npatch);
  if (L.fp64)
    hipLaunchKernelGGL(cfl_kernel<double>, grid, dim3(256), 0, st, to_rargs<double>(L));
  else
    hipLaunchKernelGGL(cfl_kernel<float>, grid, dim3(256), 0, st, to_rargs<float>(L));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || L.psmax || L.fold_only) return e;
  hipLaunchKernelGGL(finish_cfl_kernel, dim3(1), dim3(1), 0, st, L.scal);
  return hipGetLastError();
}

hipError_t launch_totals(const LaunchReduce& L, hipStream_t st) {
  dim3 grid(L.chunks, L.npatch);
  if (L.fp64)
    hipLaunchKernelGGL(totals_kernel<double>, grid, dim3(256), 0, st, to_rargs<double>(L));
  else
    hipLaunchKernelGGL(totals_kernel<float>, grid, dim3(256), 0, st, to_rargs<float>(L));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, st, L.partials,
                     int64_t(L.chunks) * L.npatch, L.scal);
  return hipGetLastError();
}

// In-place streaming pass over a buffer of n16 16-byte words: every word is
// read and written back unchanged (xor with a runtime zero keeps the
// compiler from dropping the pair).  The memory-only ceiling of a sweep.
__global__ void __launch_bounds__(256) stream_kernel(uint4* p, int64_t n16, unsigned zero) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n16;
       i += int64_t(gridDim.x) * 256) {
    uint4 v = p[i];
    v.x ^= zero;
    p[i] = v;
  }
}

hipError_t launch_stream(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(stream_kernel, dim3(unsigned(blocks)), dim3(256), 0, st,
                     static_cast<uint4*>(p), n16, 0u);
  return hipGetLastError();
}

hipError_t launch_finish_step(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(finish_step_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_finish_cfl(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(finish_cfl_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_init_scalars(DevScalars* s, double cfl, double t, double t_end,
                               hipStream_t st) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(1), 0, st, s, cfl, t, t_end);
  return hipGetLastError();
}
// Per-patch time steps (one thread per patch): with advance, t += dt
// first; then the next dt from the patch's folded CFL maximum, capped by
// t_end - t, as next_dt does for a single dt.
__global__ void patch_dt_kernel(double* t, double* dt, unsigned long long* psmax, int32_t n,
                                DevScalars* s, int advance) {
  const int p = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n) return;
  double tp = t[p];
  if (advance) {
    tp += dt[p];
    t[p] = tp;
  }
  const double smax = __longlong_as_double((long long)psmax[p]);
  double d = s->cfl / smax;
  if (!(smax > 0.0) || !(smax < __builtin_huge_val())) {
    atomicOr(&s->error, kErrSpeed);
    d = 0.0;
  }
  if (s->t_end > 0.0) d = fmin(d, fmax(0.0, s->t_end - tp));
  dt[p] = d;
  psmax[p] = 0ull;
}

__global__ void fill_kernel(double* a, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    a[i] = v;
}

hipError_t launch_patch_dt(double* t, double* dt, unsigned long long* psmax, int32_t n,
                           DevScalars* s, int advance, hipStream_t st) {
  hipLaunchKernelGGL(patch_dt_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, t, dt,
                     psmax, n, s, advance);
  return hipGetLastError();
}

hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t st) {
  const int64_t b = std::min<int64_t>((n + 255) / 256, 1024);
  if (b < 1) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(unsigned(b)), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

hipError_t launch_step_results(const DevScalars* s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(step_results_kernel, dim3(1), dim3(1), 0, st, s, out);
  return hipGetLastError();
}
hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t st) {
  hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(1), 0, st, s, dt);
  return hipGetLastError();
}
hipError_t launch_set_time(DevScalars* s, double t, double t_end, hipStream_t st) {
  hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(1), 0, st, s, t, t_end);
  return hipGetLastError();
}
hipError_t launch_clear_error(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(clear_error_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_timing_begin(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(timing_begin_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_timing_end(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(timing_end_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_reset_tickets(DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(reset_tickets_kernel, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}

// the x sweep packs whole pencils into waves when a pencil has at most 64
// lanes; longer pencils span several waves of one workgroup
bool x_wave_ok(int n, int v) { return n % v == 0 && n / v <= 64; }

// LDS bytes of one z-plane (second axis 1) or x-z plane (second axis 2) of
// a patch in the plane sweeps (0 if it does not fit in a workgroup's share)
int plane_lds_bytes(const PatchDev& P, int fp64, int axis2) {
  if (P.n[0] > kPlanePitch) return 0;
  const int64_t b = int64_t(5) * kPlanePitch * P.n[axis2] * (fp64 ? 8 : 4);
  return b <= kPlaneLdsBytes ? int(b) : 0;
}

}  // namespace hydro
