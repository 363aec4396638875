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
  double grav;               // gravity along the sweep axis
  double gamma;
  DevScalars* scal;
};

template <class T>
__device__ __forceinline__ SweepConst<T> make_const(double dt, double dx, double gamma,
                                                    double g) {
  SweepConst<T> k;
  k.gamma = T(gamma);
  k.gm1 = T(gamma - 1.0);
  k.inv_gm1 = T(1.0 / (gamma - 1.0));
  double dtdx = dt / dx;
  k.dtdx = T(dtdx);
  k.half_dtdx = T(0.5 * dtdx);
  k.kick = T(0.5 * dt * g);
  k.dtg = T(dt * g);
  k.has_g = (g != 0.0);
  return k;
}

// plane indices of (normal, transverse 1, transverse 2) momenta per axis
template <int AXIS> struct Rot;
template <> struct Rot<0> { static constexpr int n = 1, t1 = 2, t2 = 3; };
template <> struct Rot<1> { static constexpr int n = 2, t1 = 1, t2 = 3; };
template <> struct Rot<2> { static constexpr int n = 3, t1 = 1, t2 = 2; };

template <class T, int AXIS>
__device__ __forceinline__ Cons<T> load_cell(const T* __restrict__ p, int64_t pl) {
  Cons<T> U;
  U.r = p[0];
  U.mn = p[Rot<AXIS>::n * pl];
  U.mt1 = p[Rot<AXIS>::t1 * pl];
  U.mt2 = p[Rot<AXIS>::t2 * pl];
  U.e = p[4 * pl];
  return U;
}

template <class T, int AXIS>
__device__ __forceinline__ void store_cell(T* __restrict__ p, int64_t pl, const Cons<T>& U) {
  p[0] = U.r;
  p[Rot<AXIS>::n * pl] = U.mn;
  p[Rot<AXIS>::t1 * pl] = U.mt1;
  p[Rot<AXIS>::t2 * pl] = U.mt2;
  p[4 * pl] = U.e;
}

// Signal speed over the cell width, maxed over the active axes, of an
// updated cell.  U is rotated back to the physical frame (rho, mx, my, mz,
// E) first so that the result does not depend on which sweep computed it:
// the folded maximum of a step and a standalone reduction of the same state
// give the same bits.  id* are 1/dx per physical axis, zero when inactive.
template <class T, int AXIS>
__device__ __forceinline__ T cell_speed(const Cons<T>& S, const SweepConst<T>& k,
                                        const T id[3]) {
  Cons<T> U;  // physical frame: mn holds mx, mt1 my, mt2 mz
  U.r = S.r;
  U.e = S.e;
  if (AXIS == 0) { U.mn = S.mn; U.mt1 = S.mt1; U.mt2 = S.mt2; }
  if (AXIS == 1) { U.mn = S.mt1; U.mt1 = S.mn; U.mt2 = S.mt2; }
  if (AXIS == 2) { U.mn = S.mt1; U.mt1 = S.mt2; U.mt2 = S.mn; }
  Prim<T> W = to_prim(U, k);
  T c = sqrt_(k.gamma * W.p * rcp(W.r));
  T s = (fabs_(W.u) + c) * id[0];
  s = fmax_(s, (fabs_(W.t1) + c) * id[1]);
  s = fmax_(s, (fabs_(W.t2) + c) * id[2]);
  return s;
}

template <class T>
__device__ __forceinline__ void inv_widths(const PatchDev& P, T id[3]) {
  for (int a = 0; a < 3; ++a) id[a] = P.n[a] > 1 ? T(1.0 / P.dx[a]) : T(0);
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax_(v, __shfl_xor(v, off));
  return v;
}

// Workgroup max of smax folded into the FP64 atomic, and the sticky error.
template <class T>
__device__ void finish_block(DevScalars* scal, T smax, bool bad, bool do_cfl, T* red) {
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&scal->error, kErrState);
  if (!do_cfl) return;
  T m = wave_max(smax);
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    T b = red[0];
    for (int i = 1; i < nw; ++i) b = fmax_(b, red[i]);
    double d = double(b);
    if (!(d >= 0.0)) d = __builtin_nan("");  // NaN propagates as the largest bits
    unsigned long long bits = (unsigned long long)__double_as_longlong(d);
    atomicMax(&scal->smax_bits, bits);
  }
}

// --------------------------------------------------------------------------
// Lane runs along x
// --------------------------------------------------------------------------

// LDS use per workgroup: 15 values per thread (edge primitives, last face
// state; the first face flux reuses the primitive slots).
template <class T>
constexpr int xlds_values() { return 15; }

template <class T, int V>
__device__ void xsweep_tile(const SweepArgs<T>& a, const PatchDev& P, int64_t tile,
                            const SweepConst<T>& k, T* lds, T& smax, bool& bad) {
  const int N = P.n[0];
  const int LPP = N / V;           // lanes per pencil
  const int B = blockDim.x;
  const int PPW = B / LPP;         // pencils per workgroup
  const int tid = threadIdx.x;
  const int lane = tid % LPP;
  const int pw = tid / LPP;
  const int64_t npen = int64_t(P.n[1]) * P.n[2];
  const int64_t q = tile * PPW + pw;
  const bool act = (pw < PPW) && (q < npen);
  const int64_t pl = P.plane;
  T* base = a.pool + P.base0 + lane * V;
  if (act) base += (q % P.n[1]) * int64_t(P.sy) + (q / P.n[1]) * int64_t(P.sz);

  T* lw = lds;            // [10][B]: W first (0..4), W last (5..9); later F first
  T* lp = lds + 10 * B;   // [5][B]: Wp of the last cell

  Cons<T> U[V];
  Prim<T> W[V];
  if (act) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      U[c] = load_cell<T, 0>(base + c, pl);
      W[c] = to_prim(U[c], k);
    }
    lw[0 * B + tid] = W[0].r; lw[1 * B + tid] = W[0].u; lw[2 * B + tid] = W[0].t1;
    lw[3 * B + tid] = W[0].t2; lw[4 * B + tid] = W[0].p;
    lw[5 * B + tid] = W[V - 1].r; lw[6 * B + tid] = W[V - 1].u; lw[7 * B + tid] = W[V - 1].t1;
    lw[8 * B + tid] = W[V - 1].t2; lw[9 * B + tid] = W[V - 1].p;
  }
  __syncthreads();

  auto read_w = [&](int slot, int t) {
    Prim<T> r;
    r.r = lw[(slot + 0) * B + t]; r.u = lw[(slot + 1) * B + t]; r.t1 = lw[(slot + 2) * B + t];
    r.t2 = lw[(slot + 3) * B + t]; r.p = lw[(slot + 4) * B + t];
    return r;
  };

  Prim<T> Wl, Wr;  // cell left of the first, right of the last
  Prim<T> Wm[V], Wp[V];
  if (act) {
    if (lane > 0) {
      Wl = read_w(5, tid - 1);
    } else if (a.bc_lo == kBcPeriodic) {
      Wl = read_w(5, tid + LPP - 1);
    } else if (a.bc_lo == kBcOutflow) {
      Wl = W[0];
    } else {
      Wl = mirror(W[0]);
    }
    if (lane < LPP - 1) {
      Wr = read_w(0, tid + 1);
    } else if (a.bc_hi == kBcPeriodic) {
      Wr = read_w(0, tid - (LPP - 1));
    } else if (a.bc_hi == kBcOutflow) {
      Wr = W[V - 1];
    } else {
      Wr = mirror(W[V - 1]);
    }
#pragma unroll
    for (int c = 0; c < V; ++c) {
      const Prim<T>& L = c == 0 ? Wl : W[c - 1];
      const Prim<T>& R = c == V - 1 ? Wr : W[c + 1];
      face_states(L, W[c], R, k, k.kick, Wm[c], Wp[c]);
    }
    lp[0 * B + tid] = Wp[V - 1].r; lp[1 * B + tid] = Wp[V - 1].u; lp[2 * B + tid] = Wp[V - 1].t1;
    lp[3 * B + tid] = Wp[V - 1].t2; lp[4 * B + tid] = Wp[V - 1].p;
  }
  __syncthreads();

  Cons<T> F[V];
  if (act) {
    Prim<T> WpL;  // face state W+ of the cell left of the first
    if (lane > 0 || a.bc_lo == kBcPeriodic) {
      int t = lane > 0 ? tid - 1 : tid + LPP - 1;
      WpL.r = lp[0 * B + t]; WpL.u = lp[1 * B + t]; WpL.t1 = lp[2 * B + t];
      WpL.t2 = lp[3 * B + t]; WpL.p = lp[4 * B + t];
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
#pragma unroll
    for (int c = 0; c < V; ++c) F[c] = hllc(c == 0 ? WpL : Wp[c - 1], Wm[c], k);
  }
  __syncthreads();  // every lane has read the primitive slots
  if (act) {
    lw[0 * B + tid] = F[0].r; lw[1 * B + tid] = F[0].mn; lw[2 * B + tid] = F[0].mt1;
    lw[3 * B + tid] = F[0].mt2; lw[4 * B + tid] = F[0].e;
  }
  __syncthreads();
  if (act) {
    Cons<T> FR;  // flux at the right face of the last cell
    if (lane < LPP - 1 || a.bc_hi == kBcPeriodic) {
      int t = lane < LPP - 1 ? tid + 1 : tid - (LPP - 1);
      FR.r = lw[0 * B + t]; FR.mn = lw[1 * B + t]; FR.mt1 = lw[2 * B + t];
      FR.mt2 = lw[3 * B + t]; FR.e = lw[4 * B + t];
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
    T id[3];
    inv_widths<T>(P, id);
#pragma unroll
    for (int c = 0; c < V; ++c) {
      update(U[c], F[c], c == V - 1 ? FR : F[c + 1], k);
      store_cell<T, 0>(base + c, pl, U[c]);
      bad |= !cell_ok(U[c]);
      if (a.do_cfl) smax = fmax_(smax, cell_speed<T, 0>(U[c], k, id));
    }
  }
}

template <class T, int V, bool PERSIST>
__global__ void __launch_bounds__(512) sweep_x_kernel(SweepArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  __shared__ int item_s;
  __shared__ T red[8];
  const double dt = a.scal->dt;
  T smax = T(0);
  bool bad = false;
  if (!PERSIST) {
    SweepConst<T> k = make_const<T>(dt, a.single.dx[0], a.gamma, a.grav);
    xsweep_tile<T, V>(a, a.single, blockIdx.x, k, lds, smax, bad);
  } else {
    for (;;) {
      if (threadIdx.x == 0) item_s = int(atomicAdd(&a.scal->tickets[0], 1u));
      __syncthreads();
      const int it = item_s;
      __syncthreads();
      if (it >= a.nitems) break;
      const WorkItem w = a.items[it];
      const PatchDev P = a.patches[w.patch];
      SweepConst<T> k = make_const<T>(dt, P.dx[0], a.gamma, a.grav);
      xsweep_tile<T, V>(a, P, w.tile, k, lds, smax, bad);
      __syncthreads();
    }
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0, red);
}

// --------------------------------------------------------------------------
// Column marches along y (AXIS 1) or z (AXIS 2)
// --------------------------------------------------------------------------

template <class T, int AXIS>
__device__ void colsweep_tile(const SweepArgs<T>& a, const PatchDev& P, int64_t tile,
                              const SweepConst<T>& k, T& smax, bool& bad) {
  constexpr int TA = AXIS == 1 ? 2 : 1;   // the other transverse axis
  const int N = P.n[AXIS];
  const int nx = P.n[0];
  const int64_t ncol = int64_t(nx) * P.n[TA];
  const int64_t sd = AXIS == 1 ? P.sy : P.sz;
  const int64_t st = AXIS == 1 ? P.sz : P.sy;
  const int Q = a.q, S = a.s;
  const int l = threadIdx.x % Q;
  const int seg = threadIdx.x / Q;
  const int64_t col = tile * Q + l;
  const int L = (N + S - 1) / S;
  const int ja = seg * L;
  const int jb = min(N, ja + L);
  const bool act = (seg < S) && (col < ncol) && (ja < jb);
  const int64_t pl = P.plane;
  T* cbase = a.pool + P.base0;
  if (act) cbase += (col % nx) + (col / nx) * st;

  // halo cells ja-2, ja-1, jb, jb+1 with the boundary conditions applied
  Prim<T> H[4];
  if (act) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      int j = h < 2 ? ja - 2 + h : jb + h - 2;
      bool mir = false;
      if (j < 0) {
        if (a.bc_lo == kBcPeriodic) j += N;
        else if (a.bc_lo == kBcOutflow) j = 0;
        else { j = -j - 1; mir = true; }
      } else if (j >= N) {
        if (a.bc_hi == kBcPeriodic) j -= N;
        else if (a.bc_hi == kBcOutflow) j = N - 1;
        else { j = 2 * N - 1 - j; mir = true; }
      }
      Prim<T> W = to_prim(load_cell<T, AXIS>(cbase + j * sd, pl), k);
      H[h] = mir ? mirror(W) : W;
    }
  }
  __syncthreads();  // every halo copy is taken before any cell is written
  if (!act) return;

  T id[3];
  inv_widths<T>(P, id);
  const T kick_lo = (ja == 0 && a.bc_lo == kBcReflect) ? -k.kick : k.kick;
  const T kick_hi = (jb == N && a.bc_hi == kBcReflect) ? -k.kick : k.kick;

  Cons<T> U0 = load_cell<T, AXIS>(cbase + ja * sd, pl);
  Prim<T> W0 = to_prim(U0, k);
  Cons<T> U1;
  Prim<T> W1;
  if (ja + 1 < jb) {
    U1 = load_cell<T, AXIS>(cbase + (ja + 1) * sd, pl);
    W1 = to_prim(U1, k);
  } else {
    W1 = H[2];
  }
  Prim<T> WpPrev, WmC, WpC, dummy;
  face_states(H[0], H[1], W0, k, kick_lo, dummy, WpPrev);   // cell ja-1
  face_states(H[1], W0, W1, k, k.kick, WmC, WpC);           // cell ja
  Cons<T> Fl = hllc(WpPrev, WmC, k);
  WpPrev = WpC;

  for (int j = ja; j < jb; ++j) {
    Cons<T> U2;
    Prim<T> W2;
    if (j + 2 < jb) {
      U2 = load_cell<T, AXIS>(cbase + int64_t(j + 2) * sd, pl);
      W2 = to_prim(U2, k);
    } else {
      W2 = (j + 2 == jb) ? H[2] : H[3];
    }
    Prim<T> Wm1, Wp1;
    face_states(W0, W1, W2, k, (j + 1 == jb) ? kick_hi : k.kick, Wm1, Wp1);  // cell j+1
    Cons<T> Fr = hllc(WpPrev, Wm1, k);
    update(U0, Fl, Fr, k);
    store_cell<T, AXIS>(cbase + int64_t(j) * sd, pl, U0);
    bad |= !cell_ok(U0);
    if (a.do_cfl) smax = fmax_(smax, cell_speed<T, AXIS>(U0, k, id));
    U0 = U1;
    U1 = U2;
    W0 = W1;
    W1 = W2;
    WpPrev = Wp1;
    Fl = Fr;
  }
}

template <class T, int AXIS, bool PERSIST>
__global__ void __launch_bounds__(512) sweep_col_kernel(SweepArgs<T> a) {
  __shared__ int item_s;
  __shared__ T red[8];
  const double dt = a.scal->dt;
  T smax = T(0);
  bool bad = false;
  if (!PERSIST) {
    SweepConst<T> k = make_const<T>(dt, a.single.dx[AXIS], a.gamma, a.grav);
    colsweep_tile<T, AXIS>(a, a.single, blockIdx.x, k, smax, bad);
  } else {
    for (;;) {
      if (threadIdx.x == 0) item_s = int(atomicAdd(&a.scal->tickets[AXIS], 1u));
      __syncthreads();
      const int it = item_s;
      __syncthreads();
      if (it >= a.nitems) break;
      const WorkItem w = a.items[it];
      const PatchDev P = a.patches[w.patch];
      SweepConst<T> k = make_const<T>(dt, P.dx[AXIS], a.gamma, a.grav);
      colsweep_tile<T, AXIS>(a, P, w.tile, k, smax, bad);
      __syncthreads();
    }
  }
  finish_block(a.scal, smax, bad, a.do_cfl != 0, red);
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
};

template <class T>
__global__ void __launch_bounds__(256) cfl_kernel(ReduceArgs<T> a) {
  __shared__ T red[16];
  const PatchDev P = a.patches ? a.patches[blockIdx.y] : a.single;
  const int64_t cells = int64_t(P.n[0]) * P.n[1] * P.n[2];
  SweepConst<T> k = make_const<T>(0.0, 1.0, a.gamma, 0.0);
  T id[3];
  inv_widths<T>(P, id);
  T smax = T(0);
  bool bad = false;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cells;
       c += int64_t(gridDim.x) * blockDim.x) {
    int x = int(c % P.n[0]);
    int64_t r = c / P.n[0];
    int y = int(r % P.n[1]);
    int z = int(r / P.n[1]);
    const T* p = a.pool + P.base0 + x + int64_t(y) * P.sy + int64_t(z) * P.sz;
    Cons<T> U = load_cell<T, 0>(p, P.plane);
    bad |= !cell_ok(U);
    smax = fmax_(smax, cell_speed<T, 0>(U, k, id));
  }
  finish_block(a.scal, smax, bad, true, red);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
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
  s->tickets[0] = s->tickets[1] = s->tickets[2] = s->tickets[3] = 0u;
  s->saved[0] = s->saved[1] = 0.0;
  for (int v = 0; v < 6; ++v) s->totals[v] = 0.0;
}

__global__ void set_dt_kernel(DevScalars* s, double dt) { s->dt = dt; }
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
};

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
  a.grav = L.grav;
  a.gamma = L.gamma;
  a.scal = L.scal;
  return a;
}

int64_t x_tiles(const PatchDev& P, const SweepCfg& c) {
  int lpp = P.n[0] / c.v;
  int ppw = c.block / lpp;
  int64_t npen = int64_t(P.n[1]) * P.n[2];
  return (npen + ppw - 1) / ppw;
}

int64_t col_tiles(const PatchDev& P, int axis, const SweepCfg& c) {
  int64_t ncol = int64_t(P.n[0]) * P.n[axis == 1 ? 2 : 1];
  return (ncol + c.q - 1) / c.q;
}

template <class T, int V, bool PERSIST>
static hipError_t launch_x_v(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  size_t lds = size_t(xlds_values<T>()) * L.cfg.block * sizeof(T);
  hipLaunchKernelGGL((sweep_x_kernel<T, V, PERSIST>), grid, dim3(L.cfg.block), lds, st,
                     to_args<T>(L));
  return hipGetLastError();
}

template <class T, bool PERSIST>
static hipError_t launch_x(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  switch (L.cfg.v) {
    case 1: return launch_x_v<T, 1, PERSIST>(L, st, grid);
    case 2: return launch_x_v<T, 2, PERSIST>(L, st, grid);
    case 4: return launch_x_v<T, 4, PERSIST>(L, st, grid);
    default: return hipErrorInvalidValue;
  }
}

template <class T, bool PERSIST>
static hipError_t launch_col(const LaunchSweep& L, hipStream_t st, dim3 grid) {
  dim3 block(L.cfg.q * L.cfg.s);
  if (L.axis == 1)
    hipLaunchKernelGGL((sweep_col_kernel<T, 1, PERSIST>), grid, block, 0, st, to_args<T>(L));
  else
    hipLaunchKernelGGL((sweep_col_kernel<T, 2, PERSIST>), grid, block, 0, st, to_args<T>(L));
  return hipGetLastError();
}

template <class T>
static hipError_t launch_sweep_t(const LaunchSweep& L, hipStream_t st) {
  if (L.persistent) {
    dim3 grid(L.nblocks);
    return L.axis == 0 ? launch_x<T, true>(L, st, grid) : launch_col<T, true>(L, st, grid);
  }
  if (L.axis == 0) return launch_x<T, false>(L, st, dim3(unsigned(x_tiles(L.single, L.cfg))));
  return launch_col<T, false>(L, st, dim3(unsigned(col_tiles(L.single, L.axis, L.cfg))));
}

hipError_t launch_sweep(const LaunchSweep& L, hipStream_t st) {
  return L.fp64 ? launch_sweep_t<double>(L, st) : launch_sweep_t<float>(L, st);
}

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
};

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
  return a;
}

hipError_t launch_cfl(const LaunchReduce& L, hipStream_t st) {
  dim3 grid(L.chunks, L.npatch);
  if (L.fp64)
    hipLaunchKernelGGL(cfl_kernel<double>, grid, dim3(256), 0, st, to_rargs<double>(L));
  else
    hipLaunchKernelGGL(cfl_kernel<float>, grid, dim3(256), 0, st, to_rargs<float>(L));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
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

size_t x_lds_bytes(const SweepCfg& c, int fp64) {
  return size_t(15) * c.block * (fp64 ? 8 : 4);
}

}  // namespace hydro
