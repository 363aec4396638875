// amr.hip -- operators around the batched patches for adaptive refinement
// (ratio 2): the stored ghost layers, conservative restriction and
// MC-limited conservative prolongation.
//
// The paper's codes run the hydrodynamics on adaptively refined grids (its
// description of their capabilities) without fixing these operators; they
// are the standard conservative ones.  The sweep kernels apply the physical
// boundary conditions on the fly and never read stored ghosts, so these are
// for the layers around the step: regridding, coarse-fine data exchange,
// output and checkpoints.  Every operator is one HBM-bound pass over the
// cells it writes, and each reproduces its definition's floating-point
// operations in order, so results are bitwise those of a plain evaluation:
//   * ghosts: stored index i of an axis maps to interior i (inside), to
//     i mod n (periodic), to the edge cell (outflow) or to the mirror image
//     with period 2n (reflect: ghost -k copies cell k-1), axis by axis; the
//     momentum normal to a reflecting side is negated;
//   * restriction: coarse = (sum of the 8 children in (dz, dy, dx) order)/8;
//   * prolongation: child = ((U_c + s_x D_x) + s_y D_y) + s_z D_z with
//     s = -1/4 or +1/4 and D the monotonised-central slope from the two
//     coarse neighbours along each axis; for the ghosts of a subcycled fine
//     step, U_c is first interpolated in time, U_old + theta (U - U_old);
//   * flux registers: the flux of a sweep through the coarse-fine faces,
//     evaluated from the cells the sweep reads with the sweep's own
//     arithmetic (euler.hpp), so a coarse register holds the very flux the
//     coarse update applied; fine fluxes are averaged over the 2 x 2 fine
//     faces of a coarse face in (t2, t1) order;
//   * refluxing: the uncovered coarse cell across a coarse-fine face trades
//     the coarse flux for the fine one, U += (R_c - R_f)/dx on a patch's low
//     side and (R_f - R_c)/dx on its high side (Berger & Colella 1989).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "euler.hpp"
#include "launch.hpp"

namespace hydro {

constexpr int kAmrBlock = 256;

// Interior source of stored index i (interior 0..n-1) along one axis.
__device__ __forceinline__ int ghost_src(int i, int n, int bclo, int bchi, bool& flip) {
  if (i >= 0 && i < n) return i;
  const int bc = i < 0 ? bclo : bchi;
  if (bc == kBcPeriodic) {
    const int m = i % n;
    return m < 0 ? m + n : m;
  }
  if (bc == kBcOutflow) return i < 0 ? 0 : n - 1;
  flip = true;
  const int k = i < 0 ? -i - 1 : i - n;  // distance beyond the edge
  const int m = k % (2 * n);
  const int d = m < n ? m : 2 * n - 1 - m;
  return i < 0 ? d : n - 1 - d;
}

template <class T>
struct AmrArgs {
  T* pool;
  const PatchDev* patches;  // null: single grid
  PatchDev single;
  int ng;                   // single grid: stored ghost layers
  int bc[6];
  AmrLink links[kAmrLinksPerLaunch];
  int ghosts_only;
  T* fpool;                 // fine side of the links
  const PatchDev* fpatches;
  int finset;
  const T* cold;            // prolongation: coarse data at the start of the step
  int margin;               // snapshot: coarse cells around each covered box
  double theta;
  double* reg;
  int64_t nreg;
  int link0, maxface;
  int axis, side, fine;
  double dt, weight, gamma, grav;
  const AmrLink* dlinks;
};

// Link blockIdx.y of a launch.
template <class T>
__device__ __forceinline__ AmrLink link_of(const AmrArgs<T>& a) {
  return a.dlinks ? a.dlinks[blockIdx.y] : a.links[blockIdx.y];
}

// Fine patch of a link: the table entry, or the patch inside a ghost-free
// stored box whose outer `inset` layers are its ghost shell.
__device__ __forceinline__ PatchDev fine_patch(const PatchDev* t, int i, int inset) {
  PatchDev F = t[i];
  if (inset) {
    F.base0 += int64_t(inset) * (1 + int64_t(F.sy) + int64_t(F.sz));
    for (int a = 0; a < 3; ++a) F.n[a] -= 2 * inset;
    F.ng = inset;
  }
  return F;
}

// Element stride of an axis, and the two transverse axes of a sweep along
// `axis` in ascending order.
__device__ __forceinline__ int64_t axis_stride(const PatchDev& P, int a) {
  return a == 0 ? 1 : a == 1 ? int64_t(P.sy) : int64_t(P.sz);
}
// Component a of a 3-vector by selects (a runtime index into a local array
// would put the array in scratch memory).
template <class U>
__device__ __forceinline__ U sel3(int a, U x, U y, U z) {
  return a == 0 ? x : a == 1 ? y : z;
}
__device__ __forceinline__ int ext(const PatchDev& P, int a) {
  return sel3(a, P.n[0], P.n[1], P.n[2]);
}
__device__ __forceinline__ double width(const PatchDev& P, int a) {
  return sel3(a, P.dx[0], P.dx[1], P.dx[2]);
}
__device__ __forceinline__ int t1_of(int axis) { return axis == 0 ? 1 : 0; }
__device__ __forceinline__ int t2_of(int axis) { return axis == 2 ? 1 : 2; }

// Every stored ghost cell of the grid (y = 0) or of patch blockIdx.y, from
// the interior.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) fill_ghosts_kernel(AmrArgs<T> a) {
  const PatchDev P = a.patches ? a.patches[blockIdx.y] : a.single;
  const int g = a.patches ? P.ng : a.ng;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const unsigned sx = unsigned(nx + 2 * g), sxy = sx * unsigned(ny + 2 * g);
  const unsigned total = sxy * unsigned(nz + 2 * g);  // a stored patch holds < 2^32 cells
  T* p0 = a.pool + P.base0;
  for (unsigned c = blockIdx.x * kAmrBlock + threadIdx.x; c < total;
       c += gridDim.x * kAmrBlock) {
    const unsigned kk = c / sxy, rem = c - kk * sxy;
    const unsigned jj = rem / sx;
    const int k = int(kk) - g, j = int(jj) - g, i = int(rem - jj * sx) - g;
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) continue;
    bool fx = false, fy = false, fz = false;
    const int si = ghost_src(i, nx, a.bc[0], a.bc[1], fx);
    const int sj = ghost_src(j, ny, a.bc[2], a.bc[3], fy);
    const int sk = ghost_src(k, nz, a.bc[4], a.bc[5], fz);
    const int64_t src = int64_t(si) + int64_t(sj) * P.sy + int64_t(sk) * P.sz;
    const int64_t dst = int64_t(i) + int64_t(j) * P.sy + int64_t(k) * P.sz;
    p0[dst] = p0[src];
    p0[dst + P.plane] = fx ? -p0[src + P.plane] : p0[src + P.plane];
    p0[dst + 2 * P.plane] = fy ? -p0[src + 2 * P.plane] : p0[src + 2 * P.plane];
    p0[dst + 3 * P.plane] = fz ? -p0[src + 3 * P.plane] : p0[src + 3 * P.plane];
    p0[dst + 4 * P.plane] = p0[src + 4 * P.plane];
  }
}

// Coarse cells covered by the fine patch of link blockIdx.y.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) restrict_kernel(AmrArgs<T> a) {
  const AmrLink L = link_of(a);
  const PatchDev F = fine_patch(a.fpatches, L.fine, a.finset), C = a.patches[L.coarse];
  const unsigned cx = unsigned(F.n[0] / 2), cxy = cx * unsigned(F.n[1] / 2);
  const unsigned total = cxy * unsigned(F.n[2] / 2);
  const T* f0 = a.fpool + F.base0;
  T* c0 = a.pool + C.base0;
  if (blockIdx.x * kAmrBlock >= total) return;
  for (unsigned c = blockIdx.x * kAmrBlock + threadIdx.x; c < total;
       c += gridDim.x * kAmrBlock) {
    const unsigned k = c / cxy, rem = c - k * cxy;
    const unsigned j = rem / cx, i = rem - j * cx;
    const int64_t fb = int64_t(2 * i) + int64_t(2 * j) * F.sy + int64_t(2 * k) * F.sz;
    const int64_t cb = int64_t(L.ox + int(i)) + int64_t(L.oy + int(j)) * C.sy +
                       int64_t(L.oz + int(k)) * C.sz;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T* f = f0 + fb + v * F.plane;
      double s = 0.0;
      bool first = true;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const double x = double(f[dx + dy * F.sy + dz * F.sz]);
            s = first ? x : s + x;
            first = false;
          }
      c0[cb + v * C.plane] = T(s * 0.125);
    }
  }
}

// Monotonised-central slope from one-sided differences a and b: zero unless
// both are strictly positive or both strictly negative (a sign test: a
// product of two tiny differences could underflow to zero).
__device__ __forceinline__ double mc_slope(double a, double b) {
  const double m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
  const bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
  return same ? copysign(m, a) : 0.0;
}

// Fine cells (interior, or the stored ghost shell) of link blockIdx.y, one
// coarse parent per thread: the parent's value and its three limited slopes
// are formed once and give each of its children that is written.  SHELL (a
// thin ghost shell): only the parents with a ghost child, and variable
// blockIdx.z per thread; else the whole box of parents, all five variables
// per thread (their loads issued together).
template <class T, bool COLD, bool SHELL>
__global__ void __launch_bounds__(kAmrBlock) prolong_kernel(AmrArgs<T> a) {
  const AmrLink L = link_of(a);
  const PatchDev F = fine_patch(a.fpatches, L.fine, a.finset), C = a.patches[L.coarse];
  const int nx = F.n[0], ny = F.n[1], nz = F.n[2];
  const int g = a.ghosts_only ? F.ng : 0;
  // parents of the fine cells -g .. n + g - 1 along each axis
  const int lo = (-g) >> 1;
  const unsigned px = unsigned(((nx + g - 1) >> 1) - lo + 1);
  const unsigned py = unsigned(((ny + g - 1) >> 1) - lo + 1);
  const unsigned pz = unsigned(((nz + g - 1) >> 1) - lo + 1);
  const unsigned pxy = px * py;
  // ghosts only: the parents outside the block of parents [0, (n + 1) / 2)
  // along some axis (the others have every child in the interior), as three
  // parts: whole planes below and above the block along z; within the
  // block's z range, whole rows below and above it along y; within both,
  // the cells below and above it along x
  const unsigned ix = unsigned((nx + 1) >> 1), iy = unsigned((ny + 1) >> 1),
                 iz = unsigned((nz + 1) >> 1);
  const unsigned oz = pz - iz, oy = py - iy, ox = px - ix;
  const unsigned nz_part = oz * pxy, ny_part = iz * oy * px;
  const unsigned total = SHELL ? pxy * pz - ix * iy * iz : pxy * pz;
  // t-th parent outside the block [0, I) along an axis: lo .. -1, then I ..
  auto outside = [&](unsigned t, unsigned I) {
    return int(t) < -lo ? lo + int(t) : int(I) + int(t) + lo;
  };
  T* f0 = a.fpool + F.base0;
  const T* c0 = a.pool + C.base0;
  const T* o0 = COLD ? a.cold + C.base0 : nullptr;
  const double th = a.theta;
  if (blockIdx.x * kAmrBlock >= total) return;
  for (unsigned c = blockIdx.x * kAmrBlock + threadIdx.x; c < total;
       c += gridDim.x * kAmrBlock) {
    int pi, pj, pk;
    if (!SHELL) {
      const unsigned kk = c / pxy, rem = c - kk * pxy;
      const unsigned jj = rem / px;
      pk = int(kk) + lo;
      pj = int(jj) + lo;
      pi = int(rem - jj * px) + lo;
      // a parent whose children are all interior has none in the ghost shell
      if (a.ghosts_only && pi >= 0 && 2 * pi < nx && pj >= 0 && 2 * pj < ny && pk >= 0 &&
          2 * pk < nz)
        continue;
    } else if (c < nz_part) {
      const unsigned kk = c / pxy, rem = c - kk * pxy;
      const unsigned jj = rem / px;
      pk = outside(kk, iz);
      pj = int(jj) + lo;
      pi = int(rem - jj * px) + lo;
    } else if (c < nz_part + ny_part) {
      const unsigned d = c - nz_part, row = oy * px;
      const unsigned kk = d / row, rem = d - kk * row;
      const unsigned jj = rem / px;
      pk = int(kk);
      pj = outside(jj, iy);
      pi = int(rem - jj * px) + lo;
    } else {
      const unsigned d = c - nz_part - ny_part, row = iy * ox;
      const unsigned kk = d / row, rem = d - kk * row;
      const unsigned jj = rem / ox;
      pk = int(kk);
      pj = int(jj);
      pi = outside(rem - jj * ox, ix);
    }
    const int64_t pc = int64_t(L.ox + pi) + int64_t(L.oy + pj) * C.sy +
                       int64_t(L.oz + pk) * C.sz;
    const int v0 = SHELL ? int(blockIdx.z) : 0;
#pragma unroll
    for (int v = v0; v < (SHELL ? v0 + 1 : 5); ++v) {
      const T* q = c0 + pc + v * C.plane;
      const T* qo = COLD ? o0 + pc + v * C.plane : nullptr;
      // coarse value at offset d, interpolated in time when a start copy is given
      auto cv = [&](int64_t d) {
        if constexpr (!COLD) {
          return double(q[d]);
        } else {
          const double o = double(qo[d]);
          return o + th * (double(q[d]) - o);
        }
      };
      const double u = cv(0);
      const double dx = mc_slope(u - cv(-1), cv(1) - u);
      const double dy = mc_slope(u - cv(-C.sy), cv(C.sy) - u);
      const double dz = mc_slope(u - cv(-C.sz), cv(C.sz) - u);
      T* fv = f0 + v * F.plane;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        const int i = 2 * pi + (ch & 1), j = 2 * pj + ((ch >> 1) & 1), k = 2 * pk + (ch >> 2);
        if (i < -g || i >= nx + g || j < -g || j >= ny + g || k < -g || k >= nz + g) continue;
        const bool inside = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
        if (inside == bool(a.ghosts_only)) continue;
        const double ox = (ch & 1) ? 0.25 : -0.25, oy = ((ch >> 1) & 1) ? 0.25 : -0.25,
                     oz = (ch >> 2) ? 0.25 : -0.25;
        fv[int64_t(i) + int64_t(j) * F.sy + int64_t(k) * F.sz] =
            T(((u + ox * dx) + oy * dy) + oz * dz);
      }
    }
  }
}

// Copy of the coarse cells within a.margin of the box link blockIdx.y
// covers (every cell its ghost prolongation reads), into a.cold at the
// pool's offsets.  Boxes of neighbouring links may overlap; they copy the
// same values.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) snapshot_kernel(AmrArgs<T> a) {
  const AmrLink L = link_of(a);
  const PatchDev F = fine_patch(a.fpatches, L.fine, a.finset), C = a.patches[L.coarse];
  const int m = a.margin;
  const unsigned bx = unsigned(F.n[0] / 2 + 2 * m), bxy = bx * unsigned(F.n[1] / 2 + 2 * m);
  const unsigned total = bxy * unsigned(F.n[2] / 2 + 2 * m);
  const T* c0 = a.pool + C.base0;
  T* o0 = const_cast<T*>(a.cold) + C.base0;
  for (unsigned c = blockIdx.x * kAmrBlock + threadIdx.x; c < total;
       c += gridDim.x * kAmrBlock) {
    const unsigned kk = c / bxy, rem = c - kk * bxy;
    const unsigned jj = rem / bx;
    const int64_t cell = int64_t(L.ox - m + int(rem - jj * bx)) +
                         int64_t(L.oy - m + int(jj)) * C.sy + int64_t(L.oz - m + int(kk)) * C.sz;
#pragma unroll
    for (int v = 0; v < 5; ++v) o0[cell + v * C.plane] = c0[cell + v * C.plane];
  }
}

// Flux through the face between cells f - 1 and f along `axis` at
// transverse indices (i1, i2), from the four cells f - 2 .. f + 1 exactly as
// a sweep computes it (interior cells: the full gravity half kick).
// Returned in the sweep frame (rho, m_n, m_t1, m_t2, E); lab_var maps a
// sweep-frame component to its lab index (kept out of the local array so
// that it stays in registers).
__device__ __forceinline__ int lab_var(int axis, int v) {
  return v == 1 ? 1 + axis : v == 2 ? 1 + t1_of(axis) : v == 3 ? 1 + t2_of(axis) : v;
}

template <class T>
__device__ __forceinline__ void face_flux(const T* p0, const PatchDev& P, int axis, int f,
                                          int i1, int i2, const SweepConst<T>& k,
                                          double out[5]) {
  const int a1 = t1_of(axis), a2 = t2_of(axis);
  const int64_t sd = axis_stride(P, axis);
  const int64_t c0 = int64_t(f) * sd + int64_t(i1) * axis_stride(P, a1) +
                     int64_t(i2) * axis_stride(P, a2);
  Prim<T> W[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T* q = p0 + c0 + (m - 2) * sd;
    Cons<T> U;
    U.r = q[0];
    U.mn = q[(1 + axis) * P.plane];
    U.mt1 = q[(1 + a1) * P.plane];
    U.mt2 = q[(1 + a2) * P.plane];
    U.e = q[4 * P.plane];
    W[m] = to_prim(U, k);
  }
  Prim<T> Wm0, Wp0, Wm1, Wp1;
  face_states(W[0], W[1], W[2], k, k.kick, Wm0, Wp0);  // cell f - 1
  face_states(W[1], W[2], W[3], k, k.kick, Wm1, Wp1);  // cell f
  const Cons<T> F = hllc(Wp0, Wm1, k);
  out[0] = double(F.r);
  out[1] = double(F.mn);
  out[2] = double(F.mt1);
  out[3] = double(F.mt2);
  out[4] = double(F.e);
}

// Flux registers of link blockIdx.y, side blockIdx.z, along a.axis: coarse
// faces (a.fine = 0) or the means of the fine faces (a.fine = 1), times
// a.weight, added to the register.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) flux_reg_kernel(AmrArgs<T> a) {
  const AmrLink L = link_of(a);
  const int side = int(blockIdx.z);
  const PatchDev F = fine_patch(a.fpatches, L.fine, a.finset);
  const int axis = a.axis, a1 = t1_of(axis), a2 = t2_of(axis);
  const int m1 = ext(F, a1) / 2, m2 = ext(F, a2) / 2;
  const int nface = m1 * m2;
  double* reg = a.reg + (a.fine ? a.nreg : 0) +
                (((int64_t(a.link0) + blockIdx.y) * 3 + axis) * 2 + side) * a.maxface * 5;
  const PatchDev C = a.patches[L.coarse];
  const SweepConst<T> k = make_const<T>(a.dt, a.fine ? width(F, axis) : width(C, axis),
                                        a.gamma, a.grav);
  double acc[5];
  if (!a.fine) {
    const int f = sel3(axis, L.ox, L.oy, L.oz) + (side ? ext(F, axis) / 2 : 0);
    const int c1 = sel3(a1, L.ox, L.oy, L.oz), c2 = sel3(a2, L.ox, L.oy, L.oz);
    for (int fc = blockIdx.x * kAmrBlock + threadIdx.x; fc < nface;
         fc += gridDim.x * kAmrBlock) {
      const int j1 = fc % m1, j2 = fc / m1;
      face_flux(a.pool + C.base0, C, axis, f, c1 + j1, c2 + j2, k, acc);
#pragma unroll
      for (int v = 0; v < 5; ++v) reg[int64_t(fc) * 5 + lab_var(axis, v)] += a.weight * acc[v];
    }
  } else if (axis == 0) {
    // x faces: sixteen lanes per coarse face, lane 4q + m on cell m of the
    // 4-cell stencil of fine face q (t2, t1 offsets (q >> 1, q & 1)), so the
    // four lanes of a stencil read one contiguous run.  Each lane forms its
    // cell's primitives; the face states of cells f - 1 (m = 1) and f (m = 2)
    // take their neighbours' primitives by shuffle, and lane m = 2 forms the
    // flux from exactly the operands a sweep uses.  The segment's first lane
    // sums the four fine fluxes in the order (0,0), (0,1), (1,0), (1,1).
    const int f = side ? ext(F, 0) : 0;
    const int l = threadIdx.x & 15, q = l >> 2, m = l & 3;
    for (int t = blockIdx.x * kAmrBlock + threadIdx.x; t < 16 * nface;
         t += gridDim.x * kAmrBlock) {
      const int fc = t >> 4;
      const int j1 = fc % m1, j2 = fc / m1;
      const int64_t cell = int64_t(f - 2 + m) + int64_t(2 * j1 + (q & 1)) * F.sy +
                           int64_t(2 * j2 + (q >> 1)) * F.sz;
      const T* c = a.fpool + F.base0 + cell;
      Cons<T> U;
      U.r = c[0];
      U.mn = c[F.plane];
      U.mt1 = c[2 * F.plane];
      U.mt2 = c[3 * F.plane];
      U.e = c[4 * F.plane];
      const Prim<T> W = to_prim(U, k);
      // neighbours m - 1 and m + 1 within the stencil (the ends take
      // unused values)
      Prim<T> Wl, Wr;
      Wl.r = __shfl(W.r, l - 1, 16);
      Wl.u = __shfl(W.u, l - 1, 16);
      Wl.t1 = __shfl(W.t1, l - 1, 16);
      Wl.t2 = __shfl(W.t2, l - 1, 16);
      Wl.p = __shfl(W.p, l - 1, 16);
      Wl.ri = T(0);
      Wr.r = __shfl(W.r, l + 1, 16);
      Wr.u = __shfl(W.u, l + 1, 16);
      Wr.t1 = __shfl(W.t1, l + 1, 16);
      Wr.t2 = __shfl(W.t2, l + 1, 16);
      Wr.p = __shfl(W.p, l + 1, 16);
      Wr.ri = T(0);
      Prim<T> Wm, Wp;
      face_states(Wl, W, Wr, k, k.kick, Wm, Wp);
      // lane m = 2 takes W+ of cell f - 1 from lane m = 1
      Prim<T> L1;
      L1.r = __shfl(Wp.r, l - 1, 16);
      L1.u = __shfl(Wp.u, l - 1, 16);
      L1.t1 = __shfl(Wp.t1, l - 1, 16);
      L1.t2 = __shfl(Wp.t2, l - 1, 16);
      L1.p = __shfl(Wp.p, l - 1, 16);
      L1.ri = T(0);
      const Cons<T> Fx = hllc(L1, Wm, k);
      const double fl[5] = {double(Fx.r), double(Fx.mn), double(Fx.mt1), double(Fx.mt2),
                            double(Fx.e)};
      double s5[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double x0 = __shfl(fl[v], 2, 16), x1 = __shfl(fl[v], 6, 16);
        const double x2 = __shfl(fl[v], 10, 16), x3 = __shfl(fl[v], 14, 16);
        s5[v] = ((x0 + x1) + x2) + x3;
      }
      if (l == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
          reg[int64_t(fc) * 5 + lab_var(0, v)] += a.weight * (0.25 * s5[v]);
      }
    }
  } else {
    // four consecutive lanes per coarse face, lane q on the fine face with
    // (t2, t1) offsets (q >> 1, q & 1); the group's first lane sums the four
    // in the order (0,0), (0,1), (1,0), (1,1).  Groups are whole: the block
    // size and the trip bound are multiples of 4.
    const int f = side ? ext(F, axis) : 0;
    const int q = threadIdx.x & 3;
    for (int t = blockIdx.x * kAmrBlock + threadIdx.x; t < 4 * nface;
         t += gridDim.x * kAmrBlock) {
      const int fc = t >> 2;
      const int j1 = fc % m1, j2 = fc / m1;
      face_flux(a.fpool + F.base0, F, axis, f, 2 * j1 + (q & 1), 2 * j2 + (q >> 1), k, acc);
      double s[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double x0 = __shfl(acc[v], 0, 4), x1 = __shfl(acc[v], 1, 4);
        const double x2 = __shfl(acc[v], 2, 4), x3 = __shfl(acc[v], 3, 4);
        s[v] = ((x0 + x1) + x2) + x3;
      }
      if (q == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
          reg[int64_t(fc) * 5 + lab_var(axis, v)] += a.weight * (0.25 * s[v]);
      }
    }
  }
}
static_assert(kAmrBlock % 16 == 0, "whole lane groups per workgroup");

// Refluxing of link blockIdx.y across its a.side faces along a.axis.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) reflux_kernel(AmrArgs<T> a) {
  const AmrLink L = link_of(a);
  const PatchDev F = fine_patch(a.fpatches, L.fine, a.finset);
  const PatchDev C = a.patches[L.coarse];
  const int axis = a.axis, a1 = t1_of(axis), a2 = t2_of(axis), side = a.side;
  const int m1 = ext(F, a1) / 2, m2 = ext(F, a2) / 2;
  const int nface = m1 * m2;
  const int od = sel3(axis, L.ox, L.oy, L.oz);
  const int c1 = sel3(a1, L.ox, L.oy, L.oz), c2 = sel3(a2, L.ox, L.oy, L.oz);
  const int64_t ro = (((int64_t(a.link0) + blockIdx.y) * 3 + axis) * 2 + side) * a.maxface * 5;
  const double* rc = a.reg + ro;
  const double* rf = a.reg + a.nreg + ro;
  const int c = side ? od + ext(F, axis) / 2 : od - 1;  // the uncovered coarse cell
  const double dx = width(C, axis);
  T* c0 = a.pool + C.base0;
  for (int fc = blockIdx.x * kAmrBlock + threadIdx.x; fc < nface; fc += gridDim.x * kAmrBlock) {
    const int j1 = fc % m1, j2 = fc / m1;
    const int64_t cell = int64_t(c) * axis_stride(C, axis) +
                         int64_t(c1 + j1) * axis_stride(C, a1) +
                         int64_t(c2 + j2) * axis_stride(C, a2);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double rcv = rc[int64_t(fc) * 5 + v], rfv = rf[int64_t(fc) * 5 + v];
      const double delta = side ? rfv - rcv : rcv - rfv;
      T* u = c0 + cell + v * C.plane;
      *u = T(double(*u) + delta / dx);
    }
  }
}

template <class T>
static AmrArgs<T> to_aargs(const LaunchAmr& L) {
  AmrArgs<T> a{};
  a.pool = static_cast<T*>(L.pool);
  a.patches = L.patches;
  a.single = L.single;
  a.ng = L.ng;
  for (int i = 0; i < 6; ++i) a.bc[i] = L.bc[i];
  // by-value links only without a device table (launch_amr caps them at
  // kAmrLinksPerLaunch); with one, nlinks may exceed the array
  if (!L.dlinks) {
    const int m = std::min<int32_t>(L.nlinks, kAmrLinksPerLaunch);
    for (int i = 0; i < m; ++i) a.links[i] = L.links[i];
  }
  a.ghosts_only = L.ghosts_only;
  a.fpool = L.fpool ? static_cast<T*>(L.fpool) : a.pool;
  a.fpatches = L.fpatches ? L.fpatches : L.patches;
  a.finset = L.finset;
  a.cold = static_cast<const T*>(L.cold);
  a.margin = L.margin;
  a.theta = L.theta;
  a.reg = L.reg;
  a.nreg = L.nreg;
  a.link0 = L.link0;
  a.maxface = L.maxface;
  a.axis = L.axis;
  a.side = L.side;
  a.fine = L.fine;
  a.dt = L.dt;
  a.weight = L.weight;
  a.gamma = L.gamma;
  a.grav = L.grav;
  a.dlinks = L.dlinks;
  return a;
}

struct LinkChunk {
  AmrLink l[kAmrLinksPerLaunch];
};

__global__ void upload_links_kernel(AmrLink* dst, LinkChunk src, int n) {
  const int i = int(threadIdx.x);
  if (i < n) dst[i] = src.l[i];
}

hipError_t launch_amr_upload(AmrLink* dst, const AmrLink* src, int32_t n, hipStream_t st) {
  for (int32_t b = 0; b < n; b += kAmrLinksPerLaunch) {
    LinkChunk c{};
    const int m = std::min<int32_t>(kAmrLinksPerLaunch, n - b);
    for (int i = 0; i < m; ++i) c.l[i] = src[b + i];
    hipLaunchKernelGGL(upload_links_kernel, dim3(1), dim3(kAmrLinksPerLaunch), 0, st, dst + b,
                       c, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static_assert(sizeof(AmrArgs<double>) <= 4096, "AMR kernel arguments exceed 4 KiB");

static unsigned amr_blocks(int64_t cells) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>((cells + kAmrBlock - 1) / kAmrBlock,
                                                         kAmrMaxBlocks)));
}

template <class T>
static hipError_t launch_amr_t(const LaunchAmr& L, hipStream_t st) {
  const AmrArgs<T> a = to_aargs<T>(L);
  if (L.op == kAmrFill) {
    // a batch: a few workgroups per patch striding over its stored cells
    const unsigned ny = L.patches ? unsigned(L.npatch) : 1u;
    const unsigned nx = L.patches ? std::min(amr_blocks(L.cells), 32u) : amr_blocks(L.cells);
    hipLaunchKernelGGL(fill_ghosts_kernel<T>, dim3(nx, ny), dim3(kAmrBlock), 0, st, a);
  } else if (L.op == kAmrRestrict) {
    hipLaunchKernelGGL(restrict_kernel<T>, dim3(amr_blocks(L.cells), unsigned(L.nlinks)),
                       dim3(kAmrBlock), 0, st, a);
  } else if (L.op == kAmrProlong) {
    const dim3 grid(amr_blocks(L.cells), unsigned(L.nlinks), L.shell ? 5u : 1u);
    if (L.shell && !L.ghosts_only) return hipErrorInvalidValue;
    if (L.cold) {
      if (L.shell)
        hipLaunchKernelGGL((prolong_kernel<T, true, true>), grid, dim3(kAmrBlock), 0, st, a);
      else
        hipLaunchKernelGGL((prolong_kernel<T, true, false>), grid, dim3(kAmrBlock), 0, st, a);
    } else {
      if (L.shell)
        hipLaunchKernelGGL((prolong_kernel<T, false, true>), grid, dim3(kAmrBlock), 0, st, a);
      else
        hipLaunchKernelGGL((prolong_kernel<T, false, false>), grid, dim3(kAmrBlock), 0, st, a);
    }
  } else if (L.op == kAmrSnapshot) {
    hipLaunchKernelGGL(snapshot_kernel<T>, dim3(amr_blocks(L.cells), unsigned(L.nlinks)),
                       dim3(kAmrBlock), 0, st, a);
  } else if (L.op == kAmrFlux) {
    hipLaunchKernelGGL(flux_reg_kernel<T>, dim3(amr_blocks(L.cells), unsigned(L.nlinks), 2u),
                       dim3(kAmrBlock), 0, st, a);
  } else {
    hipLaunchKernelGGL(reflux_kernel<T>, dim3(amr_blocks(L.cells), unsigned(L.nlinks)),
                       dim3(kAmrBlock), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_amr(const LaunchAmr& L, hipStream_t st) {
  if (L.op < kAmrFill || L.op > kAmrSnapshot) return hipErrorInvalidValue;
  if (L.op == kAmrSnapshot && (!L.cold || L.margin < 0)) return hipErrorInvalidValue;
  if (L.op != kAmrFill &&
      (!L.patches || L.nlinks < 1 || (!L.dlinks && L.nlinks > kAmrLinksPerLaunch) ||
       L.nlinks > 65535))
    return hipErrorInvalidValue;
  if ((L.op == kAmrFlux || L.op == kAmrReflux) &&
      (!L.reg || L.maxface < 1 || L.axis < 0 || L.axis > 2 || L.side < 0 || L.side > 1))
    return hipErrorInvalidValue;
  return L.fp64 ? launch_amr_t<double>(L, st) : launch_amr_t<float>(L, st);
}

}  // namespace hydro
