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
//     coarse neighbours along each axis.
#include <hip/hip_runtime.h>

#include <algorithm>

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
};

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
  const AmrLink L = a.links[blockIdx.y];
  const PatchDev F = a.patches[L.fine], C = a.patches[L.coarse];
  const unsigned cx = unsigned(F.n[0] / 2), cxy = cx * unsigned(F.n[1] / 2);
  const unsigned total = cxy * unsigned(F.n[2] / 2);
  const T* f0 = a.pool + F.base0;
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

// Monotonised-central slope from one-sided differences a and b.
__device__ __forceinline__ double mc_slope(double a, double b) {
  const double m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
  return a * b > 0.0 ? copysign(m, a) : 0.0;
}

// Fine cells (interior, or the stored ghost shell) of link blockIdx.y.
template <class T>
__global__ void __launch_bounds__(kAmrBlock) prolong_kernel(AmrArgs<T> a) {
  const AmrLink L = a.links[blockIdx.y];
  const PatchDev F = a.patches[L.fine], C = a.patches[L.coarse];
  const int nx = F.n[0], ny = F.n[1], nz = F.n[2];
  const int g = a.ghosts_only ? F.ng : 0;
  const unsigned sx = unsigned(nx + 2 * g), sxy = sx * unsigned(ny + 2 * g);
  const unsigned total = sxy * unsigned(nz + 2 * g);
  T* f0 = a.pool + F.base0;
  const T* c0 = a.pool + C.base0;
  if (blockIdx.x * kAmrBlock >= total) return;
  for (unsigned c = blockIdx.x * kAmrBlock + threadIdx.x; c < total;
       c += gridDim.x * kAmrBlock) {
    const unsigned kk = c / sxy, rem = c - kk * sxy;
    const unsigned jj = rem / sx;
    const int k = int(kk) - g, j = int(jj) - g, i = int(rem - jj * sx) - g;
    const bool inside = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
    if (a.ghosts_only && inside) continue;
    const int64_t pc = int64_t(L.ox + (i >> 1)) + int64_t(L.oy + (j >> 1)) * C.sy +
                       int64_t(L.oz + (k >> 1)) * C.sz;
    const double ox = (i & 1) ? 0.25 : -0.25, oy = (j & 1) ? 0.25 : -0.25,
                 oz = (k & 1) ? 0.25 : -0.25;
    const int64_t dst = int64_t(i) + int64_t(j) * F.sy + int64_t(k) * F.sz;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T* q = c0 + pc + v * C.plane;
      const double u = double(q[0]);
      const double dx = mc_slope(u - double(q[-1]), double(q[1]) - u);
      const double dy = mc_slope(u - double(q[-C.sy]), double(q[C.sy]) - u);
      const double dz = mc_slope(u - double(q[-C.sz]), double(q[C.sz]) - u);
      f0[dst + v * F.plane] = T(((u + ox * dx) + oy * dy) + oz * dz);
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
  for (int i = 0; i < L.nlinks; ++i) a.links[i] = L.links[i];
  a.ghosts_only = L.ghosts_only;
  return a;
}

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
  } else {
    hipLaunchKernelGGL(prolong_kernel<T>, dim3(amr_blocks(L.cells), unsigned(L.nlinks)),
                       dim3(kAmrBlock), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_amr(const LaunchAmr& L, hipStream_t st) {
  if (L.op != kAmrFill && (!L.patches || L.nlinks < 1 || L.nlinks > kAmrLinksPerLaunch))
    return hipErrorInvalidValue;
  return L.fp64 ? launch_amr_t<double>(L, st) : launch_amr_t<float>(L, st);
}

}  // namespace hydro
