// diag.hip -- in-situ diagnostics on the GPU: PDFs (histograms) of cell
// quantities and slab profiles with mixing measures.
//
// Large runs need their analysis done where the data is (the paper's
// discussion of the capabilities needed at the exascale); it fixes no
// diagnostic, so these are standard ones of stratified and shear-layer
// flows.  Each is one HBM-bound pass over the interior cells.
//
// Cell quantities are evaluated in FP64 with IEEE operations (no contraction:
// the library is built with -ffp-contract=off; FP64 division and square
// root are correctly rounded), in a fixed order:
//   m2 = mx mx + my my + mz mz,  ke = (0.5 m2) / rho,  p = (gamma-1)(E - ke),
//   speed = sqrt(m2) / rho,      mach = speed / sqrt((gamma p) / rho).
// An FP32 state is widened first (exact), so a quantity's bin is a pure
// function of the stored bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft.hpp"
#include "launch.hpp"

namespace hydro {

constexpr int kDiagBlock = 256;
constexpr int kDiagCells = 4;   // cells per thread in flight (loads before arithmetic)

template <class T, int Q>
__device__ __forceinline__ double diag_quantity(const T* p0, int64_t plane, int64_t o,
                                                double gamma) {
  const double r = double(p0[o]);
  if constexpr (Q == kQRho) {
    return r;
  } else {
    const double mx = double(p0[o + plane]), my = double(p0[o + 2 * plane]);
    const double mz = double(p0[o + 3 * plane]);
    const double m2 = mx * mx + my * my + mz * mz;
    if constexpr (Q == kQSpeed) {
      return __builtin_sqrt(m2) / r;
    } else {
      const double e = double(p0[o + 4 * plane]);
      const double p = (gamma - 1.0) * (e - (0.5 * m2) / r);
      if constexpr (Q == kQPressure) return p;
      // |v| / c = sqrt(|m|^2 / (gamma p rho)): one division and one root
      return __builtin_sqrt(m2 / ((gamma * p) * r));
    }
  }
}

// Bin of value v: 0 below lo (or NaN), 1 + floor((v - lo) w) inside,
// nbins + 1 at or above hi.
__device__ __forceinline__ int diag_bin(double v, double lo, double w, int nbins) {
  if (!(v >= lo)) return 0;
  const double t = (v - lo) * w;
  return t < double(nbins) ? 1 + int(t) : nbins + 1;
}

// Adds one to counter b (b < 0: nothing) for every lane of the wave.  Lanes
// that share the bin of the first lane still pending add together with one
// atomic, twice over (a flow with few distinct values, like a two-density
// layer, puts most of a wave in one or two bins); the lanes left add one
// by one.  Integer adds commute, so the counts do not depend on the grouping.
template <class C>
__device__ __forceinline__ void count_bin(C* ctr, int b) {
  bool todo = b >= 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const unsigned long long m = __ballot(todo);
    if (m == 0ull) return;  // wave-uniform
    const int lead = __shfl(b, int(__builtin_ctzll(m)));
    const bool mine = todo && b == lead;
    const unsigned long long same = __ballot(mine);
    if (mine) {
      if ((threadIdx.x & 63) == unsigned(__builtin_ctzll(same)))
        atomicAdd(&ctr[lead], C(__builtin_popcountll(same)));
      todo = false;
    }
  }
  if (todo) atomicAdd(&ctr[b], C(1));
}

__global__ void __launch_bounds__(kDiagBlock) zero_u64_kernel(unsigned long long* p, int n) {
  for (int i = blockIdx.x * kDiagBlock + threadIdx.x; i < n; i += gridDim.x * kDiagBlock)
    p[i] = 0ull;
}

template <class T>
struct DiagArgs {
  const T* pool;
  const PatchDev* patches;  // null: single grid
  PatchDev single;
  double gamma;
  int nbins;
  double lo, w;
  unsigned long long* counts;
  bool lds;                 // per-workgroup LDS counters (nbins + 2 <= kPdfLdsBins)
  int axis, chunks;
  FastDiv dnx, dny;         // single grid: division by nx and ny
  double rho_lo, drho, dx_axis;
  double* partials;
  double* out;
};

// Histogram of quantity Q over the interior cells of one grid (y = 0) or of
// patch blockIdx.y: workgroups stride over the flattened cells (x fastest,
// coalesced), count into LDS, then add their nonzero counters to the global
// 64-bit counters (exact: integer adds commute).
template <class T, int Q>
__global__ void __launch_bounds__(kDiagBlock) pdf_kernel(DiagArgs<T> a) {
  extern __shared__ unsigned int hist[];
  const bool batch = a.patches != nullptr;
  const PatchDev P = batch ? a.patches[blockIdx.y] : a.single;
  const int nb2 = a.nbins + 2;
  if (a.lds) {
    for (int i = threadIdx.x; i < nb2; i += kDiagBlock) hist[i] = 0u;
    __syncthreads();
  }
  const unsigned nx = unsigned(P.n[0]), ny = unsigned(P.n[1]);
  const unsigned cells = nx * ny * unsigned(P.n[2]);
  const FastDiv dnx = batch ? FastDiv(nx) : a.dnx, dny = batch ? FastDiv(ny) : a.dny;
  const T* p0 = a.pool + P.base0;
  constexpr int U = kDiagCells;
  const unsigned stride = gridDim.x * kDiagBlock * U;
  for (unsigned i0 = blockIdx.x * kDiagBlock * U + threadIdx.x; i0 < cells; i0 += stride) {
    // the U cells' offsets, then their quantities (all loads issued first)
    int64_t o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned i = min(i0 + unsigned(u) * kDiagBlock, cells - 1);
      const unsigned row = dnx.div(i), x = i - row * nx;
      const unsigned z = dny.div(row), y = row - z * ny;
      o[u] = int64_t(x) + int64_t(y) * P.sy + int64_t(z) * P.sz;
    }
    double q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = diag_quantity<T, Q>(p0, P.plane, o[u], a.gamma);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool valid = i0 + unsigned(u) * kDiagBlock < cells;
      const int b = valid ? diag_bin(q[u], a.lo, a.w, a.nbins) : -1;
      if (a.lds)
        count_bin(hist, b);
      else
        count_bin(a.counts, b);
    }
  }
  if (a.lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < nb2; i += kDiagBlock)
      if (hist[i]) atomicAdd(&a.counts[i], (unsigned long long)hist[i]);
  }
}

// The five conserved values of one cell, widened to FP64.
template <class T>
__device__ __forceinline__ void load_cell(const T* p0, int64_t plane, int64_t o, double (&c)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) c[v] = double(p0[o + v * plane]);
}

// Adds the five profile fields of one cell: rho, p, ke, f, f (1 - f).
template <class T>
__device__ __forceinline__ void profile_add(const double (&c)[5], const DiagArgs<T>& a,
                                            double (&acc)[5]) {
  const double r = c[0];
  const double m2 = c[1] * c[1] + c[2] * c[2] + c[3] * c[3];
  const double ke = (0.5 * m2) / r;
  const double p = (a.gamma - 1.0) * (c[4] - ke);
  const double f = __builtin_fmin(__builtin_fmax((r - a.rho_lo) / a.drho, 0.0), 1.0);
  acc[0] += r;
  acc[1] += p;
  acc[2] += ke;
  acc[3] += f;
  acc[4] += f * (1.0 - f);
}

// Slabs normal to y (axis 1) or z (axis 2): workgroup (c, s) sums the cells
// j = c 256 U + t + u 256 (u < U), then the same plus C 256 U, ... of slab s
// (x fastest), then reduces its threads in a fixed order into
// partials[s][c][5].
template <class T>
__global__ void __launch_bounds__(kDiagBlock) profile_slab_kernel(DiagArgs<T> a) {
  __shared__ double red[kDiagBlock / 64][5];
  const PatchDev& P = a.single;
  const int s = blockIdx.y, c = blockIdx.x;
  const unsigned nx = unsigned(P.n[0]);
  const unsigned rows = unsigned(a.axis == 2 ? P.n[1] : P.n[2]);
  const unsigned cells = nx * rows;
  const T* p0 = a.pool + P.base0;
  const int64_t srow = a.axis == 2 ? P.sy : P.sz;          // stride between the slab's rows
  const int64_t sbase = int64_t(s) * (a.axis == 2 ? P.sz : P.sy);
  constexpr int U = kDiagCells;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (unsigned j0 = unsigned(c) * kDiagBlock * U + threadIdx.x; j0 < cells;
       j0 += unsigned(a.chunks) * kDiagBlock * U) {
    double cv[U][5];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned j = min(j0 + unsigned(u) * kDiagBlock, cells - 1);
      const unsigned r = a.dnx.div(j), x = j - r * nx;
      load_cell<T>(p0, P.plane, sbase + int64_t(x) + int64_t(r) * srow, cv[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j0 + unsigned(u) * kDiagBlock < cells) profile_add<T>(cv[u], a, acc);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v)
    for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int v = 0; v < 5; ++v) red[wave][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = red[0][threadIdx.x];
    for (int w = 1; w < kDiagBlock / 64; ++w) t += red[w][threadIdx.x];
    a.partials[(int64_t(s) * a.chunks + c) * 5 + threadIdx.x] = t;
  }
}

// Slabs normal to x (axis 0): thread x of workgroup (c, xb) sums rows
// c, c + C, ... (U of them in flight) of the grid at its own x into
// partials[x][c][5].
template <class T>
__global__ void __launch_bounds__(kDiagBlock) profile_xslab_kernel(DiagArgs<T> a) {
  const PatchDev& P = a.single;
  const int c = blockIdx.x;
  const int x = blockIdx.y * kDiagBlock + threadIdx.x;
  if (x >= P.n[0]) return;
  const unsigned ny = unsigned(P.n[1]), rows = ny * unsigned(P.n[2]);
  const T* p0 = a.pool + P.base0;
  constexpr int U = kDiagCells;
  const unsigned C = unsigned(a.chunks);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (unsigned r0 = unsigned(c); r0 < rows; r0 += C * U) {
    double cv[U][5];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned r = min(r0 + unsigned(u) * C, rows - 1);
      const unsigned z = a.dny.div(r), y = r - z * ny;
      load_cell<T>(p0, P.plane, int64_t(x) + int64_t(y) * P.sy + int64_t(z) * P.sz, cv[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (r0 + unsigned(u) * C < rows) profile_add<T>(cv[u], a, acc);
  }
  for (int v = 0; v < 5; ++v) a.partials[(int64_t(x) * a.chunks + c) * 5 + v] = acc[v];
}

// Sum of v over the workgroup in a fixed order (wave shuffles, then the
// waves in order); the result is returned to every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();  // red is free
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < kDiagBlock / 64; ++w) t += red[w];
  return t;
}

// Slab means out[s][v] = sum_c partials[s][c][v] / cells per slab (thread t
// takes slabs t, t + 256, ...), then the mixing width and mixedness from
// per-thread sums reduced in a fixed order (one workgroup).
__global__ void __launch_bounds__(kDiagBlock) profile_final_kernel(const double* partials,
                                                                     int nslab, int chunks,
                                                                     double cells_per_slab,
                                                                     double dx_axis, double* out) {
  __shared__ double red[kDiagBlock / 64];
  double w = 0.0, num = 0.0, den = 0.0;
  for (int s = threadIdx.x; s < nslab; s += kDiagBlock) {
    double m[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double t = 0.0;
      for (int c = 0; c < chunks; ++c) t += partials[(int64_t(s) * chunks + c) * 5 + v];
      m[v] = t / cells_per_slab;
      out[s * 5 + v] = m[v];
    }
    w += 4.0 * m[3] * (1.0 - m[3]);
    den += m[3] * (1.0 - m[3]);
    num += m[4];
  }
  w = block_sum(w, red);
  den = block_sum(den, red);
  num = block_sum(num, red);
  if (threadIdx.x == 0) {
    out[nslab * 5] = w * dx_axis;
    out[nslab * 5 + 1] = den > 0.0 ? num / den : 0.0;
  }
}

// --------------------------------------------------------------------------
// One-dimensional kinetic-energy spectrum along x
// --------------------------------------------------------------------------
//
// A workgroup owns groups of P (even) whole x-lines (y, z): groups
// blockIdx.x, blockIdx.x + gridDim.x, ...  For each line it widens rho and m
// to FP64 and forms u = m / rho (IEEE division); it packs the complex lines
// ux + i uy of every x-line and uz + i uz' of every pair of x-lines (3P/2
// lines, no line of zeros), and transforms them in LDS with the in-place
// mixed-radix Stockham FFT of fft.hpp (radices 16, 4, 2, 3; output in
// natural order).  For a real pair packed as a + i b,
// |A(k)|^2 + |B(k)|^2 = (|Z(k)|^2 + |Z(N-k)|^2) / 2, so the power summed over
// the components and lines needs no unpacking.  Thread t accumulates k = t,
// t + 256, ... over its workgroup's lines (fixed order), writes its
// partial spectrum, and one workgroup sums the partials in a fixed order.

// x-lines per pass: the 3/2 complex lines of every x-line of a pass fill at
// most kSpecElems complex values of LDS
constexpr int kSpecElems = 4096;
constexpr int kSpecBlock = 512;  // threads of the spectrum kernel

template <class T, int P>
// Short lines (P >= 4) keep their registers (two waves per SIMD); long
// lines (P = 2) take four waves per SIMD, which measured faster (768^3:
// 5.5 against 6.7 ms) despite a few spilled registers.
__global__ void __launch_bounds__(kSpecBlock, P >= 4 ? 2 : 4) spectrum_kernel(DiagArgs<T> a, FftPlan sp) {
  extern __shared__ double2 sbuf[];
  const PatchDev& Pd = a.single;
  const int n = sp.n;
  double2* W = sbuf;       // W[t] = exp(-2 pi i t / n)
  double2* buf = sbuf + n;  // 3P/2 complex lines (fft_pad slots), transformed in place
  static_assert(P % 2 == 0, "x-lines are paired for their uz lines");
  for (int t = threadIdx.x; t < n; t += kSpecBlock) {
    double sn, cs;
    sincospi(-2.0 * double(t) / double(n), &sn, &cs);
    W[t] = make_double2(cs, sn);
  }
  constexpr int KPT = (kSpecMaxLen / 2 + 1 + kSpecBlock - 1) / kSpecBlock;  // k per thread
  double acc[KPT];
#pragma unroll
  for (int i = 0; i < KPT; ++i) acc[i] = 0.0;
  const int ny = Pd.n[1], lines = Pd.n[1] * Pd.n[2];
  const int groups = (lines + P - 1) / P;
  const T* p0 = a.pool + Pd.base0;
  // this thread's cells c = t + 256 i of the pass (line c / n of the group,
  // x = c mod n), fetched one pass ahead so that the next pass's loads are
  // in flight during the current transform
  constexpr int XPT = kSpecElems / 2 / kSpecBlock;
  T fr[XPT], fm[XPT][3];
  auto fetch = [&](int grp) {
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int c = threadIdx.x + i * kSpecBlock;
      const int lp = c / n;
      const int x = c - lp * n, line = grp * P + lp;
      if (lp < P && line < lines) {
        const int z = line / ny, y = line - z * ny;
        const int64_t o = int64_t(y) * Pd.sy + int64_t(z) * Pd.sz + x;
        fr[i] = p0[o];
#pragma unroll
        for (int v = 0; v < 3; ++v) fm[i][v] = p0[o + (v + 1) * Pd.plane];
      }
    }
  };
  if (int(blockIdx.x) < groups) fetch(blockIdx.x);
  for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    __syncthreads();  // the previous pass's buffer and the twiddles
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int c = threadIdx.x + i * kSpecBlock;
      const int lp = c / n;
      const int x = c - lp * n;
      if (lp < P) {
        double2 z1 = make_double2(0.0, 0.0);  // a missing last line: zeros
        double uz = 0.0;
        if (grp * P + lp < lines) {
          const double r = double(fr[i]);
          z1 = make_double2(double(fm[i][0]) / r, double(fm[i][1]) / r);
          uz = double(fm[i][2]) / r;
        }
        buf[fft_pad(lp * n + x)] = z1;
        // the real (even lp) or imaginary (odd lp) part of the pair's uz line
        double* zp = reinterpret_cast<double*>(&buf[fft_pad((P + (lp >> 1)) * n + x)]);
        zp[lp & 1] = uz;
      }
    }
    if (grp + int(gridDim.x) < groups) fetch(grp + gridDim.x);
    __syncthreads();
    fft_lines_inplace<kSpecElems, kSpecBlock>(buf, 3 * P / 2, n, sp, W);
    // the lines of the pass that hold data: its x-lines, then the uz line of
    // every pair with at least one x-line (a missing x-line left zeros)
    const int have = min(P, lines - grp * P);
    const int nz = (have + 1) >> 1;
#pragma unroll
    for (int q = 0; q < P + P / 2; ++q) {
      if (q < P ? q >= have : q - P >= nz) continue;
      const int z = q * n;
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int k = threadIdx.x + i * kSpecBlock;
        if (k <= n / 2) {
          const int km = k == 0 ? 0 : n - k;
          const double2 a1 = buf[fft_pad(z + k)], b1 = buf[fft_pad(z + km)];
          acc[i] += 0.5 * ((a1.x * a1.x + a1.y * a1.y) + (b1.x * b1.x + b1.y * b1.y));
        }
      }
    }
  }
  const int nk = n / 2 + 1;
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int k = threadIdx.x + i * kSpecBlock;
    if (k < nk) a.partials[int64_t(blockIdx.x) * nk + k] = acc[i];
  }
}

// E[k] = sum over workgroups of the partials / (lines n^2), halved at k = 0
// and at the Nyquist wavenumber of an even n.  Workgroup k: thread t sums
// partials t, t + 256, ..., then a fixed-order workgroup sum.
__global__ void __launch_bounds__(kDiagBlock) spectrum_final_kernel(const double* partials,
                                                                      int blocks, int n,
                                                                      double lines, double* out) {
  __shared__ double red[kDiagBlock / 64];
  const int nk = n / 2 + 1, k = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kDiagBlock) t += partials[int64_t(b) * nk + k];
  t = block_sum(t, red);
  if (threadIdx.x == 0) {
    double e = t / lines / (double(n) * double(n));
    if (k == 0 || (2 * k == n)) e *= 0.5;
    out[k] = e;
  }
}

template <class T>
static DiagArgs<T> to_dargs(const LaunchDiag& L) {
  DiagArgs<T> a;
  a.pool = static_cast<const T*>(L.pool);
  a.patches = L.patches;
  a.single = L.single;
  a.gamma = L.gamma;
  a.nbins = L.nbins;
  a.lo = L.lo;
  a.w = L.w;
  a.counts = L.counts;
  a.lds = L.nbins + 2 <= kPdfLdsBins;
  a.axis = L.axis;
  a.chunks = L.chunks;
  a.dnx = FastDiv(uint32_t(L.single.n[0]));
  a.dny = FastDiv(uint32_t(L.single.n[1]));
  a.rho_lo = L.rho_lo;
  a.drho = L.drho;
  a.dx_axis = L.dx_axis;
  a.partials = L.partials;
  a.out = L.out;
  return a;
}

template <class T>
static hipError_t launch_pdf_t(const LaunchDiag& L, hipStream_t st) {
  const DiagArgs<T> a = to_dargs<T>(L);
  const int nb2 = L.nbins + 2;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(unsigned(std::min(1024, (nb2 + kDiagBlock - 1) / kDiagBlock))),
                     dim3(kDiagBlock), 0, st, L.counts, nb2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = a.lds ? size_t(nb2) * sizeof(unsigned int) : 0;
  dim3 grid;
  if (L.patches) {
    grid = dim3(kPdfPatchBlocks, unsigned(L.npatch));
  } else {
    const int64_t cells = int64_t(L.single.n[0]) * L.single.n[1] * L.single.n[2];
    const int64_t b = (cells + 4 * kDiagBlock - 1) / (4 * kDiagBlock);
    grid = dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>(b, kPdfMaxBlocks))));
  }
  switch (L.quantity) {
    case kQRho: hipLaunchKernelGGL((pdf_kernel<T, kQRho>), grid, dim3(kDiagBlock), lds, st, a); break;
    case kQPressure: hipLaunchKernelGGL((pdf_kernel<T, kQPressure>), grid, dim3(kDiagBlock), lds, st, a); break;
    case kQSpeed: hipLaunchKernelGGL((pdf_kernel<T, kQSpeed>), grid, dim3(kDiagBlock), lds, st, a); break;
    case kQMach: hipLaunchKernelGGL((pdf_kernel<T, kQMach>), grid, dim3(kDiagBlock), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_diag_pdf(const LaunchDiag& L, hipStream_t st) {
  if (L.nbins < 1 || L.nbins > kPdfMaxBins) return hipErrorInvalidValue;
  return L.fp64 ? launch_pdf_t<double>(L, st) : launch_pdf_t<float>(L, st);
}

template <class T>
static hipError_t launch_profile_t(const LaunchDiag& L, hipStream_t st) {
  const DiagArgs<T> a = to_dargs<T>(L);
  const int ns = L.single.n[L.axis];
  if (L.axis == 0)
    hipLaunchKernelGGL(profile_xslab_kernel<T>,
                       dim3(unsigned(L.chunks), unsigned((ns + kDiagBlock - 1) / kDiagBlock)),
                       dim3(kDiagBlock), 0, st, a);
  else
    hipLaunchKernelGGL(profile_slab_kernel<T>, dim3(unsigned(L.chunks), unsigned(ns)),
                       dim3(kDiagBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double cells = double(L.single.n[0]) * L.single.n[1] * L.single.n[2];
  hipLaunchKernelGGL(profile_final_kernel, dim3(1), dim3(kDiagBlock), 0, st, L.partials, ns,
                     L.chunks, cells / ns, L.dx_axis, L.out);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_spectrum_t(const LaunchDiag& L, hipStream_t st) {
  const DiagArgs<T> a = to_dargs<T>(L);
  FftPlan sp;
  if (!make_fft_plan(L.single.n[0], sp)) return hipErrorInvalidValue;
  // x-lines per pass: 8 (an FP64 state: 4, for its prefetch registers) for
  // lines of up to 256 cells, else 2 (3P/2 n <= kSpecElems)
  constexpr int PS = sizeof(T) == 8 ? 4 : 8;
  if (sp.n <= 256) {
    const size_t lds = size_t(sp.n + fft_lds(3 * PS / 2 * sp.n)) * sizeof(double2);
    hipLaunchKernelGGL((spectrum_kernel<T, PS>), dim3(unsigned(L.chunks)), dim3(kSpecBlock), lds,
                       st, a, sp);
  } else {
    const size_t lds = size_t(sp.n + fft_lds(3 * sp.n)) * sizeof(double2);
    hipLaunchKernelGGL((spectrum_kernel<T, 2>), dim3(unsigned(L.chunks)), dim3(kSpecBlock), lds,
                       st, a, sp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double lines = double(L.single.n[1]) * L.single.n[2];
  hipLaunchKernelGGL(spectrum_final_kernel, dim3(unsigned(sp.n / 2 + 1)), dim3(kDiagBlock), 0,
                     st, L.partials, L.chunks, sp.n, lines, L.out);
  return hipGetLastError();
}

hipError_t launch_diag_spectrum(const LaunchDiag& L, hipStream_t st) {
  const int n = L.single.n[0];
  if (L.patches || n < 2 || n > kSpecMaxLen || L.chunks < 1) return hipErrorInvalidValue;
  return L.fp64 ? launch_spectrum_t<double>(L, st) : launch_spectrum_t<float>(L, st);
}

hipError_t launch_diag_profile(const LaunchDiag& L, hipStream_t st) {
  if (L.axis < 0 || L.axis > 2 || L.chunks < 1 || L.patches) return hipErrorInvalidValue;
  return L.fp64 ? launch_profile_t<double>(L, st) : launch_profile_t<float>(L, st);
}

}  // namespace hydro
