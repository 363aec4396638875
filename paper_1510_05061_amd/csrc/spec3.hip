// spec3.hip -- shell kinetic-energy spectrum of a single grid.
//
// In-situ analysis is one of the capabilities the paper asks of exascale
// codes (its discussion of the capabilities needed); for turbulence the
// standard reduction is the kinetic-energy spectrum summed over shells of
// integer wavevectors, K = round(|k|):
//   E[K] = sum_{round(|k|) = K} sum_c |u_hat_c(k)|^2 / (2 N^2),  u = m / rho,
// with u_hat the unnormalised three-dimensional DFT over the grid (N cells),
// so that sum_K E[K] = <|u|^2> / 2.
//
// Four passes over HBM, all in FP64 (an FP32 state is widened first):
//   x  each x-line: u = m / rho; ux + i uy of every x-line and uz + i uz' of
//      every pair of x-lines as complex lines (3/2 complex FFTs per x-line)
//      in LDS, unpacked into the three half spectra kx = 0 .. nx/2 (real
//      input: the other half is their conjugate); written as three planes
//      U_c[z][y][kx] of complex values.
//   y  tiles of 4 neighbouring kx columns of one (c, z): FFT along y in LDS,
//      written back in place.
//   z  tiles of 4 kx columns of one ky: FFT along z of each component in
//      turn, the power summed over the components in registers, then
//      P[ky][kz][kx] = w(kx) sum_c |U_c|^2 with w = 2 for the kx whose
//      conjugate partner -kx is not stored (0 < kx < nx/2), else 1.
//   bin  rows (ky, kz) of P: along a row the shell grows with kx, so the
//      lanes of a wave holding 64 consecutive kx form runs of equal shell; a
//      segmented scan sums each run in lane order and the run's last lane
//      adds it to its wave's shell bins in LDS.  The bins of the waves, then
//      of the workgroups, are summed in a fixed order: the spectrum is
//      bitwise reproducible for a grid shape and launch size.
// Every FFT is the in-place Stockham FFT of fft.hpp, with twiddle tables
// exp(-2 pi i t / n) computed once per call into the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "fft.hpp"
#include "launch.hpp"

namespace hydro {

constexpr int kS3Block = 256;
constexpr int kS3Elems = 4096;  // complex elements of the x pass's lines in LDS
constexpr int kS3T = 4;         // kx columns per tile of the y and z passes
constexpr int kS3MaxLen = 1024;
constexpr int kS3ColElems = kS3T * kS3MaxLen;

struct Spec3Args {
  const void* pool;
  int64_t base0, plane;  // state: interior cell (0,0,0) of plane 0, elements per plane
  int32_t sy, sz;        // state strides along y and z
  int32_t n[3];          // nx, ny, nz
  int32_t nh;            // nx / 2 + 1
  int32_t ntk;           // tiles along kx: ceil(nh / kS3T)
  int32_t gx;            // x-lines per pass of the x kernel
  int32_t nb;            // shells
  int64_t cplane;        // complex values per component plane: nz ny nh
  double2* U;            // 3 component planes [z][y][kx]
  double* P;             // power [ky][kz][kx]
  double* partials;      // [bin workgroup][shell]
  const double2* tw;     // twiddles: nx, then ny, then nz values
  FastDiv dnx, dny, dnz, dnh;
};

__global__ void spec3_twiddle_kernel(double2* tw, int nx, int ny, int nz) {
  const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= nx + ny + nz) return;
  const int n = t < nx ? nx : (t < nx + ny ? ny : nz);
  const int i = t < nx ? t : (t < nx + ny ? t - nx : t - nx - ny);
  double sn, cs;
  sincospi(-2.0 * double(i) / double(n), &sn, &cs);
  tw[t] = make_double2(cs, sn);
}

// Tile b of nt, remapped so that the consecutive tiles, which share cache
// lines, run on one XCD: dispatch sends workgroup b to XCD b mod 8, so XCD x
// takes the contiguous range of tiles x q + min(x, r) .. (nt = 8 q + r).
__device__ __forceinline__ int xcd_tile(int b, int nt) {
  const int q = nt >> 3, r = nt & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

template <class T>
__global__ void __launch_bounds__(kS3Block) spec3_x_kernel(Spec3Args a, FftPlan px) {
  extern __shared__ double2 s3lds[];
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2], nh = a.nh, G = a.gx;
  double2* W = s3lds;
  double2* buf = s3lds + nx;
  for (int t = threadIdx.x; t < nx; t += kS3Block) W[t] = a.tw[t];
  const int lines = ny * nz, groups = (lines + G - 1) / G;
  const T* p0 = static_cast<const T*>(a.pool) + a.base0;
  constexpr int EPT = kS3Elems / 2 / kS3Block;  // x cells per thread and pass
  for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    __syncthreads();  // the twiddles, and the previous pass's reads of buf
    T r[EPT], m[EPT][3];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {  // every load before any arithmetic
      const int e = threadIdx.x + i * kS3Block;
      const int lp = int(a.dnx.div(uint32_t(e))), x = e - lp * nx, line = grp * G + lp;
      if (lp < G && line < lines) {
        const int z = int(a.dny.div(uint32_t(line))), y = line - z * ny;
        const int64_t o = int64_t(y) * a.sy + int64_t(z) * a.sz + x;
        r[i] = p0[o];
#pragma unroll
        for (int v = 0; v < 3; ++v) m[i][v] = p0[o + (v + 1) * a.plane];
      }
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kS3Block;
      const int lp = int(a.dnx.div(uint32_t(e))), x = e - lp * nx, line = grp * G + lp;
      if (lp < G) {
        double2 z1 = make_double2(0.0, 0.0);  // lines past the end: zeros
        double uz = 0.0;
        if (line < lines) {
          const double rho = double(r[i]);
          z1 = make_double2(double(m[i][0]) / rho, double(m[i][1]) / rho);
          uz = double(m[i][2]) / rho;
        }
        buf[fft_pad(lp * nx + x)] = z1;
        // uz of x-lines 2q and 2q + 1 as the real and imaginary parts of
        // line G + q (the odd last x-line of a pass with zeros beside it)
        double* zp = reinterpret_cast<double*>(&buf[fft_pad((G + (lp >> 1)) * nx + x)]);
        zp[lp & 1] = uz;
        if ((G & 1) && lp == G - 1) zp[1] = 0.0;
      }
    }
    __syncthreads();
    fft_lines_inplace<kS3Elems, kS3Block>(buf, G + (G + 1) / 2, nx, px, W);
    // Z = X + i Y with X, Y the DFTs of two real lines (ux and uy of an
    // x-line, or uz of two x-lines):
    // X(k) = (Z(k) + conj Z(n-k)) / 2, Y(k) = -i (Z(k) - conj Z(n-k)) / 2
    for (int e = threadIdx.x; e < G * nh; e += kS3Block) {
      const int lp = int(a.dnh.div(uint32_t(e))), k = e - lp * nh, line = grp * G + lp;
      if (line >= lines) continue;
      const int z = int(a.dny.div(uint32_t(line))), y = line - z * ny;
      const int km = k == 0 ? 0 : nx - k;
      const double2 zk = buf[fft_pad(lp * nx + k)];
      const double2 zm = conj2(buf[fft_pad(lp * nx + km)]);
      const double2 s = cadd(zk, zm), d = cmi(csub(zk, zm));
      const int64_t o = (int64_t(z) * ny + y) * nh + k;
      a.U[o] = make_double2(0.5 * s.x, 0.5 * s.y);
      a.U[o + a.cplane] = make_double2(0.5 * d.x, 0.5 * d.y);
      const int q = (G + (lp >> 1)) * nx;
      const double2 wk = buf[fft_pad(q + k)], wm = conj2(buf[fft_pad(q + km)]);
      const double2 w = (lp & 1) ? cmi(csub(wk, wm)) : cadd(wk, wm);
      a.U[o + 2 * a.cplane] = make_double2(0.5 * w.x, 0.5 * w.y);
    }
  }
}

// FFT along y (ZP false: tile = (c, z, kx tile), in place) or z (ZP true:
// tile = (ky, kx tile), the three components in turn, power out).
template <bool ZP>
__global__ void __launch_bounds__(kS3Block) spec3_col_kernel(Spec3Args a, FftPlan pl) {
  extern __shared__ double2 s3lds[];
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2], nh = a.nh, L = pl.n, ls = L + 1;
  double2* W = s3lds;
  double2* buf = s3lds + L;
  const double2* tw = a.tw + (ZP ? nx + ny : nx);
  for (int t = threadIdx.x; t < L; t += kS3Block) W[t] = tw[t];
  const int nt = (ZP ? ny : 3 * nz) * a.ntk;
  const int tile = xcd_tile(int(blockIdx.x), nt);
  const int o = tile / a.ntk, kx0 = (tile - o * a.ntk) * kS3T;
  // line element j of column t at col[j S + t]
  const int64_t S = ZP ? int64_t(ny) * nh : int64_t(nh);
  constexpr int EPT = kS3ColElems / kS3Block;
  double pw[ZP ? EPT : 1];
#pragma unroll
  for (int i = 0; i < (ZP ? EPT : 1); ++i) pw[i] = 0.0;
  for (int c = 0; c < (ZP ? 3 : 1); ++c) {
    double2* col = ZP ? a.U + c * a.cplane + int64_t(o) * nh + kx0
                      : a.U + int64_t(o) * ny * nh + kx0;
    __syncthreads();  // the twiddles, and the previous component's reads of buf
    double2 v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kS3Block, t = e & (kS3T - 1), j = e / kS3T;
      v[i] = make_double2(0.0, 0.0);
      if (j < L && kx0 + t < nh) v[i] = col[j * S + t];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kS3Block, t = e & (kS3T - 1), j = e / kS3T;
      if (j < L) buf[fft_pad(t * ls + j)] = v[i];
    }
    __syncthreads();
    fft_lines_inplace<kS3ColElems, kS3Block>(buf, kS3T, ls, pl, W);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kS3Block, t = e & (kS3T - 1), j = e / kS3T;
      if (j < L && kx0 + t < nh) {
        const double2 u = buf[fft_pad(t * ls + j)];
        if (ZP)
          pw[i] += u.x * u.x + u.y * u.y;
        else
          col[j * S + t] = u;
      }
    }
  }
  if (ZP) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * kS3Block, t = e & (kS3T - 1), j = e / kS3T;
      const int kx = kx0 + t;
      if (j < L && kx < nh) {
        const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        a.P[(int64_t(o) * nz + j) * nh + kx] = w * pw[i];
      }
    }
  }
}

// Shell of the integer wavevector with |k|^2 = m2: round(sqrt(m2)), taken
// exactly (sqrt of an integer is never a half-integer): K = floor(sqrt(m2)),
// plus one when K + 1/2 <= sqrt(m2), i.e. K^2 + K < m2.
__device__ __forceinline__ int shell_of(int m2) {
  int K = int(__builtin_sqrt(double(m2)));
  if (K * K + K < m2) ++K;
  return K;
}

__global__ void __launch_bounds__(kS3Block) spec3_bin_kernel(Spec3Args a) {
  extern __shared__ double s3bins[];  // one row of a.nb shells per wave
  const int nb = a.nb, ny = a.n[1], nz = a.n[2], nh = a.nh;
  constexpr int NW = kS3Block / 64;
  for (int i = threadIdx.x; i < NW * nb; i += kS3Block) s3bins[i] = 0.0;
  __syncthreads();
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* bins = s3bins + wid * nb;
  const int64_t rows = int64_t(ny) * nz;
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  for (int64_t r = r0 + wid; r < r1; r += NW) {
    const int ky = int(a.dnz.div(uint32_t(r))), kz = int(r) - ky * nz;
    const int sy = 2 * ky <= ny ? ky : ky - ny, sz = 2 * kz <= nz ? kz : kz - nz;
    const int myz = sy * sy + sz * sz;
    const double* row = a.P + r * nh;
    for (int c0 = 0; c0 < nh; c0 += 64) {
      const int kx = c0 + lane;
      const bool valid = kx < nh;
      double v = valid ? row[kx] : 0.0;
      const int K = valid ? shell_of(myz + kx * kx) : INT_MAX;
      // inclusive scan within runs of equal K (contiguous: K grows with kx)
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double up = __shfl_up(v, d);
        const int Ku = __shfl_up(K, d);
        if (lane >= d && Ku == K) v += up;
      }
      const int Kn = __shfl_down(K, 1);
      if (valid && (lane == 63 || Kn != K)) bins[K] += v;  // one lane per run: distinct K
    }
  }
  __syncthreads();
  for (int K = threadIdx.x; K < nb; K += kS3Block) {
    double s = s3bins[K];
    for (int w = 1; w < NW; ++w) s += s3bins[w * nb + K];
    a.partials[int64_t(blockIdx.x) * nb + K] = s;
  }
}

// out[K] = (sum over the bin workgroups, in order) / (2 N^2); workgroup K.
__global__ void __launch_bounds__(kS3Block) spec3_final_kernel(const double* partials, int nwg,
                                                                 int nb, double norm, double* out) {
  __shared__ double red[kS3Block];
  const int K = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nwg; b += kS3Block) t += partials[int64_t(b) * nb + K];
  red[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kS3Block; ++i) s += red[i];
    out[K] = s / norm;
  }
}

// Regions of the workspace, each 256-byte aligned.
static size_t s3_align(size_t b) { return (b + 255) & ~size_t(255); }

static int shell_count_host(const int n[3]) {
  const int64_t m2 = int64_t(n[0] / 2) * (n[0] / 2) + int64_t(n[1] / 2) * (n[1] / 2) +
                     int64_t(n[2] / 2) * (n[2] / 2);
  int64_t K = 0;
  while (4 * m2 >= (2 * K + 1) * (2 * K + 1)) ++K;  // K - 1/2 <= |k| < K + 1/2
  return int(K) + 1;
}

bool spec3_shape_ok(const PatchDev& P) {
  for (int a = 0; a < 3; ++a) {
    FftPlan p;
    if (P.n[a] > kS3MaxLen || !make_fft_plan(P.n[a], p)) return false;
  }
  return true;
}

size_t spec3_workspace_bytes(const PatchDev& P, int* nb) {
  const int64_t nh = P.n[0] / 2 + 1;
  const int64_t cells = nh * P.n[1] * P.n[2];
  const int shells = shell_count_host(P.n);
  if (nb) *nb = shells;
  return s3_align(size_t(3 * cells) * sizeof(double2)) + s3_align(size_t(cells) * sizeof(double)) +
         s3_align(size_t(kSpec3BinBlocks) * shells * sizeof(double)) +
         s3_align(size_t(P.n[0] + P.n[1] + P.n[2]) * sizeof(double2));
}

template <class T>
static hipError_t launch_s3(const LaunchSpec3& L, hipStream_t st) {
  const PatchDev& P = L.single;
  FftPlan px, py, pz;
  if (!make_fft_plan(P.n[0], px) || !make_fft_plan(P.n[1], py) || !make_fft_plan(P.n[2], pz))
    return hipErrorInvalidValue;
  Spec3Args a{};
  a.pool = L.pool;
  a.base0 = P.base0;
  a.plane = P.plane;
  a.sy = P.sy;
  a.sz = P.sz;
  for (int i = 0; i < 3; ++i) a.n[i] = P.n[i];
  a.nh = P.n[0] / 2 + 1;
  a.ntk = (a.nh + kS3T - 1) / kS3T;
  a.gx = std::max(1, (kS3Elems / 2) / P.n[0]);
  a.nb = shell_count_host(P.n);
  a.cplane = int64_t(a.nh) * P.n[1] * P.n[2];
  char* w = static_cast<char*>(L.work);
  a.U = reinterpret_cast<double2*>(w);
  w += s3_align(size_t(3 * a.cplane) * sizeof(double2));
  a.P = reinterpret_cast<double*>(w);
  w += s3_align(size_t(a.cplane) * sizeof(double));
  a.partials = reinterpret_cast<double*>(w);
  w += s3_align(size_t(kSpec3BinBlocks) * a.nb * sizeof(double));
  double2* tw = reinterpret_cast<double2*>(w);
  a.tw = tw;
  a.dnx = FastDiv(uint32_t(P.n[0]));
  a.dny = FastDiv(uint32_t(P.n[1]));
  a.dnz = FastDiv(uint32_t(P.n[2]));
  a.dnh = FastDiv(uint32_t(a.nh));
  const int ntw = P.n[0] + P.n[1] + P.n[2];
  hipLaunchKernelGGL(spec3_twiddle_kernel, dim3(unsigned((ntw + 255) / 256)), dim3(256), 0, st, tw,
                     P.n[0], P.n[1], P.n[2]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int groups = (P.n[1] * P.n[2] + a.gx - 1) / a.gx;
  const int xgrid = std::min(groups, 8 * std::max(1, L.cu_count));
  const size_t xlds = size_t(P.n[0] + fft_lds((a.gx + (a.gx + 1) / 2) * P.n[0])) * sizeof(double2);
  hipLaunchKernelGGL(spec3_x_kernel<T>, dim3(unsigned(xgrid)), dim3(kS3Block), xlds, st, a, px);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t ylds = size_t(P.n[1] + fft_lds(kS3T * (P.n[1] + 1))) * sizeof(double2);
  hipLaunchKernelGGL(spec3_col_kernel<false>, dim3(unsigned(3 * P.n[2] * a.ntk)), dim3(kS3Block),
                     ylds, st, a, py);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t zlds = size_t(P.n[2] + fft_lds(kS3T * (P.n[2] + 1))) * sizeof(double2);
  hipLaunchKernelGGL(spec3_col_kernel<true>, dim3(unsigned(P.n[1] * a.ntk)), dim3(kS3Block), zlds,
                     st, a, pz);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(spec3_bin_kernel, dim3(unsigned(kSpec3BinBlocks)), dim3(kS3Block),
                     size_t(kS3Block / 64) * a.nb * sizeof(double), st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double N = double(P.n[0]) * P.n[1] * P.n[2];
  hipLaunchKernelGGL(spec3_final_kernel, dim3(unsigned(a.nb)), dim3(kS3Block), 0, st, a.partials,
                     kSpec3BinBlocks, a.nb, 2.0 * N * N, L.out);
  return hipGetLastError();
}

hipError_t launch_diag_spectrum3d(const LaunchSpec3& L, hipStream_t st) {
  if (!spec3_shape_ok(L.single) || !L.work || !L.out) return hipErrorInvalidValue;
  return L.fp64 ? launch_s3<double>(L, st) : launch_s3<float>(L, st);
}

}  // namespace hydro
