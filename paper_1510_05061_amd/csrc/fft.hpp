// fft.hpp -- device helpers shared by the spectra (diag.hip, spec3.hip):
// division by invariant integers, complex arithmetic in FP64, and an
// in-place mixed-radix (4, 2, 3) Stockham FFT of complex lines held in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hydro {

// Unsigned 32-bit division by an invariant d >= 1 with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the unsigned algorithm of their figure 4.1):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, and for every n
// q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) with t = mulhi(m, n).
struct FastDiv {
  uint32_t d, m, s1, s2;
  __host__ __device__ FastDiv() : d(1), m(1), s1(0), s2(0) {}
  __host__ __device__ explicit FastDiv(uint32_t div) : d(div) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < div) ++l;
    m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - div)) / div + 1);
    s1 = l < 1 ? l : 1;
    s2 = l > 1 ? l - 1 : 0;
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// -i a
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// W_16^e = exp(-2 pi i e / 16) times a, for the internal twiddles of the
// 16-point DFT (e = b c, b and c in 0..3)
template <int E>
__device__ __forceinline__ double2 w16(double2 a) {
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double H = 0.70710678118654752440;   // cos(pi/4)
  if constexpr (E == 0) return a;
  else if constexpr (E == 1) return cmul(a, make_double2(C1, -S1));
  else if constexpr (E == 2) return cmul(a, make_double2(H, -H));
  else if constexpr (E == 3) return cmul(a, make_double2(S1, -C1));
  else if constexpr (E == 4) return cmi(a);
  else if constexpr (E == 6) return cmul(a, make_double2(-H, -H));
  else return cmul(a, make_double2(-C1, S1));  // E == 9
}

// Forward R-point DFT (R = 2, 3, 4, 16) of v in place, W_R = exp(-2 pi i / R).
// R = 16 as 4 x 4: with r = 4a + b and k = c + 4d,
// X[c + 4d] = sum_b W_4^(bd) W_16^(bc) sum_a x[4a + b] W_4^(ac).
template <int R>
__device__ __forceinline__ void dft_small(double2 (&v)[R]) {
  if constexpr (R == 16) {
    double2 y[4][4];  // y[b][c]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double2 t[4] = {v[b], v[4 + b], v[8 + b], v[12 + b]};
      dft_small<4>(t);
#pragma unroll
      for (int c = 0; c < 4; ++c) y[b][c] = t[c];
    }
    y[1][1] = w16<1>(y[1][1]); y[1][2] = w16<2>(y[1][2]); y[1][3] = w16<3>(y[1][3]);
    y[2][1] = w16<2>(y[2][1]); y[2][2] = w16<4>(y[2][2]); y[2][3] = w16<6>(y[2][3]);
    y[3][1] = w16<3>(y[3][1]); y[3][2] = w16<6>(y[3][2]); y[3][3] = w16<9>(y[3][3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double2 t[4] = {y[0][c], y[1][c], y[2][c], y[3][c]};
      dft_small<4>(t);
#pragma unroll
      for (int d = 0; d < 4; ++d) v[c + 4 * d] = t[d];
    }
  } else if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = cmi(csub(v[1], v[3]));  // -i (v1 - v3)
    v[0] = cadd(s02, s13);
    v[1] = cadd(d02, d13);
    v[2] = csub(s02, s13);
    v[3] = csub(d02, d13);
  } else {  // R == 3: W_3 = -1/2 - i sqrt(3)/2
    const double h = 0.86602540378443864676;  // sqrt(3) / 2
    const double2 t1 = cadd(v[1], v[2]);
    const double2 t2 = make_double2(v[0].x - 0.5 * t1.x, v[0].y - 0.5 * t1.y);
    const double2 dd = csub(v[1], v[2]);
    const double2 t3 = make_double2(h * dd.y, -h * dd.x);  // -i h (v1 - v2)
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
}

// Stages of an FFT of length n = 16^a 4^b 2^c 3^d (radix 16 first, then 4,
// 2, 3: fewer stages mean fewer LDS round trips and barriers), built on the
// host.  Stage s has radix rad[s], span ns[s] (product of
// the earlier radices) and twiddle step tw[s] = n / (ns R).
constexpr int kFftMaxStages = 12;
struct FftPlan {
  int n;
  int nst;
  int rad[kFftMaxStages];
  int ns[kFftMaxStages];
  int tw[kFftMaxStages];
  FastDiv nsd[kFftMaxStages];  // division by ns
  FastDiv md[kFftMaxStages];   // division by n / R (butterflies per line)
};

// false if n is not 2^a 3^b (1 <= n)
inline bool make_fft_plan(int n, FftPlan& p) {
  p = FftPlan{};
  p.n = n;
  if (n < 1) return false;
  int m = n;
  while (m % 16 == 0 && p.nst < kFftMaxStages) { p.rad[p.nst++] = 16; m /= 16; }
  while (m % 4 == 0 && p.nst < kFftMaxStages) { p.rad[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0 && p.nst < kFftMaxStages) { p.rad[p.nst++] = 2; m /= 2; }
  while (m % 3 == 0 && p.nst < kFftMaxStages) { p.rad[p.nst++] = 3; m /= 3; }
  if (m != 1) return false;
  for (int s = 0, ns = 1; s < p.nst; ns *= p.rad[s], ++s) {
    p.ns[s] = ns;
    p.tw[s] = n / (ns * p.rad[s]);
    p.nsd[s] = FastDiv(uint32_t(ns));
    p.md[s] = FastDiv(uint32_t(n / p.rad[s]));
  }
  return true;
}

// LDS slot of complex element o of an FFT buffer: one pad slot after every
// 16 elements.  A radix-16 stage writes its outputs 16 elements apart (256
// bytes, the same banks for every lane); with the pad they land 272 bytes
// apart, on different banks.  A buffer of n elements takes fft_lds(n) slots.
__host__ __device__ __forceinline__ int fft_pad(int o) { return o + (o >> 4); }
__host__ __device__ __forceinline__ int fft_lds(int n) { return n + (n >> 4) + 1; }

// One radix-R stage of the Stockham autosort FFT (Govindaraju et al., SC
// 2008) over nl complex lines in LDS (line l at buf + l ls), in place:
// butterfly j of a line takes the elements j + r n/R, twiddled by
// W^(r (j mod ns) tw), through an R-point DFT to (j div ns) ns R +
// (j mod ns) + r ns.  Every thread first holds the inputs of its
// butterflies (j = t, t + B, ... over the nl n/R of the stage, at most MAXB)
// in registers; after a barrier it writes the outputs; a second barrier
// ends the stage.  Element o of the buffer sits at slot fft_pad(o).
// W[t] = exp(-2 pi i t / n) in LDS.  B = blockDim.x.
template <int R, int MAXB>
__device__ __forceinline__ void fft_stage_inplace(double2* buf, int nl, int ls, int n, int ns,
                                                  int tw, const FastDiv& md, const FastDiv& nsd,
                                                  const double2* W) {
  const int m = n / R, nb = nl * m;
  double2 v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = int(threadIdx.x) + b * int(blockDim.x);
    dst[b] = -1;
    if (j < nb) {
      const int l = int(md.div(uint32_t(j))), jj = j - l * m;
      const int q = int(nsd.div(uint32_t(jj))), k = jj - q * ns;
      const int s = l * ls + jj;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 x = buf[fft_pad(s + r * m)];
        v[b][r] = r == 0 ? x : cmul(x, W[r * k * tw]);
      }
      dst[b] = l * ls + q * ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    if (dst[b] >= 0) {
      dft_small<R>(v[b]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[fft_pad(dst[b] + r * ns)] = v[b][r];
    }
  }
  __syncthreads();
}

// The whole FFT of nl lines of length p.n (nl p.n <= EMAX elements) with a
// workgroup of BLOCK threads; the caller has made the input visible
// (barrier) and the output is visible to every thread on return.
template <int EMAX, int BLOCK>
__device__ void fft_lines_inplace(double2* buf, int nl, int ls, const FftPlan& p, const double2* W) {
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    if (R == 16)
      fft_stage_inplace<16, (EMAX + 16 * BLOCK - 1) / (16 * BLOCK)>(
          buf, nl, ls, p.n, p.ns[s], p.tw[s], p.md[s], p.nsd[s], W);
    else if (R == 4)
      fft_stage_inplace<4, (EMAX + 4 * BLOCK - 1) / (4 * BLOCK)>(buf, nl, ls, p.n, p.ns[s], p.tw[s],
                                                                p.md[s], p.nsd[s], W);
    else if (R == 2)
      fft_stage_inplace<2, (EMAX + 2 * BLOCK - 1) / (2 * BLOCK)>(buf, nl, ls, p.n, p.ns[s], p.tw[s],
                                                                p.md[s], p.nsd[s], W);
    else
      fft_stage_inplace<3, (EMAX + 3 * BLOCK - 1) / (3 * BLOCK)>(buf, nl, ls, p.n, p.ns[s], p.tw[s],
                                                                p.md[s], p.nsd[s], W);
  }
}

}  // namespace hydro
