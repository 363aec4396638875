// euler.hpp -- per-zone and per-interface arithmetic of the split
// MUSCL-Hancock / HLLC update, shared by every sweep kernel of the library.
//
// A star is modelled as an ideal-gas fluid on a Cartesian grid (Zingale et
// al., arXiv:1510.05061, introduction).  Every sweep kernel (x lane-runs,
// y/z column marches, batched patches) calls exactly these inline
// functions, so a pencil produces the same bits whichever kernel sweeps it.
// The library is built with -ffp-contract=off; every fused multiply-add
// below is written out with fma(), so no contraction depends on the
// surrounding kernel.
//
// Scheme (state U = (rho, m_n, m_t1, m_t2, E) rotated into the sweep frame):
//   * primitive reconstruction with the monotonised-central limiter
//     (van Leer 1977): D = 0 unless both one-sided differences have the
//     same strict sign, else sign * min(2|a|, 2|b|, |a+b|/2);
//   * Hancock predictor in primitive form (Toro 2009 sec. 14.4):
//     W-/+ = W -/+ D/2 - (dt/dx)/2 A(W) D, plus a gravity half kick on the
//     normal velocity; a cell whose face state has rho <= 0 or p <= 0 falls
//     back to zero slopes;
//   * HLLC flux (Toro, Spruce & Speares 1994; Toro 2009 sec. 10.4) with
//     Davis (1988) wave-speed bounds;
//   * conservative update U -= (dt/dx)(F_{i+1/2} - F_{i-1/2}), then the
//     time-centred gravity source on the normal momentum and an energy
//     source built from the two face mass fluxes.
#pragma once

#include <hip/hip_runtime.h>

namespace hydro {

template <class T>
struct Prim {
  T r, u, t1, t2, p;
  T ri;  // 1 / rho of a cell-centred state (unused on face states)
};

template <class T>
struct Cons {
  T r, mn, mt1, mt2, e;
};

// Reciprocal, division and square-root policies.
//  * FP32: the hardware reciprocal and reciprocal square root (about 1 ulp).
//  * FP64: the hardware estimates refined by two Newton steps (about 1 ulp
//    in double), instead of the longer IEEE-exact division and square-root
//    sequences.
// Both are deterministic instruction sequences, so every kernel that calls
// them produces the same bits; both stay far inside the FP64 parity bound
// and the FP32 L1 bound against the oracle.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqrt_(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  double e = __builtin_fma(-(h * y), y, 0.5);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-(h * y), y, 0.5);
  return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double div_(double a, double b) { return a * rcp(b); }
__device__ __forceinline__ float div_(float a, float b) { return a * rcp(b); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmin_(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fmin_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double fmax_(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double fabs_(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float fabs_(float a) { return __builtin_fabsf(a); }

// Sound speed sqrt(gamma p / rho) written as gamma p / sqrt(gamma p rho):
// one reciprocal square root, no division.
template <class T>
__device__ __forceinline__ T sound(T gamma, T p, T rho) {
  T gp = gamma * p;
  return gp * rsqrt_(gp * rho);
}

// Constants of one sweep, in the arithmetic type.
template <class T>
struct SweepConst {
  T gamma;        // ratio of specific heats
  T gm1;          // gamma - 1
  T inv_gm1;      // 1 / (gamma - 1)
  T dtdx;         // dt / dx
  T kick;         // dt g / 2 along the sweep axis (gravity half kick)
  T dtg;          // dt g along the sweep axis
  bool has_g;     // g along the sweep axis is nonzero
};

// Constants of a sweep of length dt over cells of width dx along an axis
// with gravity g, rounded once from FP64 into the arithmetic type.
template <class T>
__device__ __forceinline__ SweepConst<T> make_const(double dt, double dx, double gamma,
                                                    double g) {
  SweepConst<T> k;
  k.gamma = T(gamma);
  k.gm1 = T(gamma - 1.0);
  k.inv_gm1 = T(1.0 / (gamma - 1.0));
  double dtdx = dt / dx;
  k.dtdx = T(dtdx);
  k.kick = T(0.5 * dt * g);
  k.dtg = T(dt * g);
  k.has_g = (g != 0.0);
  return k;
}

// Conserved -> primitive; p = (gamma-1)(E - |m|^2 / (2 rho)).
template <class T>
__device__ __forceinline__ Prim<T> to_prim(const Cons<T>& U, const SweepConst<T>& k) {
  Prim<T> W;
  T ri = rcp(U.r);
  W.ri = ri;
  W.r = U.r;
  W.u = U.mn * ri;
  W.t1 = U.mt1 * ri;
  W.t2 = U.mt2 * ri;
  T ke = fma_(U.mn, W.u, fma_(U.mt1, W.t1, U.mt2 * W.t2));  // |m|^2 / rho
  W.p = k.gm1 * fma_(T(-0.5), ke, U.e);
  return W;
}

// Mirror image across a wall normal to the sweep axis.
template <class T>
__device__ __forceinline__ Prim<T> mirror(const Prim<T>& W) {
  Prim<T> M = W;
  M.u = -W.u;
  return M;
}

// minmod(x, y) = median(x, y, 0): the smaller magnitude when x and y share a
// strict sign, else 0.  One v_med3 in FP32.
__device__ __forceinline__ float minmod(float x, float y) {
  return __builtin_amdgcn_fmed3f(x, y, 0.0f);
}
__device__ __forceinline__ double minmod(double x, double y) {
  return __builtin_fmax(__builtin_fmin(x, y), __builtin_fmin(__builtin_fmax(x, y), 0.0));
}

// Half of the MC limited slope from the left difference a and the right
// difference b.  MC = sign(a) min(2|a|, 2|b|, |a+b|/2) when a and b share a
// strict sign, else 0 (van Leer 1977); equivalently
// MC = minmod((a+b)/2, 2 minmod(a, b)), so MC/2 = minmod((a+b)/4, minmod(a, b))
// (scaling by a power of two is exact).
template <class T>
__device__ __forceinline__ T half_mc(T a, T b) {
  return minmod(T(0.25) * (a + b), minmod(a, b));
}

// Face states (W-, W+) of the cell W with left and right neighbours Wl, Wr.
// `kick` is the gravity half kick of this cell (negated for a mirrored ghost
// behind a reflecting wall, whose gravity is mirrored too).  With d = D/2:
// W-/+ = W - (dt/dx) A(W) d -/+ d.
template <class T>
__device__ __forceinline__ void face_states(const Prim<T>& Wl, const Prim<T>& W,
                                            const Prim<T>& Wr, const SweepConst<T>& k,
                                            T kick, Prim<T>& Wm, Prim<T>& Wp) {
  Prim<T> d;
  d.r = half_mc(W.r - Wl.r, Wr.r - W.r);
  d.u = half_mc(W.u - Wl.u, Wr.u - W.u);
  d.t1 = half_mc(W.t1 - Wl.t1, Wr.t1 - W.t1);
  d.t2 = half_mc(W.t2 - Wl.t2, Wr.t2 - W.t2);
  d.p = half_mc(W.p - Wl.p, Wr.p - W.p);
  // A(W) d for the primitive Euler system
  T ar = fma_(W.u, d.r, W.r * d.u);
  T au = fma_(W.u, d.u, d.p * W.ri);
  T at1 = W.u * d.t1;
  T at2 = W.u * d.t2;
  T ap = fma_(k.gamma * W.p, d.u, W.u * d.p);
  T h = k.dtdx;
  T br = fma_(-h, ar, W.r), bu = fma_(-h, au, W.u), bt1 = fma_(-h, at1, W.t1);
  T bt2 = fma_(-h, at2, W.t2), bp = fma_(-h, ap, W.p);
  Wm.r = br - d.r;
  Wp.r = br + d.r;
  Wm.u = bu - d.u;
  Wp.u = bu + d.u;
  Wm.t1 = bt1 - d.t1;
  Wp.t1 = bt1 + d.t1;
  Wm.t2 = bt2 - d.t2;
  Wp.t2 = bt2 + d.t2;
  Wm.p = bp - d.p;
  Wp.p = bp + d.p;
  T lo = fmin_(fmin_(Wm.r, Wp.r), fmin_(Wm.p, Wp.p));
  if (lo <= T(0)) {  // first order for this cell
    Wm = W;
    Wp = W;
  }
  if (k.has_g) {
    Wm.u += kick;
    Wp.u += kick;
  }
}

// HLLC flux across the interface between the left face state L and the
// right face state R.  Branches: S_L >= 0 -> F_L; S* >= 0 -> left star;
// S_R > 0 -> right star; else F_R.  Only the upwind side is evaluated.
template <class T>
__device__ __forceinline__ Cons<T> hllc(const Prim<T>& L, const Prim<T>& R,
                                        const SweepConst<T>& k) {
  T cL = sound(k.gamma, L.p, L.r);
  T cR = sound(k.gamma, R.p, R.r);
  T SL = fmin_(L.u - cL, R.u - cR);
  T SR = fmax_(L.u + cL, R.u + cR);
  T aL = L.r * (SL - L.u);
  T aR = R.r * (SR - R.u);
  T num = (R.p - L.p) + fma_(aL, L.u, -(aR * R.u));
  T den = aL - aR;
  T Ss = div_(num, den);
  bool left = (SL >= T(0)) | (Ss >= T(0));
  bool star = left ? (SL < T(0)) : (SR > T(0));
  T r = left ? L.r : R.r;
  T u = left ? L.u : R.u;
  T t1 = left ? L.t1 : R.t1;
  T t2 = left ? L.t2 : R.t2;
  T p = left ? L.p : R.p;
  T S = left ? SL : SR;
  T v2 = fma_(u, u, fma_(t1, t1, t2 * t2));
  T E = fma_(p, k.inv_gm1, T(0.5) * r * v2);
  T ru = r * u;
  Cons<T> F;
  F.r = ru;
  F.mn = fma_(ru, u, p);
  F.mt1 = ru * t1;
  F.mt2 = ru * t2;
  F.e = u * (E + p);
  if (star) {
    // U*_K - U_K written through g = f_K - 1 = (S* - u)/(S_K - S*), with
    // f_K = (S_K - u)/(S_K - S*):
    //   rho: rho g;  m_n: rho ((S* - u) + g S*);  m_t: rho t g;
    //   E:   g E + f_K (S* - u)(rho S* + p/(S_K - u)).
    // Every term carries S* - u or g, so a state with S* = u (a contact at
    // rest, a mirror wall) gets no star correction at all, whatever the
    // rounding of the reciprocals.
    T dS = Ss - u;
    T g = div_(dS, S - Ss);
    T f = T(1) + g;
    T rg = r * g;
    T q = fma_(p, rcp(S - u), r * Ss);
    F.r = fma_(S, rg, F.r);
    F.mn = fma_(S, r * fma_(g, Ss, dS), F.mn);
    F.mt1 = fma_(S, rg * t1, F.mt1);
    F.mt2 = fma_(S, rg * t2, F.mt2);
    F.e = fma_(S, fma_(g, E, f * dS * q), F.e);
  }
  return F;
}

// Conservative update of one cell from its left and right face fluxes,
// then the gravity source.
template <class T>
__device__ __forceinline__ void update(Cons<T>& U, const Cons<T>& Fl, const Cons<T>& Fr,
                                       const SweepConst<T>& k) {
  T r_old = U.r;
  U.r = fma_(-k.dtdx, Fr.r - Fl.r, U.r);
  U.mn = fma_(-k.dtdx, Fr.mn - Fl.mn, U.mn);
  U.mt1 = fma_(-k.dtdx, Fr.mt1 - Fl.mt1, U.mt1);
  U.mt2 = fma_(-k.dtdx, Fr.mt2 - Fl.mt2, U.mt2);
  U.e = fma_(-k.dtdx, Fr.e - Fl.e, U.e);
  if (k.has_g) {
    U.mn = fma_(k.dtg, T(0.5) * (r_old + U.r), U.mn);
    U.e = fma_(k.dtg, T(0.5) * (Fl.r + Fr.r), U.e);
  }
}

// Health of an updated cell from its primitives: rho > 0, p > 0 and a finite
// energy (a NaN fails every comparison).
template <class T>
__device__ __forceinline__ bool cell_ok(const Cons<T>& U, const Prim<T>& W) {
  return (W.r > T(0)) && (W.p > T(0)) && (fabs_(U.e) < T(__builtin_huge_val()));
}

}  // namespace hydro
