/*
 * oracle.c -- plain, slow, FP64 CPU oracle for one compressible-Euler zone
 * update (the finite-volume scheme used to model a star as a fluid in
 * Zingale, Calder, Malone & Timmes, arXiv:1510.05061, introduction).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It is used by tests/, by __graft_entry__.smoke() and by
 * the cpu_baseline leg of bench.py, and by nothing else.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * The paper names no numerical method; the scheme below is the textbook one
 * it implies for a "star as a fluid" on a decomposed grid:
 *   - ideal-gas Euler equations in conserved form U = (rho, mx, my, mz, E);
 *   - piecewise-linear reconstruction of the primitive variables with the
 *     monotonised-central (MC) limiter (van Leer 1977, J. Comput. Phys. 23,
 *     276);
 *   - the MUSCL-Hancock half-step predictor in primitive form
 *     (Toro 2009, "Riemann Solvers and Numerical Methods for Fluid
 *     Dynamics", 3rd ed., sec. 14.4);
 *   - the HLLC approximate Riemann solver (Toro, Spruce & Speares 1994,
 *     Shock Waves 4, 25; Toro 2009 sec. 10.4) with Davis (1988) wave speeds;
 *   - conservative flux differencing in dimensionally split sweeps, ordered
 *     x,y,z on even steps and z,y,x on odd steps (Strang 1968);
 *   - a constant gravity source: half kick in the predictor, time-centred
 *     momentum source and an energy source built from the face mass fluxes;
 *   - a global CFL reduction dt = C / max_i max_d (|v_d| + c) / dx_d
 *     (the "global communication each timestep" of the paper's section
 *     "Capabilities needed"; nearest-neighbour communication is the ghost
 *     fill below).
 *
 * Layout: array of cells, 5 doubles per cell, with NG explicit ghost layers
 * on every side of every axis (deliberately unlike the GPU's plane layout).
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 5
#define NG 2

enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1, ORC_REFLECT = 2 };

enum {
  ORC_OK = 0,
  ORC_EINVAL = 1,
  ORC_ENOMEM = 2,
  ORC_ENUMERIC = 3
};

typedef struct {
  int32_t n[3];        /* interior cells along x, y, z */
  int32_t bc[6];       /* xlo, xhi, ylo, yhi, zlo, zhi */
  double dx[3];        /* cell widths */
  double gamma;        /* ratio of specific heats */
  double cfl;          /* Courant number */
  double grav[3];      /* constant gravitational acceleration */
  int32_t nthreads;    /* OpenMP threads (<=0: library default) */
  int32_t pad;
} orc_params;

/* ------------------------------------------------------------------ */
/* Grid with ghost layers                                              */
/* ------------------------------------------------------------------ */

typedef struct {
  int n[3];
  int s[3];        /* stored extent = n + 2*NG */
  double *u;       /* s[2]*s[1]*s[0] cells * NV */
} grid;

static size_t cell_index(const grid *g, int i, int j, int k) {
  /* i, j, k are interior-based indices in [-NG, n+NG) */
  return (((size_t)(k + NG) * g->s[1] + (size_t)(j + NG)) * g->s[0] +
          (size_t)(i + NG)) * NV;
}

static int grid_alloc(grid *g, const int n[3]) {
  for (int d = 0; d < 3; ++d) {
    g->n[d] = n[d];
    g->s[d] = n[d] + 2 * NG;
  }
  size_t cells = (size_t)g->s[0] * g->s[1] * g->s[2];
  g->u = (double *)calloc(cells * NV, sizeof(double));
  return g->u ? ORC_OK : ORC_ENOMEM;
}

static void grid_free(grid *g) {
  free(g->u);
  g->u = NULL;
}

/* planes[v][k][j][i] (interior only, x fastest)  <->  grid cells */
static void grid_load(grid *g, const double *planes) {
  const size_t plane = (size_t)g->n[0] * g->n[1] * g->n[2];
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        size_t src = ((size_t)k * g->n[1] + j) * g->n[0] + i;
        double *c = g->u + cell_index(g, i, j, k);
        for (int v = 0; v < NV; ++v) c[v] = planes[v * plane + src];
      }
}

static void grid_store(const grid *g, double *planes) {
  const size_t plane = (size_t)g->n[0] * g->n[1] * g->n[2];
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        size_t dst = ((size_t)k * g->n[1] + j) * g->n[0] + i;
        const double *c = g->u + cell_index(g, i, j, k);
        for (int v = 0; v < NV; ++v) planes[v * plane + dst] = c[v];
      }
}

/* ------------------------------------------------------------------ */
/* Point-wise physics                                                  */
/* ------------------------------------------------------------------ */

/* Conserved (rho, m_n, m_t1, m_t2, E) -> primitive (rho, u, t1, t2, p);
 * ideal gas p = (gamma-1) (E - |m|^2 / (2 rho)). */
void oracle_prim(const double U[NV], double gamma, double W[NV]) {
  double rho = U[0];
  double mm = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  W[0] = rho;
  W[1] = U[1] / rho;
  W[2] = U[2] / rho;
  W[3] = U[3] / rho;
  W[4] = (gamma - 1.0) * (U[4] - 0.5 * mm / rho);
}

/* MC limited slope from the left difference a and the right difference b:
 * zero unless a and b are both strictly positive or both strictly negative,
 * else sign(a) * min(2|a|, 2|b|, |a+b|/2) (van Leer 1977). */
double oracle_mc_slope(double a, double b) {
  int same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
  if (!same) return 0.0;
  double m = fmin(2.0 * fabs(a), 2.0 * fabs(b));
  m = fmin(m, 0.5 * fabs(a + b));
  return a > 0.0 ? m : -m;
}

/* Total energy of a primitive state. */
static double energy_of(const double W[NV], double gamma) {
  double v2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  return W[4] / (gamma - 1.0) + 0.5 * W[0] * v2;
}

/* Physical flux along the sweep direction of a primitive state. */
static void flux_of(const double W[NV], double E, double F[NV]) {
  double rho = W[0], u = W[1];
  F[0] = rho * u;
  F[1] = rho * u * u + W[4];
  F[2] = rho * u * W[2];
  F[3] = rho * u * W[3];
  F[4] = u * (E + W[4]);
}

/* HLLC flux between the left face state WL and the right face state WR
 * (primitive, normal velocity in slot 1), following Toro 2009 sec. 10.4.
 * Davis wave-speed bounds S_L = min(uL-cL, uR-cR), S_R = max(uL+cL, uR+cR);
 * contact speed
 *   S* = (pR - pL + rhoL uL (S_L-uL) - rhoR uR (S_R-uR)) /
 *        (rhoL (S_L-uL) - rhoR (S_R-uR));
 * star state of side K written as f_K * (rho_K, rho_K S*, rho_K t1, rho_K t2,
 * E_K + (S*-u_K)(rho_K S* + p_K/(S_K-u_K))) with f_K = (S_K-u_K)/(S_K-S*)
 * (algebraically the textbook star state; this form returns U_K exactly when
 * u_K = S* = 0); flux F*_K = F_K + S_K (U*_K - U_K).
 * S* = 0 takes the left star branch. */
void oracle_hllc(const double WL[NV], const double WR[NV], double gamma,
                 double F[NV]) {
  double rL = WL[0], uL = WL[1], pL = WL[4];
  double rR = WR[0], uR = WR[1], pR = WR[4];
  double cL = sqrt(gamma * pL / rL);
  double cR = sqrt(gamma * pR / rR);
  double SL = fmin(uL - cL, uR - cR);
  double SR = fmax(uL + cL, uR + cR);
  double num = (pR - pL) + (rL * uL * (SL - uL) - rR * uR * (SR - uR));
  double den = rL * (SL - uL) - rR * (SR - uR);
  double Ss = num / den;

  double EL = energy_of(WL, gamma), ER = energy_of(WR, gamma);
  double FL[NV], FR[NV];
  flux_of(WL, EL, FL);
  flux_of(WR, ER, FR);

  /* branch order: S_L >= 0 -> F_L; else S* >= 0 -> left star;
   * else S_R > 0 -> right star; else F_R */
  if (SL >= 0.0) {
    for (int v = 0; v < NV; ++v) F[v] = FL[v];
    return;
  }
  const double *W;
  const double *FK;
  double S, E;
  if (Ss >= 0.0) {
    W = WL; FK = FL; S = SL; E = EL;
  } else if (SR > 0.0) {
    W = WR; FK = FR; S = SR; E = ER;
  } else {
    for (int v = 0; v < NV; ++v) F[v] = FR[v];
    return;
  }
  double rho = W[0], u = W[1], p = W[4];
  double f = (S - u) / (S - Ss);
  double Us[NV], Uk[NV];
  Us[0] = f * rho;
  Us[1] = f * (rho * Ss);
  Us[2] = f * (rho * W[2]);
  Us[3] = f * (rho * W[3]);
  Us[4] = f * (E + (Ss - u) * (rho * Ss + p / (S - u)));
  Uk[0] = rho;
  Uk[1] = rho * u;
  Uk[2] = rho * W[2];
  Uk[3] = rho * W[3];
  Uk[4] = E;
  for (int v = 0; v < NV; ++v) F[v] = FK[v] + S * (Us[v] - Uk[v]);
}

/* MUSCL-Hancock face states of one cell (Toro 2009 sec. 14.4, primitive
 * form): W-/+ = W -/+ D/2 - (dt/dx)/2 * A(W) D, with
 * A(W) D = (u Drho + rho Du, u Du + Dp/rho, u Dt1, u Dt2, gamma p Du + u Dp).
 * A nonzero g adds dt*g/2 to the normal velocity of both faces. */
static void hancock(const double W[NV], const double D[NV], double dtdx,
                    double gamma, double half_dt_g, int has_g,
                    double Wm[NV], double Wp[NV]) {
  double rho = W[0], u = W[1], p = W[4];
  double AD[NV];
  AD[0] = u * D[0] + rho * D[1];
  AD[1] = u * D[1] + D[4] / rho;
  AD[2] = u * D[2];
  AD[3] = u * D[3];
  AD[4] = gamma * p * D[1] + u * D[4];
  for (int v = 0; v < NV; ++v) {
    double half_slope = 0.5 * D[v];
    double drift = 0.5 * dtdx * AD[v];
    Wm[v] = W[v] - half_slope - drift;
    Wp[v] = W[v] + half_slope - drift;
  }
  if (has_g) {
    Wm[1] += half_dt_g;
    Wp[1] += half_dt_g;
  }
}

/* ------------------------------------------------------------------ */
/* One pencil                                                          */
/* ------------------------------------------------------------------ */

/* pen: N + 2*NG cells of (rho, m_n, m_t1, m_t2, E), ghosts included;
 * updates the N interior cells in place.  Scratch arrays are sized by the
 * caller.  Ghost cells behind a reflecting wall are the mirror image of the
 * domain, so their gravity is mirrored too (lo_mirror / hi_mirror): the
 * half kick of those ghosts has the opposite sign, which keeps the two wall
 * face states exact mirror images.  Returns the number of cells that fell
 * back to zero slopes. */
static long sweep_pencil(double (*pen)[NV], int N, double dt, double dx,
                         double gamma, double g, int lo_mirror, int hi_mirror,
                         double (*W)[NV], double (*Wm)[NV], double (*Wp)[NV],
                         double (*F)[NV]) {
  const int M = N + 2 * NG;      /* stored cells; index c = i + NG */
  const double dtdx = dt / dx;
  const int has_g = (g != 0.0);
  const double half_dt_g = 0.5 * dt * g;
  long fallbacks = 0;

  for (int c = 0; c < M; ++c) oracle_prim(pen[c], gamma, W[c]);

  /* slopes and face states for cells i = -1 .. N (c = 1 .. M-2) */
  for (int c = 1; c <= M - 2; ++c) {
    double D[NV];
    for (int v = 0; v < NV; ++v)
      D[v] = oracle_mc_slope(W[c][v] - W[c - 1][v], W[c + 1][v] - W[c][v]);
    int mirrored = (c < NG && lo_mirror) || (c >= NG + N && hi_mirror);
    double kick = mirrored ? -half_dt_g : half_dt_g;
    hancock(W[c], D, dtdx, gamma, kick, has_g, Wm[c], Wp[c]);
    if (Wm[c][0] <= 0.0 || Wm[c][4] <= 0.0 || Wp[c][0] <= 0.0 ||
        Wp[c][4] <= 0.0) {
      double Z[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
      hancock(W[c], Z, dtdx, gamma, kick, has_g, Wm[c], Wp[c]);
      ++fallbacks;
    }
  }

  /* fluxes at faces i+1/2 for i = -1 .. N-1; F[c] is the face right of c */
  for (int c = 1; c <= M - 3; ++c) oracle_hllc(Wp[c], Wm[c + 1], gamma, F[c]);

  /* conservative update of interior cells, then the gravity source */
  for (int c = NG; c < NG + N; ++c) {
    double rho_old = pen[c][0];
    for (int v = 0; v < NV; ++v) pen[c][v] -= dtdx * (F[c][v] - F[c - 1][v]);
    if (has_g) {
      pen[c][1] += dt * g * (0.5 * (rho_old + pen[c][0]));
      pen[c][4] += dt * g * (0.5 * (F[c - 1][0] + F[c][0]));
    }
  }
  return fallbacks;
}

/* ------------------------------------------------------------------ */
/* Ghost fill along one axis                                           */
/* ------------------------------------------------------------------ */

/* component order of a pencil along axis d: normal, then the two other
 * axes in ascending order */
static void axis_perm(int d, int perm[3]) {
  perm[0] = d;
  perm[1] = d == 0 ? 1 : 0;
  perm[2] = d == 2 ? 1 : 2;
}

static double *cell_at(grid *g, int d, int a, int t1, int t2) {
  /* a = index along d; (t1, t2) = indices along the two other axes */
  int idx[3];
  int perm[3];
  axis_perm(d, perm);
  idx[perm[0]] = a;
  idx[perm[1]] = t1;
  idx[perm[2]] = t2;
  return g->u + cell_index(g, idx[0], idx[1], idx[2]);
}

static void fill_ghosts(grid *g, int d, const int bc[6]) {
  int perm[3];
  axis_perm(d, perm);
  const int N = g->n[d];
  const int n1 = g->n[perm[1]], n2 = g->n[perm[2]];
  for (int b = 0; b < n2; ++b)
    for (int a = 0; a < n1; ++a)
      for (int k = 1; k <= NG; ++k) {
        /* low side: ghost -k */
        double *dst = cell_at(g, d, -k, a, b);
        double *src;
        int negate = 0;
        switch (bc[2 * d]) {
          case ORC_PERIODIC: src = cell_at(g, d, N - k, a, b); break;
          case ORC_OUTFLOW: src = cell_at(g, d, 0, a, b); break;
          default: src = cell_at(g, d, k - 1, a, b); negate = 1; break;
        }
        memcpy(dst, src, NV * sizeof(double));
        if (negate) dst[1 + d] = -dst[1 + d];
        /* high side: ghost N-1+k */
        dst = cell_at(g, d, N - 1 + k, a, b);
        negate = 0;
        switch (bc[2 * d + 1]) {
          case ORC_PERIODIC: src = cell_at(g, d, k - 1, a, b); break;
          case ORC_OUTFLOW: src = cell_at(g, d, N - 1, a, b); break;
          default: src = cell_at(g, d, N - k, a, b); negate = 1; break;
        }
        memcpy(dst, src, NV * sizeof(double));
        if (negate) dst[1 + d] = -dst[1 + d];
      }
}

/* ------------------------------------------------------------------ */
/* Sweeps and steps                                                    */
/* ------------------------------------------------------------------ */

/* One sweep along axis d.  fout (may be NULL) receives the face fluxes the
 * update used: 5 planes (lab components rho, mx, my, mz, E) of the grid's
 * shape with N + 1 entries along d, entry i being the face between cells
 * i - 1 and i. */
static long sweep_axis(grid *g, int d, const orc_params *p, double dt,
                       double *fout) {
  int perm[3];
  axis_perm(d, perm);
  const int N = g->n[d];
  const int n1 = g->n[perm[1]], n2 = g->n[perm[2]];
  const int M = N + 2 * NG;
  const long npencil = (long)n1 * n2;
  long fallbacks = 0;
  int fn[3] = {g->n[0], g->n[1], g->n[2]};
  fn[d] = N + 1;
  const size_t fplane = (size_t)fn[0] * fn[1] * fn[2];

  fill_ghosts(g, d, p->bc);

#pragma omp parallel reduction(+ : fallbacks)
  {
    double(*pen)[NV] = malloc(sizeof(double[NV]) * M);
    double(*W)[NV] = malloc(sizeof(double[NV]) * M);
    double(*Wm)[NV] = malloc(sizeof(double[NV]) * M);
    double(*Wp)[NV] = malloc(sizeof(double[NV]) * M);
    double(*F)[NV] = malloc(sizeof(double[NV]) * M);
#pragma omp for schedule(static)
    for (long q = 0; q < npencil; ++q) {
      int a = (int)(q % n1), b = (int)(q / n1);
      /* gather with the components rotated to (rho, m_n, m_t1, m_t2, E) */
      for (int c = 0; c < M; ++c) {
        const double *src = cell_at(g, d, c - NG, a, b);
        pen[c][0] = src[0];
        pen[c][1] = src[1 + perm[0]];
        pen[c][2] = src[1 + perm[1]];
        pen[c][3] = src[1 + perm[2]];
        pen[c][4] = src[4];
      }
      fallbacks += sweep_pencil(pen, N, dt, p->dx[d], p->gamma, p->grav[d],
                                p->bc[2 * d] == ORC_REFLECT,
                                p->bc[2 * d + 1] == ORC_REFLECT, W, Wm, Wp, F);
      if (fout) {
        for (int i = 0; i <= N; ++i) {
          /* face i - 1/2 is the face right of stored cell NG - 1 + i */
          const double *f = F[NG - 1 + i];
          int idx[3];
          idx[perm[0]] = i;
          idx[perm[1]] = a;
          idx[perm[2]] = b;
          const size_t o = ((size_t)idx[2] * fn[1] + idx[1]) * fn[0] + idx[0];
          fout[o] = f[0];
          fout[(1 + perm[0]) * fplane + o] = f[1];
          fout[(1 + perm[1]) * fplane + o] = f[2];
          fout[(1 + perm[2]) * fplane + o] = f[3];
          fout[4 * fplane + o] = f[4];
        }
      }
      for (int c = NG; c < NG + N; ++c) {
        double *dst = cell_at(g, d, c - NG, a, b);
        dst[0] = pen[c][0];
        dst[1 + perm[0]] = pen[c][1];
        dst[1 + perm[1]] = pen[c][2];
        dst[1 + perm[2]] = pen[c][3];
        dst[4] = pen[c][4];
      }
    }
    free(pen);
    free(W);
    free(Wm);
    free(Wp);
    free(F);
  }
  return fallbacks;
}

static int params_ok(const orc_params *p) {
  for (int d = 0; d < 3; ++d) {
    if (p->n[d] < 1 || !(p->dx[d] > 0.0)) return 0;
    if (p->bc[2 * d] < 0 || p->bc[2 * d] > 2) return 0;
    if (p->bc[2 * d + 1] < 0 || p->bc[2 * d + 1] > 2) return 0;
    if ((p->bc[2 * d] == ORC_PERIODIC) != (p->bc[2 * d + 1] == ORC_PERIODIC))
      return 0;
    /* a sweep needs NG interior cells to wrap or mirror from */
    if (p->n[d] > 1 && p->n[d] < NG) return 0;
  }
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0 && p->cfl <= 1.0)) return 0;
  return 1;
}

static void set_threads(const orc_params *p) {
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#else
  (void)p;
#endif
}

/* Non-positive density or pressure, or a non-finite value, anywhere in the
 * interior. */
static int state_bad(grid *g, double gamma) {
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        const double *c = g->u + cell_index(g, i, j, k);
        double W[NV];
        oracle_prim(c, gamma, W);
        if (!(W[0] > 0.0) || !(W[4] > 0.0)) return 1;
        for (int v = 0; v < NV; ++v)
          if (!isfinite(c[v])) return 1;
      }
  return 0;
}

static double grid_cfl_dt(grid *g, const orc_params *p) {
  double smax = 0.0;
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        const double *c = g->u + cell_index(g, i, j, k);
        double W[NV];
        oracle_prim(c, p->gamma, W);
        double cs = sqrt(p->gamma * W[4] / W[0]);
        for (int d = 0; d < 3; ++d) {
          if (g->n[d] == 1) continue;
          double s = (fabs(W[1 + d]) + cs) / p->dx[d];
          if (s > smax) smax = s;
        }
      }
  return p->cfl / smax;
}

/* One Strang step in place on a grid. */
static long grid_step(grid *g, const orc_params *p, double dt, int64_t step) {
  static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
  const int *order = (step % 2 == 0) ? even : odd;
  long fallbacks = 0;
  for (int s = 0; s < 3; ++s) {
    int d = order[s];
    if (g->n[d] == 1) continue;
    fallbacks += sweep_axis(g, d, p, dt, NULL);
  }
  return fallbacks;
}

/* ------------------------------------------------------------------ */
/* Exported entry points (state as 5 planes of nz*ny*nx doubles)       */
/* ------------------------------------------------------------------ */

/* dt = cfl / max over interior cells and active axes of (|v_d|+c)/dx_d */
int oracle_cfl_dt(const orc_params *p, const double *planes, double *dt) {
  if (!params_ok(p)) return ORC_EINVAL;
  grid g;
  if (grid_alloc(&g, p->n)) return ORC_ENOMEM;
  grid_load(&g, planes);
  *dt = grid_cfl_dt(&g, p);
  grid_free(&g);
  return isfinite(*dt) && *dt > 0.0 ? ORC_OK : ORC_ENUMERIC;
}

/* One Strang step with a given dt; step parity chooses the sweep order. */
int oracle_step(const orc_params *p, double *planes, double dt, int64_t step,
                long *fallbacks) {
  if (!params_ok(p) || !(dt >= 0.0)) return ORC_EINVAL;
  set_threads(p);
  grid g;
  if (grid_alloc(&g, p->n)) return ORC_ENOMEM;
  grid_load(&g, planes);
  long fb = grid_step(&g, p, dt, step);
  if (fallbacks) *fallbacks = fb;
  int bad = state_bad(&g, p->gamma);
  grid_store(&g, planes);
  grid_free(&g);
  return bad ? ORC_ENUMERIC : ORC_OK;
}

/* A single directional sweep (axis d) with a given dt. */
int oracle_sweep(const orc_params *p, double *planes, double dt, int d,
                 long *fallbacks) {
  if (!params_ok(p) || d < 0 || d > 2 || !(dt >= 0.0)) return ORC_EINVAL;
  set_threads(p);
  grid g;
  if (grid_alloc(&g, p->n)) return ORC_ENOMEM;
  grid_load(&g, planes);
  long fb = g.n[d] > 1 ? sweep_axis(&g, d, p, dt, NULL) : 0;
  if (fallbacks) *fallbacks = fb;
  grid_store(&g, planes);
  grid_free(&g);
  return ORC_OK;
}

/* A single sweep like oracle_sweep that also returns the face fluxes it
 * applied (layout of sweep_axis' fout; the axis needs more than one cell).
 * Refinement operators use them to make coarse and fine levels agree on the
 * flux through a coarse-fine face. */
int oracle_sweep_flux(const orc_params *p, double *planes, double dt, int d,
                      double *flux, long *fallbacks) {
  if (!params_ok(p) || d < 0 || d > 2 || !(dt >= 0.0) || !flux || p->n[d] < 2)
    return ORC_EINVAL;
  set_threads(p);
  grid g;
  if (grid_alloc(&g, p->n)) return ORC_ENOMEM;
  grid_load(&g, planes);
  long fb = sweep_axis(&g, d, p, dt, flux);
  if (fallbacks) *fallbacks = fb;
  grid_store(&g, planes);
  grid_free(&g);
  return ORC_OK;
}

/* Run steps with the CFL dt, starting at time *t and step counter *step,
 * until nsteps steps are done or t reaches t_end (t_end <= 0: no limit).
 * The last step is shortened to land on t_end exactly. */
int oracle_run(const orc_params *p, double *planes, int64_t nsteps,
               double t_end, double *t, int64_t *step, long *fallbacks) {
  if (!params_ok(p)) return ORC_EINVAL;
  set_threads(p);
  grid g;
  if (grid_alloc(&g, p->n)) return ORC_ENOMEM;
  grid_load(&g, planes);
  long fb = 0;
  int rc = ORC_OK;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (t_end > 0.0 && *t >= t_end) break;
    double dt = grid_cfl_dt(&g, p);
    if (!(dt > 0.0) || !isfinite(dt)) {
      rc = ORC_ENUMERIC;
      break;
    }
    if (t_end > 0.0 && dt > t_end - *t) dt = t_end - *t;
    fb += grid_step(&g, p, dt, *step);
    *t += dt;
    *step += 1;
    if (state_bad(&g, p->gamma)) {
      rc = ORC_ENUMERIC;
      break;
    }
  }
  if (fallbacks) *fallbacks = fb;
  grid_store(&g, planes);
  grid_free(&g);
  return rc;
}

/* Neumaier compensated sum helper. */
typedef struct {
  double s, c;
} ksum;

static void ksum_add(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}

/* Conserved totals times the cell volume: rho, mx, my, mz, E and
 * E + rho*phi with phi = -(g . x) at cell centres (origin at the low
 * corner). */
int oracle_totals(const orc_params *p, const double *planes, double out[6]) {
  if (!params_ok(p)) return ORC_EINVAL;
  const double vol = p->dx[0] * p->dx[1] * p->dx[2];
  const size_t plane = (size_t)p->n[0] * p->n[1] * p->n[2];
  ksum acc[6];
  memset(acc, 0, sizeof(acc));
  for (int k = 0; k < p->n[2]; ++k)
    for (int j = 0; j < p->n[1]; ++j)
      for (int i = 0; i < p->n[0]; ++i) {
        size_t q = ((size_t)k * p->n[1] + j) * p->n[0] + i;
        double x = (i + 0.5) * p->dx[0];
        double y = (j + 0.5) * p->dx[1];
        double z = (k + 0.5) * p->dx[2];
        double phi = -(p->grav[0] * x + p->grav[1] * y + p->grav[2] * z);
        for (int v = 0; v < NV; ++v) ksum_add(&acc[v], planes[v * plane + q] * vol);
        ksum_add(&acc[5], (planes[4 * plane + q] + planes[q] * phi) * vol);
      }
  for (int v = 0; v < 6; ++v) out[v] = acc[v].s + acc[v].c;
  return ORC_OK;
}

/* Exposed pieces for unit pins. */
void oracle_hancock(const double W[NV], const double D[NV], double dtdx,
                    double gamma, double half_dt_g, int has_g, double Wm[NV],
                    double Wp[NV]) {
  hancock(W, D, dtdx, gamma, half_dt_g, has_g, Wm, Wp);
}

int oracle_abi_version(void) { return 1; }
