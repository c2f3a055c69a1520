/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the finite-volume step of
 * "diffhydro" (Horowitz, Lukic, Nagamine & Oku, arXiv 2512.13403).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load liboracle.so.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (one time step, paper App. A):
 *   1. dt from the CFL condition (App. A.4), or a fixed dt;
 *   2. the semi-discrete operator L(U) of the unsplit method of lines
 *      (App. A.3, the rhs equation): MUSCL reconstruction on primitive
 *      variables with a slope limiter (App. A.1), HLLC fluxes with Davis wave
 *      speeds (App. A.2), conservative differencing per axis;
 *   3. the explicit Runge-Kutta update (App. A.3): the two-stage RK2 (Heun /
 *      SSP-RK2, the default), the three-stage SSPRK3, or forward Euler;
 *   4. operator-split sources on the result, in the order forcing -> gravity
 *      -> cooling: OU forcing (Sec. 3.1.1), multigrid self-gravity (Sec. 6.2,
 *      in oracle_mg.c), optically thin cooling integrated exactly per cell
 *      (Sec. 4 with the synthetic cooling curve described at or_cool_cell).
 *
 * Layout: U is [5][nz][ny][nx] (x fastest), fields (rho, m_x, m_y, m_z, E),
 * as the state vector u[0]=rho, u[1]=m_x, ..., u[-1]=E of the Sec. 2.1
 * listing.  Everything is double precision.
 *
 * The loops are written pencil by pencil so that each line can be checked
 * against the equations by eye; speed is not a goal.  OpenMP only splits
 * independent pencils; every reduction is done in a fixed order so results do
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------------- */
/* indexing and boundaries                                                    */
/* ------------------------------------------------------------------------- */

static inline long or_cells(const or_config *c) {
  return (long)c->n[0] * c->n[1] * c->n[2];
}

static inline long or_idx(const or_config *c, long i, long j, long k) {
  return (k * c->n[1] + j) * c->n[0] + i;
}

/* Ghost-cell rule.  Periodic: wrap (the roll of the App. A.3 rhs equation).
 * Outflow: zero-gradient copy of the edge cell (not in the paper; used by the
 * Sod tube, whose x ends are transmissive). */
static inline long or_bc(long i, long n, int bc) {
  if (bc == OR_BC_PERIODIC) {
    long r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* ------------------------------------------------------------------------- */
/* equation of state (Sec. 3, the definition of U and P)                      */
/* ------------------------------------------------------------------------- */

/* conserved (rho, m, E) -> primitive (rho, v, P) with
 * P = (gamma - 1) (E - rho |v|^2 / 2). */
static void cons_to_prim(const double u[5], double gamma, double w[5]) {
  double rho = u[0];
  double vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
  w[0] = rho;
  w[1] = vx;
  w[2] = vy;
  w[3] = vz;
  w[4] = (gamma - 1.0) * (u[4] - 0.5 * rho * (vx * vx + vy * vy + vz * vz));
}

void or_primitives(const or_config *c, const double *U, double *W) {
  long N = or_cells(c);
#pragma omp parallel for schedule(static)
  for (long q = 0; q < N; ++q) {
    double u[5], w[5];
    for (int f = 0; f < 5; ++f) u[f] = U[f * N + q];
    cons_to_prim(u, c->gamma, w);
    for (int f = 0; f < 5; ++f) W[f * N + q] = w[f];
  }
}

/* ------------------------------------------------------------------------- */
/* CFL time step (App. A.4)                                                   */
/* ------------------------------------------------------------------------- */

/* dt = C * min over cells and axes of dx_a / (|v_a| + c_s), written as
 * C / max_cells max_a (|v_a| + c_s) / dx_a.  c_s^2 = gamma P / rho (App. A.2). */
double or_cfl_dt(const or_config *c, const double *U) {
  long N = or_cells(c);
  double smax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : smax)
  for (long q = 0; q < N; ++q) {
    double u[5], w[5];
    for (int f = 0; f < 5; ++f) u[f] = U[f * N + q];
    cons_to_prim(u, c->gamma, w);
    double cs = sqrt(c->gamma * w[4] / w[0]);
    for (int a = 0; a < 3; ++a) {
      double s = (fabs(w[1 + a]) + cs) / c->h[a];
      if (s > smax) smax = s;
    }
  }
  double dt = c->cfl / smax;
  /* the cooling-time limit of Sec. 4.3 (oracle_cool.c), when c_cool > 0 */
  if ((c->flags & OR_SRC_COOLING) && c->cool_ccool > 0.0) {
    double dc = or_cool_dt_limit(c, U);
    if (dc < dt) dt = dc;
  }
  return dt;
}

/* ------------------------------------------------------------------------- */
/* slope limiters (App. A.1)                                                  */
/* ------------------------------------------------------------------------- */

/* minmod(a, b): the argument of smaller magnitude when both have the same
 * sign, else 0.  A tie |a| = |b| takes a. */
static double lim_minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) <= fabs(b) ? a : b;
}

/* van Leer (harmonic mean): 2ab/(a+b) when ab > 0, else 0. */
static double lim_vanleer(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return 2.0 * a * b / (a + b);
}

/* monotonised central: minmod(2 minmod-compatible bounds, central). */
static double lim_mc(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double cen = 0.5 * (a + b);
  double m = fmin(fabs(cen), fmin(2.0 * fabs(a), 2.0 * fabs(b)));
  return a > 0.0 ? m : -m;
}

/* superbee: maxmod(minmod(2a, b), minmod(a, 2b)). */
static double lim_superbee(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double s1 = fmin(2.0 * fabs(a), fabs(b));
  double s2 = fmin(fabs(a), 2.0 * fabs(b));
  double m = fmax(s1, s2);
  return a > 0.0 ? m : -m;
}

/* Delta W_i = limiter(W_{i+1} - W_i, W_i - W_{i-1})  (App. A.1).
 * OR_LIM_NONE is the piecewise-constant reconstruction (slope 0). */
static double limited_slope(int limiter, double wm, double w0, double wp) {
  double a = wp - w0, b = w0 - wm;
  switch (limiter) {
    case OR_LIM_MINMOD: return lim_minmod(a, b);
    case OR_LIM_VANLEER: return lim_vanleer(a, b);
    case OR_LIM_MC: return lim_mc(a, b);
    case OR_LIM_SUPERBEE: return lim_superbee(a, b);
    default: return 0.0;
  }
}

/* ------------------------------------------------------------------------- */
/* HLLC approximate Riemann solver (App. A.2)                                 */
/* ------------------------------------------------------------------------- */

/* States are given in a frame aligned with the face normal:
 * w = (rho, v_n, v_t1, v_t2, P); the flux comes back in the same frame
 * (mass, normal momentum, two tangential momenta, energy).
 *
 * Wave speeds: S_L = min(v_L - c_L, v_R - c_R), S_R = max(v_L + c_L, v_R + c_R)
 * (App. A.2).  The contact speed, star states and four-region selection are
 * the standard HLLC construction (Toro, Riemann Solvers and Numerical Methods
 * for Fluid Dynamics, 3rd ed., Sec. 10.4), which the paper names but does not
 * print. */
static void flux_of(const double w[5], double gamma, double U[5], double F[5]) {
  double rho = w[0], vn = w[1], t1 = w[2], t2 = w[3], p = w[4];
  double E = p / (gamma - 1.0) + 0.5 * rho * (vn * vn + t1 * t1 + t2 * t2);
  U[0] = rho;
  U[1] = rho * vn;
  U[2] = rho * t1;
  U[3] = rho * t2;
  U[4] = E;
  F[0] = rho * vn;
  F[1] = rho * vn * vn + p;
  F[2] = rho * vn * t1;
  F[3] = rho * vn * t2;
  F[4] = vn * (E + p);
}

static void star_state(const double w[5], const double U[5], double S,
                       double sstar, double Us[5]) {
  double rho = w[0], vn = w[1], p = w[4];
  double fac = rho * (S - vn) / (S - sstar);
  Us[0] = fac;
  Us[1] = fac * sstar;
  Us[2] = fac * w[2];
  Us[3] = fac * w[3];
  Us[4] = fac * (U[4] / rho + (sstar - vn) * (sstar + p / (rho * (S - vn))));
}

static void riemann_hllc(const double wl[5], const double wr[5], double gamma,
                         double F[5]) {
  double UL[5], FL[5], UR[5], FR[5];
  flux_of(wl, gamma, UL, FL);
  flux_of(wr, gamma, UR, FR);
  double cl = sqrt(gamma * wl[4] / wl[0]);
  double cr = sqrt(gamma * wr[4] / wr[0]);
  double SL = fmin(wl[1] - cl, wr[1] - cr);
  double SR = fmax(wl[1] + cl, wr[1] + cr);
  double num = wr[4] - wl[4] + wl[0] * wl[1] * (SL - wl[1]) -
               wr[0] * wr[1] * (SR - wr[1]);
  double den = wl[0] * (SL - wl[1]) - wr[0] * (SR - wr[1]);
  double sstar = num / den;
  if (0.0 <= SL) {
    for (int f = 0; f < 5; ++f) F[f] = FL[f];
  } else if (0.0 <= sstar) {
    double Us[5];
    star_state(wl, UL, SL, sstar, Us);
    for (int f = 0; f < 5; ++f) F[f] = FL[f] + SL * (Us[f] - UL[f]);
  } else if (0.0 < SR) {
    double Us[5];
    star_state(wr, UR, SR, sstar, Us);
    for (int f = 0; f < 5; ++f) F[f] = FR[f] + SR * (Us[f] - UR[f]);
  } else {
    for (int f = 0; f < 5; ++f) F[f] = FR[f];
  }
}

/* HLL (two-wave) flux with the same Davis speeds (App. A.2, alternatives). */
static void riemann_hll(const double wl[5], const double wr[5], double gamma,
                        double F[5]) {
  double UL[5], FL[5], UR[5], FR[5];
  flux_of(wl, gamma, UL, FL);
  flux_of(wr, gamma, UR, FR);
  double cl = sqrt(gamma * wl[4] / wl[0]);
  double cr = sqrt(gamma * wr[4] / wr[0]);
  double SL = fmin(wl[1] - cl, wr[1] - cr);
  double SR = fmax(wl[1] + cl, wr[1] + cr);
  if (0.0 <= SL) {
    for (int f = 0; f < 5; ++f) F[f] = FL[f];
  } else if (SR <= 0.0) {
    for (int f = 0; f < 5; ++f) F[f] = FR[f];
  } else {
    for (int f = 0; f < 5; ++f)
      F[f] = (SR * FL[f] - SL * FR[f] + SL * SR * (UR[f] - UL[f])) / (SR - SL);
  }
}

/* Rusanov (local Lax-Friedrichs) flux (App. A.2, alternatives). */
static void riemann_rusanov(const double wl[5], const double wr[5], double gamma,
                            double F[5]) {
  double UL[5], FL[5], UR[5], FR[5];
  flux_of(wl, gamma, UL, FL);
  flux_of(wr, gamma, UR, FR);
  double cl = sqrt(gamma * wl[4] / wl[0]);
  double cr = sqrt(gamma * wr[4] / wr[0]);
  double smax = fmax(fabs(wl[1]) + cl, fabs(wr[1]) + cr);
  for (int f = 0; f < 5; ++f)
    F[f] = 0.5 * (FL[f] + FR[f]) - 0.5 * smax * (UR[f] - UL[f]);
}

static void riemann(int solver, const double wl[5], const double wr[5],
                    double gamma, double F[5]) {
  if (solver == OR_RS_HLL)
    riemann_hll(wl, wr, gamma, F);
  else if (solver == OR_RS_RUSANOV)
    riemann_rusanov(wl, wr, gamma, F);
  else
    riemann_hllc(wl, wr, gamma, F);
}

/* ------------------------------------------------------------------------- */
/* the semi-discrete operator L(U)  (App. A.3, the rhs equation)             */
/* ------------------------------------------------------------------------- */

/* L(U)_i = - sum_a (F_{a,i+1/2} - F_{a,i-1/2}) / dx_a, accumulated over x,
 * then y, then z.  For each pencil along axis a the primitive variables are
 * gathered with two ghost cells per side, limited slopes are formed for every
 * cell that touches a face (App. A.1), left/right face states are
 * W^L_{i+1/2} = W_i + Delta W_i / 2 and W^R_{i+1/2} = W_{i+1} - Delta W_{i+1}/2,
 * and the Riemann flux of every one of the n+1 faces is differenced. */
void or_rhs(const or_config *c, const double *U, double *L) {
  long N = or_cells(c);
  double *W = (double *)malloc(sizeof(double) * 5 * N);
  or_primitives(c, U, W);
  memset(L, 0, sizeof(double) * 5 * N);

  for (int a = 0; a < 3; ++a) {
    long n = c->n[a];
    int b1 = (a + 1) % 3, b2 = (a + 2) % 3; /* the two other axes */
    long npencil = (long)c->n[b1] * c->n[b2];
    double inv_h = 1.0 / c->h[a];
    /* velocity component indices in the face frame: normal, t1, t2 */
    int vn = 1 + a, vt1 = 1 + b1, vt2 = 1 + b2;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npencil; ++p) {
      long j1 = p % c->n[b1], j2 = p / c->n[b1];
      /* gathered primitives in the face frame, cells -2 .. n+1 */
      double (*wg)[5] = malloc(sizeof(double[5]) * (n + 4));
      double (*slope)[5] = malloc(sizeof(double[5]) * (n + 2));
      double (*flux)[5] = malloc(sizeof(double[5]) * (n + 1));
      long cellq[3];
      for (long i = -2; i < n + 2; ++i) {
        cellq[a] = or_bc(i, n, c->bc[a]);
        cellq[b1] = j1;
        cellq[b2] = j2;
        long q = or_idx(c, cellq[0], cellq[1], cellq[2]);
        wg[i + 2][0] = W[0 * N + q];
        wg[i + 2][1] = W[vn * N + q];
        wg[i + 2][2] = W[vt1 * N + q];
        wg[i + 2][3] = W[vt2 * N + q];
        wg[i + 2][4] = W[4 * N + q];
      }
      /* slopes for cells -1 .. n */
      for (long i = -1; i <= n; ++i)
        for (int f = 0; f < 5; ++f)
          slope[i + 1][f] = limited_slope(c->limiter, wg[i + 1][f],
                                          wg[i + 2][f], wg[i + 3][f]);
      /* face f sits between cells f-1 and f, for f = 0 .. n */
      for (long fidx = 0; fidx <= n; ++fidx) {
        double wl[5], wr[5];
        for (int f = 0; f < 5; ++f) {
          wl[f] = wg[fidx + 1][f] + 0.5 * slope[fidx][f];     /* cell fidx-1 */
          wr[f] = wg[fidx + 2][f] - 0.5 * slope[fidx + 1][f]; /* cell fidx */
        }
        double fr[5];
        riemann(c->riemann, wl, wr, c->gamma, fr);
        flux[fidx][0] = fr[0];
        flux[fidx][vn] = fr[1];
        flux[fidx][vt1] = fr[2];
        flux[fidx][vt2] = fr[3];
        flux[fidx][4] = fr[4];
        if (c->flux_corr) {
          /* the face between cells fidx-1 and fidx is the +a face of cell
           * fidx-1 (boundary-mapped for the face below the first cell) */
          cellq[a] = or_bc(fidx - 1, n, c->bc[a]);
          cellq[b1] = j1;
          cellq[b2] = j2;
          long qc = or_idx(c, cellq[0], cellq[1], cellq[2]);
          for (int f = 0; f < 5; ++f) flux[fidx][f] += c->flux_corr[f * N + qc];
        }
      }
      for (long i = 0; i < n; ++i) {
        cellq[a] = i;
        cellq[b1] = j1;
        cellq[b2] = j2;
        long q = or_idx(c, cellq[0], cellq[1], cellq[2]);
        for (int f = 0; f < 5; ++f)
          L[f * N + q] -= (flux[i + 1][f] - flux[i][f]) * inv_h;
      }
      free(wg);
      free(slope);
      free(flux);
    }
  }
  free(W);
}

/* ------------------------------------------------------------------------- */
/* RK2 (Heun = SSP-RK2) in Shu-Osher form (App. A.3)                          */
/* ------------------------------------------------------------------------- */

/* U1 = U + dt L(U);  U_new = U/2 + (U1 + dt L(U1))/2. */
void or_rk2(const or_config *c, double *U, double dt) {
  long N5 = 5 * or_cells(c);
  double *L = (double *)malloc(sizeof(double) * N5);
  double *U1 = (double *)malloc(sizeof(double) * N5);
  or_rhs(c, U, L);
  for (long q = 0; q < N5; ++q) U1[q] = U[q] + dt * L[q];
  or_rhs(c, U1, L);
  for (long q = 0; q < N5; ++q) U[q] = 0.5 * U[q] + 0.5 * (U1[q] + dt * L[q]);
  free(L);
  free(U1);
}

/* forward Euler, U_new = U + dt L(U) (App. A.3, the first-order option kept
 * for testing) */
void or_euler(const or_config *c, double *U, double dt) {
  long N5 = 5 * or_cells(c);
  double *L = (double *)malloc(sizeof(double) * N5);
  or_rhs(c, U, L);
  for (long q = 0; q < N5; ++q) U[q] = U[q] + dt * L[q];
  free(L);
}

/* SSPRK3 (App. A.3, third item), the three-stage strong-stability-preserving
 * scheme of Shu & Osher in its convex form:
 *   U1 = U + dt L(U)
 *   U2 = 3/4 U + 1/4 (U1 + dt L(U1))
 *   U_new = 1/3 U + 2/3 (U2 + dt L(U2)) */
void or_ssprk3(const or_config *c, double *U, double dt) {
  long N5 = 5 * or_cells(c);
  double *L = (double *)malloc(sizeof(double) * N5);
  double *U1 = (double *)malloc(sizeof(double) * N5);
  double *U2 = (double *)malloc(sizeof(double) * N5);
  or_rhs(c, U, L);
  for (long q = 0; q < N5; ++q) U1[q] = U[q] + dt * L[q];
  or_rhs(c, U1, L);
  for (long q = 0; q < N5; ++q) U2[q] = 0.75 * U[q] + 0.25 * (U1[q] + dt * L[q]);
  or_rhs(c, U2, L);
  for (long q = 0; q < N5; ++q) U[q] = U[q] / 3.0 + 2.0 / 3.0 * (U2[q] + dt * L[q]);
  free(L);
  free(U1);
  free(U2);
}

/* the integrator the configuration names */
void or_integrate(const or_config *c, double *U, double dt) {
  if (c->integrator == OR_RK_SSP3) or_ssprk3(c, U, dt);
  else if (c->integrator == OR_RK_EULER) or_euler(c, U, dt);
  else or_rk2(c, U, dt);
}

/* ------------------------------------------------------------------------- */
/* optically thin cooling, integrated exactly per cell (Sec. 4)               */
/* ------------------------------------------------------------------------- */

/* The paper writes the operator-split energy equation dE/dt = ... - n^2 Lambda
 * and T proportional to P/rho (Sec. 4, the energy and EOS equations).  In code
 * units n = rho and T = P/rho, so at fixed rho and momentum
 *     dT/dt = -(gamma - 1) rho Lambda(T).
 * The cooling curve is the synthetic two-branch one used for the driven
 * turbulence workload (the paper's tabulated curve is not available):
 *     Lambda = L0 (T/Tc)^(1/2)           for T >= Tc,
 *     Lambda = L0 exp((T - Tc)/Ts)       for T <  Tc,
 * which has closed-form solutions on both branches: above Tc, sqrt(T) falls
 * linearly in time; below Tc, exp(-(T - Tc)/Ts) rises linearly in time.  The
 * result is floored at T_floor (the temperature floor of Sec. 4.3). */
double or_cool_temperature(double rho, double T, double dt, double gamma,
                           double L0, double Tc, double Ts, double Tfloor) {
  double Tn;
  double k2 = (gamma - 1.0) * rho * L0 / Ts; /* rate of exp(-(T-Tc)/Ts) */
  if (T >= Tc) {
    double k1 = (gamma - 1.0) * rho * L0 / (2.0 * sqrt(Tc)); /* rate of sqrt T */
    double t1 = (sqrt(T) - sqrt(Tc)) / k1; /* time to reach Tc */
    if (dt <= t1) {
      double s = sqrt(T) - k1 * dt;
      Tn = s * s;
    } else {
      Tn = Tc - Ts * log(1.0 + k2 * (dt - t1));
    }
  } else {
    Tn = Tc - Ts * log(exp(-(T - Tc) / Ts) + k2 * dt);
  }
  return fmax(Tn, Tfloor);
}

void or_cool(const or_config *c, double *U, double dt) {
  long N = or_cells(c);
  double g = c->gamma;
#pragma omp parallel for schedule(static)
  for (long q = 0; q < N; ++q) {
    double rho = U[q];
    double ek = 0.5 * (U[N + q] * U[N + q] + U[2 * N + q] * U[2 * N + q] +
                       U[3 * N + q] * U[3 * N + q]) / rho;
    if (c->cool_model == OR_COOL_TABLE) {
      /* the paper's tabulated model and integrators (oracle_cool.c) */
      U[4 * N + q] = ek + or_cool_eth_step(c, rho, U[4 * N + q] - ek, dt);
      continue;
    }
    double T = (g - 1.0) * (U[4 * N + q] - ek) / rho;
    double Tn = or_cool_temperature(rho, T, dt, g, c->cool_lambda0, c->cool_tc,
                                    c->cool_ts, c->cool_tfloor);
    U[4 * N + q] = ek + rho * Tn / (g - 1.0);
  }
}

/* ------------------------------------------------------------------------- */
/* Ornstein-Uhlenbeck forcing (Sec. 3.1.1)                                    */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the c-th output of the
 * generator seeded with `seed` is mix(seed + (c+1) * golden). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* complex Gaussian with Re, Im ~ N(0, 1/2) for draw number d of group g,
 * by the Box-Muller transform of two 53-bit uniforms */
void or_ou_gauss(uint64_t seed, int64_t group, int mode, int comp,
                 double out[2]) {
  uint64_t d = ((uint64_t)(group + 1) * OR_OU_MAXMODES + (uint64_t)mode) * 3u +
               (uint64_t)comp;
  uint64_t x1 = splitmix64_at(seed, 2 * d), x2 = splitmix64_at(seed, 2 * d + 1);
  double u1 = (double)((x1 >> 11) + 1) * 0x1.0p-53; /* (0, 1] */
  double u2 = (double)(x2 >> 11) * 0x1.0p-53;       /* [0, 1) */
  double r = sqrt(-2.0 * log(u1));
  double th = 2.0 * M_PI * u2;
  out[0] = r * cos(th) * sqrt(0.5);
  out[1] = r * sin(th) * sqrt(0.5);
}

/* The forced modes: integer n with kmin <= |n| <= kmax, one of each +-n pair
 * (the first non-zero component positive), in lexicographic (nx, ny, nz)
 * order.  k = 0 is excluded (Sec. 3.1.1).  Returns the count. */
int or_ou_modes(double kmin, double kmax, int32_t *nvec) {
  int m = 0, r = (int)ceil(kmax);
  for (int a = -r; a <= r; ++a)
    for (int b = -r; b <= r; ++b)
      for (int d = -r; d <= r; ++d) {
        double k = sqrt((double)(a * a + b * b + d * d));
        if (k < kmin || k > kmax || k == 0.0) continue;
        int first = a != 0 ? a : (b != 0 ? b : d);
        if (first <= 0) continue;
        if (m >= OR_OU_MAXMODES) return -1;
        nvec[3 * m] = a;
        nvec[3 * m + 1] = b;
        nvec[3 * m + 2] = d;
        ++m;
      }
  return m;
}

/* projected noise M eta with M = zeta P + (1 - zeta) C, P the solenoidal and
 * C the compressive projector (Sec. 3.1, eq:turbproj) */
static void ou_projected_noise(const or_config *c, int64_t group, int mode,
                               const int32_t n[3], double out[3][2]) {
  double eta[3][2];
  for (int comp = 0; comp < 3; ++comp)
    or_ou_gauss(c->ou_seed, group, mode, comp, eta[comp]);
  double k2 = (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double z = c->ou_zeta;
  for (int i = 0; i < 3; ++i)
    for (int ri = 0; ri < 2; ++ri) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) {
        double Cij = (double)n[i] * n[j] / k2;
        double Pij = (i == j ? 1.0 : 0.0) - Cij;
        s += (z * Pij + (1.0 - z) * Cij) * eta[j][ri];
      }
      out[i][ri] = s;
    }
}

/* State layout: ahat[m][comp][re/im], 6 doubles per mode. */
void or_ou_init(const or_config *c, int nmodes, const int32_t *nvec,
                double *ahat) {
  for (int m = 0; m < nmodes; ++m) {
    double pe[3][2];
    ou_projected_noise(c, -1, m, nvec + 3 * m, pe);
    for (int i = 0; i < 3; ++i) {
      ahat[6 * m + 2 * i] = pe[i][0];
      ahat[6 * m + 2 * i + 1] = pe[i][1];
    }
  }
}

/* a(t + dt) = exp(-dt/tau) a(t) + sqrt(1 - exp(-2 dt/tau)) eta  (Sec. 3.1.1) */
void or_ou_advance(const or_config *c, int nmodes, const int32_t *nvec,
                   double *ahat, int64_t group, double dt) {
  double f = exp(-dt / c->ou_tau);
  double g = sqrt(1.0 - exp(-2.0 * dt / c->ou_tau));
  for (int m = 0; m < nmodes; ++m) {
    double pe[3][2];
    ou_projected_noise(c, group, m, nvec + 3 * m, pe);
    for (int i = 0; i < 3; ++i) {
      ahat[6 * m + 2 * i] = f * ahat[6 * m + 2 * i] + g * pe[i][0];
      ahat[6 * m + 2 * i + 1] = f * ahat[6 * m + 2 * i + 1] + g * pe[i][1];
    }
  }
}

/* a_rms / sqrt(<|a|^2>), with <|a|^2> = 2 sum_m |ahat_m|^2 by Parseval for
 * a(x) = sum_m 2 Re(ahat_m exp(2 pi i n_m . x / L)) (Sec. 3.1.1, the rms
 * normalisation) */
double or_ou_scale(const or_config *c, int nmodes, const double *ahat) {
  double s = 0.0;
  for (int q = 0; q < 6 * nmodes; ++q) s += ahat[q] * ahat[q];
  return c->ou_arms / sqrt(2.0 * s);
}

/* real-space acceleration at the centre of cell (i, j, k), x_a = (i_a + 1/2) L_a / n_a:
 * a(x) = s sum_m 2 Re(ahat_m exp(2 pi i n_m . x / L)) */
void or_ou_accel_at(const or_config *c, int nmodes, const int32_t *nvec,
                    const double *ahat, long i, long j, long k, double out[3]) {
  double s = or_ou_scale(c, nmodes, ahat);
  double a[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < nmodes; ++m) {
    const int32_t *n = nvec + 3 * m;
    double th = 2.0 * M_PI *
                (n[0] * (i + 0.5) / c->n[0] + n[1] * (j + 0.5) / c->n[1] +
                 n[2] * (k + 0.5) / c->n[2]);
    double cr = cos(th), ci = sin(th);
    for (int comp = 0; comp < 3; ++comp)
      a[comp] += 2.0 * (ahat[6 * m + 2 * comp] * cr - ahat[6 * m + 2 * comp + 1] * ci);
  }
  for (int comp = 0; comp < 3; ++comp) out[comp] = s * a[comp];
}

void or_ou_accel(const or_config *c, int nmodes, const int32_t *nvec,
                 const double *ahat, double *acc /* [3][N] */) {
  long N = or_cells(c);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < c->n[2]; ++k)
    for (long j = 0; j < c->n[1]; ++j)
      for (long i = 0; i < c->n[0]; ++i) {
        double a[3];
        or_ou_accel_at(c, nmodes, nvec, ahat, i, j, k, a);
        long q = or_idx(c, i, j, k);
        for (int comp = 0; comp < 3; ++comp) acc[comp * N + q] = a[comp];
      }
}

/* the force-listing kick of Sec. 2.1 with the Sec. 3.1.1 coupling:
 * m += rho a dt, E += (m_old . a) dt */
void or_kick(const or_config *c, double *U, const double *acc, double dt) {
  long N = or_cells(c);
#pragma omp parallel for schedule(static)
  for (long q = 0; q < N; ++q) {
    double rho = U[q];
    double dE = 0.0;
    for (int comp = 0; comp < 3; ++comp) dE += U[(1 + comp) * N + q] * acc[comp * N + q];
    for (int comp = 0; comp < 3; ++comp) U[(1 + comp) * N + q] += rho * acc[comp * N + q] * dt;
    U[4 * N + q] += dE * dt;
  }
}

/* ------------------------------------------------------------------------- */
/* one full step                                                              */
/* ------------------------------------------------------------------------- */

/* Advances U by one step.  dt_fixed > 0 uses that dt, otherwise the CFL dt;
 * either is capped at dt_cap (pass +inf for none).  `step` is the global step
 * index (it keys the OU noise).  ou_ahat holds the OU mode state (advanced in
 * place), phi the gravitational potential (warm start in, solution out).
 * Returns the dt used. */
double or_step(const or_config *c, double *U, double dt_fixed, double dt_cap,
               int64_t step, int nmodes, const int32_t *nvec, double *ou_ahat,
               double *phi, int *mg_cycles) {
  double dt = dt_fixed > 0.0 ? dt_fixed : or_cfl_dt(c, U);
  if (dt > dt_cap) dt = dt_cap;
  or_integrate(c, U, dt);
  long N = or_cells(c);
  if ((c->flags & OR_SRC_FORCING) && nmodes > 0) {
    int every = c->ou_every > 0 ? c->ou_every : 1;
    if (step % every == 0)
      or_ou_advance(c, nmodes, nvec, ou_ahat, step / every, dt * every);
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    or_ou_accel(c, nmodes, nvec, ou_ahat, acc);
    or_kick(c, U, acc, dt);
    free(acc);
  }
  if (c->flags & OR_SRC_GRAVITY) {
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    int cyc = or_gravity_accel(c, U, phi, acc);
    if (mg_cycles) *mg_cycles = cyc;
    or_kick(c, U, acc, dt);
    free(acc);
  }
  if (c->flags & OR_SRC_COOLING) or_cool(c, U, dt);
  return dt;
}

/* threads the OpenMP loops above run on (reported with CPU timings) */
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
