/*
 * oracle_cool.c -- the paper's heating/cooling model and its integrators
 * (Sec. 4: the two-branch equilibrium prescription, its physical assumptions
 * and its numerical integration), for the tabulated-model option.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * Code units as for the exact two-branch model: n = rho, T = P/rho, so the
 * thermal energy density is E_th = rho T/(gamma - 1) and, at fixed rho and
 * momentum, dE_th/dt = rho Gamma(T) - rho^2 Lambda(T) (Sec. 4, the energy
 * equation with n = rho).
 *
 *   Lambda(T) = L1 T^a1 + L2 T^a2                  for T <  tc
 *             = 10^(log-log interpolation of the    for T >= tc
 *                   table (log10 T_i, log10 L_i))
 *   Gamma(T)  = Gamma_0 for T < tc, 0 above        (the two-branch model)
 *
 * The table's values are used flat beyond its first and last points.
 * Integrators for one operator-split step dt (Sec. 4.3):
 *   trapezoid  E* = E + dt Edot(E),  E' = E + dt/2 (Edot(E) + Edot(E*));
 *   subcycled  N = ceil(dt |Edot(E)| / (f E)) substeps (1 <= N <= N_max)
 *              of dt/N, each E <- max(E_floor, E + clamp(Edot(E) dt/N,
 *              -f E, f E)) (the largest fractional change per substep f);
 *   auto       trapezoid when dt |Edot(E)| <= f E, else subcycled.
 * Every intermediate and final E_th is floored at E_floor = rho T_floor /
 * (gamma - 1), and so is the incoming one.  The step limit (Sec. 4.3) is
 *   dt <= c_cool min over cells of t_cool,  t_cool = E_th / |Edot|.
 */
#include <math.h>

#include "oracle.h"

double or_cool_lambda(const or_config *c, double T) {
  if (T < c->cool_tc) return c->cool_L1 * pow(T, c->cool_a1) + c->cool_L2 * pow(T, c->cool_a2);
  int n = c->cool_ntab;
  double x = log10(T);
  if (x <= c->cool_logT[0]) return pow(10.0, c->cool_logL[0]);
  if (x >= c->cool_logT[n - 1]) return pow(10.0, c->cool_logL[n - 1]);
  int i = 0;
  /* logT[i] <= x < logT[i+1]; the bound (never reached by a finite x inside
     the table) keeps a NaN temperature from reading past the table */
  while (i < n - 2 && !(x < c->cool_logT[i + 1])) ++i;
  double w = (x - c->cool_logT[i]) / (c->cool_logT[i + 1] - c->cool_logT[i]);
  return pow(10.0, c->cool_logL[i] + w * (c->cool_logL[i + 1] - c->cool_logL[i]));
}

/* dE_th/dt at density rho and thermal energy density Eth */
double or_cool_edot(const or_config *c, double rho, double Eth) {
  double T = (c->gamma - 1.0) * Eth / rho;
  double heat = T < c->cool_tc ? c->cool_heat : 0.0;
  return rho * heat - rho * rho * or_cool_lambda(c, T);
}

static double floor_eth(const or_config *c, double rho, double E) {
  double Ef = rho * c->cool_tfloor / (c->gamma - 1.0);
  return E > Ef ? E : Ef;
}

static double trapezoid(const or_config *c, double rho, double E, double dt) {
  double d0 = or_cool_edot(c, rho, E);
  double Ep = floor_eth(c, rho, E + dt * d0);
  double d1 = or_cool_edot(c, rho, Ep);
  return floor_eth(c, rho, E + 0.5 * dt * (d0 + d1));
}

static double subcycled(const or_config *c, double rho, double E, double dt) {
  double f = c->cool_frac;
  double d0 = or_cool_edot(c, rho, E);
  double nd = ceil(dt * fabs(d0) / (f * E));
  long N = !(nd >= 1.0) ? 1 : (nd > (double)c->cool_nsub_max ? c->cool_nsub_max : (long)nd);
  double h = dt / (double)N;
  for (long k = 0; k < N; ++k) {
    double dE = or_cool_edot(c, rho, E) * h;
    double lim = f * E;
    if (dE > lim) dE = lim;
    if (dE < -lim) dE = -lim;
    E = floor_eth(c, rho, E + dE);
  }
  return E;
}

double or_cool_eth_step(const or_config *c, double rho, double Eth, double dt) {
  double E = floor_eth(c, rho, Eth);
  int m = c->cool_integrator;
  if (m == OR_COOLINT_AUTO)
    m = dt * fabs(or_cool_edot(c, rho, E)) <= c->cool_frac * E ? OR_COOLINT_TRAPEZOID
                                                               : OR_COOLINT_SUBCYCLE;
  return m == OR_COOLINT_SUBCYCLE ? subcycled(c, rho, E, dt) : trapezoid(c, rho, E, dt);
}

/* c_cool min over cells of E_th / |Edot| (+inf when no cell heats or cools);
 * the exact two-branch model has Edot = -rho^2 Lambda_exact(T) */
double or_cool_dt_limit(const or_config *c, const double *U) {
  long N = (long)c->n[0] * c->n[1] * c->n[2];
  double rmax = 0.0;
  double g = c->gamma;
  for (long q = 0; q < N; ++q) {
    double rho = U[q];
    double ek = 0.5 * (U[N + q] * U[N + q] + U[2 * N + q] * U[2 * N + q] +
                       U[3 * N + q] * U[3 * N + q]) / rho;
    double Eth = U[4 * N + q] - ek;
    double edot;
    if (c->cool_model == OR_COOL_TABLE) {
      edot = or_cool_edot(c, rho, Eth);
    } else {
      double T = (g - 1.0) * Eth / rho;
      double L = T >= c->cool_tc ? c->cool_lambda0 * sqrt(T / c->cool_tc)
                                 : c->cool_lambda0 * exp((T - c->cool_tc) / c->cool_ts);
      edot = -rho * rho * L;
    }
    double r = fabs(edot) / Eth;
    if (r > rmax) rmax = r;
  }
  return rmax > 0.0 ? c->cool_ccool / rmax : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* derivatives of the tabulated model's step (for the adjoint)               */
/* ------------------------------------------------------------------------- */

/* dLambda/dT on the branch taken: below tc the two power laws; in the table
 * s Lambda / T with s the segment's slope d log10 Lambda / d log10 T; flat
 * beyond the table's ends (0) */
static double lambda_dT(const or_config *c, double T) {
  if (T < c->cool_tc)
    return c->cool_L1 * c->cool_a1 * pow(T, c->cool_a1 - 1.0) +
           c->cool_L2 * c->cool_a2 * pow(T, c->cool_a2 - 1.0);
  int n = c->cool_ntab;
  double x = log10(T);
  if (x <= c->cool_logT[0] || x >= c->cool_logT[n - 1]) return 0.0;
  int i = 0;
  while (i < n - 2 && !(x < c->cool_logT[i + 1])) ++i;
  double s = (c->cool_logL[i + 1] - c->cool_logL[i]) / (c->cool_logT[i + 1] - c->cool_logT[i]);
  return s * or_cool_lambda(c, T) / T;
}

/* a value with its derivatives with respect to the step's inputs E_th and rho */
typedef struct {
  double v, dE, dr;
} dual2;

/* Edot(rho, E) with dEdot/dE = -(g-1) rho Lambda'(T) and dEdot/drho =
 * Gamma - 2 rho Lambda + rho T Lambda'(T) (Gamma constant on each branch) */
static dual2 edot_d(const or_config *c, double rho, dual2 E) {
  double g1 = c->gamma - 1.0;
  double T = g1 * E.v / rho;
  double heat = T < c->cool_tc ? c->cool_heat : 0.0;
  double L = or_cool_lambda(c, T), Lp = lambda_dT(c, T);
  double pE = -g1 * rho * Lp;
  double pr = heat - 2.0 * rho * L + rho * T * Lp;
  dual2 r = {rho * heat - rho * rho * L, pE * E.dE, pE * E.dr + pr};
  return r;
}

static dual2 floor_d(const or_config *c, double rho, dual2 E) {
  double Ef = rho * c->cool_tfloor / (c->gamma - 1.0); /* as floor_eth */
  if (E.v > Ef) return E;
  dual2 f = {Ef, 0.0, c->cool_tfloor / (c->gamma - 1.0)};
  return f;
}

/* or_cool_eth_step with dE'/dEth in *dE and dE'/drho in *dr, the branches
 * (floor, limiter, integrator choice, substep count) as the forward takes
 * them */
double or_cool_eth_step_d(const or_config *c, double rho, double Eth, double dt, double *dE,
                          double *dr) {
  dual2 E = {Eth, 1.0, 0.0};
  E = floor_d(c, rho, E);
  double f = c->cool_frac;
  dual2 d0 = edot_d(c, rho, E);
  int m = c->cool_integrator;
  if (m == OR_COOLINT_AUTO)
    m = dt * fabs(d0.v) <= f * E.v ? OR_COOLINT_TRAPEZOID : OR_COOLINT_SUBCYCLE;
  if (m == OR_COOLINT_TRAPEZOID) {
    dual2 Ep = {E.v + dt * d0.v, E.dE + dt * d0.dE, E.dr + dt * d0.dr};
    Ep = floor_d(c, rho, Ep);
    dual2 d1 = edot_d(c, rho, Ep);
    dual2 r = {E.v + 0.5 * dt * (d0.v + d1.v), E.dE + 0.5 * dt * (d0.dE + d1.dE),
               E.dr + 0.5 * dt * (d0.dr + d1.dr)};
    r = floor_d(c, rho, r);
    *dE = r.dE;
    *dr = r.dr;
    return r.v;
  }
  double nd = ceil(dt * fabs(d0.v) / (f * E.v));
  long N = !(nd >= 1.0) ? 1 : (nd > (double)c->cool_nsub_max ? c->cool_nsub_max : (long)nd);
  double h = dt / (double)N;
  for (long k = 0; k < N; ++k) {
    dual2 d = edot_d(c, rho, E);
    dual2 dEk = {d.v * h, d.dE * h, d.dr * h};
    dual2 lim = {f * E.v, f * E.dE, f * E.dr};
    if (dEk.v > lim.v) dEk = lim;
    if (dEk.v < -lim.v) {
      dEk.v = -lim.v;
      dEk.dE = -lim.dE;
      dEk.dr = -lim.dr;
    }
    dual2 s = {E.v + dEk.v, E.dE + dEk.dE, E.dr + dEk.dr};
    E = floor_d(c, rho, s);
  }
  *dE = E.dE;
  *dr = E.dr;
  return E.v;
}
