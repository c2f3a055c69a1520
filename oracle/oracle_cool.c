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
  while (!(x < c->cool_logT[i + 1])) ++i; /* logT[i] <= x < logT[i+1] */
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
  long N = nd < 1.0 ? 1 : (nd > (double)c->cool_nsub_max ? c->cool_nsub_max : (long)nd);
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
