/*
 * oracle_driver.c -- drives the FP64 oracle (oracle/*.c) under the address
 * and undefined-behaviour sanitizers: small grids through every scheme,
 * integrator, boundary, source and cooling model, the multigrid and spectral
 * gravity, and the reverse-mode step.  Exit status 0 when nothing was
 * reported (the sanitizers abort on their first finding).  Test
 * infrastructure only.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static double urand(unsigned long long *s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(*s >> 11) * 0x1.0p-53;
}

/* random primitives (rho, p in [0.5, 1.5], |v| < 0.5) as a conserved state */
static void random_state(int nx, int ny, int nz, double gamma, unsigned long long seed,
                         double *U) {
  long N = (long)nx * ny * nz;
  for (long q = 0; q < N; ++q) {
    double r = 0.5 + urand(&seed), p = 0.5 + urand(&seed);
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = urand(&seed) - 0.5;
    U[q] = r;
    for (int a = 0; a < 3; ++a) U[(1 + a) * N + q] = r * v[a];
    U[4 * N + q] = p / (gamma - 1.0) + 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  }
}

static or_config base(int nx, int ny, int nz) {
  or_config c;
  memset(&c, 0, sizeof c);
  c.n[0] = nx; c.n[1] = ny; c.n[2] = nz;
  c.h[0] = 1.0 / nx; c.h[1] = 1.0 / ny; c.h[2] = 1.0 / nz;
  c.gamma = 5.0 / 3.0; c.cfl = 0.4;
  c.cool_lambda0 = 0.3; c.cool_tc = 1e-2; c.cool_ts = 1e-3; c.cool_tfloor = 1e-4;
  c.ou_seed = 3; c.ou_tau = 0.5; c.ou_arms = 1.0; c.ou_zeta = 1.0; c.ou_kmin = 1.0;
  c.ou_kmax = 2.0; c.ou_every = 1;
  c.grav_G = 1.0; c.mg_pre = 2; c.mg_post = 2; c.mg_max_cycles = 4; c.mg_coarsest = 4;
  c.mg_tol = 1e-10; c.mg_coarse_sweeps = 50;
  c.cool_nsub_max = 20; c.cool_frac = 0.1;
  return c;
}

/* a few steps and one reverse step of configuration c */
static void exercise(const or_config *c, unsigned long long seed) {
  long N = (long)c->n[0] * c->n[1] * c->n[2];
  double *U = malloc(sizeof(double) * 5 * N), *U0 = malloc(sizeof(double) * 5 * N);
  double *lam = malloc(sizeof(double) * 5 * N), *out = malloc(sizeof(double) * 5 * N);
  double *phi = calloc(N, sizeof(double)), *phi0 = calloc(N, sizeof(double));
  int32_t nvec[3 * OR_OU_MAXMODES];
  double ahat[6 * OR_OU_MAXMODES], ahat0[6 * OR_OU_MAXMODES];
  int nm = 0;
  if (c->flags & OR_SRC_FORCING) {
    nm = or_ou_modes(c->ou_kmin, c->ou_kmax, nvec);
    or_ou_init(c, nm, nvec, ahat);
  }
  random_state(c->n[0], c->n[1], c->n[2], c->gamma, seed, U);
  memcpy(U0, U, sizeof(double) * 5 * N);
  memcpy(ahat0, ahat, sizeof ahat);
  double dt = 0.5 * or_cfl_dt(c, U);
  int cyc = 0;
  for (int k = 0; k < 3; ++k) or_step(c, U, dt, INFINITY, k, nm, nvec, ahat, phi, &cyc);
  for (long q = 0; q < 5 * N; ++q) lam[q] = urand(&seed) - 0.5;
  or_step_vjp(c, U0, dt, 0, nm, nvec, ahat0, phi0, lam, out);
  for (long q = 0; q < 5 * N; ++q)
    if (!isfinite(U[q]) || !isfinite(out[q])) {
      fprintf(stderr, "non-finite result\n");
      exit(2);
    }
  free(U); free(U0); free(lam); free(out); free(phi); free(phi0);
}

int main(void) {
  /* schemes and integrators on a ragged periodic grid, and with outflow */
  for (int lim = 0; lim <= 4; ++lim)
    for (int rs = 0; rs <= 2; ++rs) {
      or_config c = base(13, 6, 5);
      c.limiter = lim;
      c.riemann = rs;
      c.integrator = (lim + rs) % 3;
      if (lim == 2) c.bc[0] = OR_BC_OUTFLOW;
      exercise(&c, 11 + 3 * lim + rs);
    }
  /* forcing and the two-branch cooling, outflow on every axis */
  {
    or_config c = base(9, 7, 6);
    c.flags = OR_SRC_FORCING | OR_SRC_COOLING;
    c.bc[0] = c.bc[1] = c.bc[2] = OR_BC_OUTFLOW;
    exercise(&c, 31);
  }
  /* the tabulated cooling model, each integrator, with the step limit */
  for (int integ = 0; integ <= 2; ++integ) {
    or_config c = base(8, 6, 5);
    c.flags = OR_SRC_COOLING;
    c.cool_model = OR_COOL_TABLE;
    c.cool_integrator = integ;
    c.cool_ccool = 0.5;
    c.cool_ntab = 17;
    for (int i = 0; i < 17; ++i) {
      c.cool_logT[i] = -2.0 + 0.25 * i;
      c.cool_logL[i] = -1.0 - 0.1 * (i - 8) * (i - 8) / 8.0;
    }
    c.cool_L1 = 3000.0; c.cool_a1 = 2.0; c.cool_L2 = 0.003; c.cool_a2 = 0.5; c.cool_heat = 0.0272;
    exercise(&c, 41 + integ);
  }
  /* gravity: multigrid V and W cycles with both smoothers, and the spectral solve */
  for (int k = 0; k < 5; ++k) {
    or_config c = base(16, 16, 16);
    c.flags = OR_SRC_GRAVITY | OR_SRC_COOLING;
    c.mg_cycle = k & 1;
    c.mg_smoother = (k >> 1) & 1;
    if (k == 4) c.grav_solver = OR_GRAV_FFT;
    exercise(&c, 51 + k);
  }
  /* a NaN temperature through the tabulated model's bounded table search */
  {
    or_config c = base(4, 4, 4);
    c.cool_model = OR_COOL_TABLE;
    c.cool_ntab = 2;
    c.cool_logT[0] = -2.0; c.cool_logT[1] = 2.0;
    c.cool_logL[0] = -1.0; c.cool_logL[1] = -1.0;
    for (int integ = 0; integ <= 2; ++integ) {
      c.cool_integrator = integ;
      (void)or_cool_eth_step(&c, 1.0, NAN, 0.1);
    }
  }
  puts("oracle driver: ok");
  return 0;
}
