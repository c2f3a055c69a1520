/*
 * oracle_mg.c -- FP64 geometric multigrid Poisson solver and self-gravity
 * acceleration of the oracle (paper Sec. 6 and 6.2, App. C).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * The discrete problem is A phi = F on a periodic cubic n^3 grid with spacing
 * h, A the seven-point Laplacian (Sec. 6.2, the (A phi)_{ijk} equation) and
 * F = 4 pi G (rho - <rho>) (Sec. 6.1, the mean-subtracted Poisson equation).
 * One V-cycle (App. C): nu1 weighted-Jacobi sweeps, residual, restriction by
 * the average of the 8 children, recursive coarse solve of the error equation
 * from a zero guess, trilinear prolongation and correction, nu2 sweeps.  The
 * coarsest grid is solved to round-off by many Jacobi sweeps.  The W-cycle
 * (App. C, the paper's default) makes two recursive cycles of the error
 * equation on each coarser level instead of one (the level just above the
 * coarsest solves it once), the second starting from the first one's result.
 * The smoother is weighted Jacobi or red-black Gauss-Seidel (Sec. 6.2.1).
 * The mean is
 * projected out of every right-hand side and of every solution, so the
 * singular periodic problem is solved on its mean-zero subspace (gauge
 * <phi> = 0, Sec. 6.1).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static inline long wrap(long i, long n) {
  long r = i % n;
  return r < 0 ? r + n : r;
}

static inline long id3(long n, long i, long j, long k) {
  return (wrap(k, n) * n + wrap(j, n)) * n + wrap(i, n);
}

/* sum in a fixed order: per z-plane partial sums, then the planes in order */
static double fixed_sum(long n, const double *x) {
  double *part = (double *)malloc(sizeof(double) * n);
  long plane = n * n;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) {
    double s = 0.0;
    for (long q = 0; q < plane; ++q) s += x[k * plane + q];
    part[k] = s;
  }
  double s = 0.0;
  for (long k = 0; k < n; ++k) s += part[k];
  free(part);
  return s;
}

static double fixed_sumsq(long n, const double *x) {
  double *part = (double *)malloc(sizeof(double) * n);
  long plane = n * n;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) {
    double s = 0.0;
    for (long q = 0; q < plane; ++q) s += x[k * plane + q] * x[k * plane + q];
    part[k] = s;
  }
  double s = 0.0;
  for (long k = 0; k < n; ++k) s += part[k];
  free(part);
  return s;
}

static void remove_mean(long n, double *x) {
  long N = n * n * n;
  double m = fixed_sum(n, x) / (double)N;
  for (long q = 0; q < N; ++q) x[q] -= m;
}

/* (A phi)_{ijk} = (sum of the six neighbours - 6 phi_{ijk}) / h^2 */
void or_laplacian(int n, double h, const double *phi, double *out) {
  double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k)
    for (long j = 0; j < n; ++j)
      for (long i = 0; i < n; ++i) {
        double nb = phi[id3(n, i - 1, j, k)] + phi[id3(n, i + 1, j, k)] +
                    phi[id3(n, i, j - 1, k)] + phi[id3(n, i, j + 1, k)] +
                    phi[id3(n, i, j, k - 1)] + phi[id3(n, i, j, k + 1)];
        out[id3(n, i, j, k)] = (nb - 6.0 * phi[id3(n, i, j, k)]) * ih2;
      }
}

/* weighted Jacobi, phi <- phi + omega D^{-1} (F - A phi), D = -6/h^2, which
 * is phi <- (1 - omega) phi + (omega/6)(sum of neighbours - h^2 F)
 * (Sec. 6.2.1, the matrix form), omega = 2/3 */
static void jacobi(long n, double h, double *phi, const double *F, double *tmp) {
  const double omega = 2.0 / 3.0;
  double h2 = h * h;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k)
    for (long j = 0; j < n; ++j)
      for (long i = 0; i < n; ++i) {
        double nb = phi[id3(n, i - 1, j, k)] + phi[id3(n, i + 1, j, k)] +
                    phi[id3(n, i, j - 1, k)] + phi[id3(n, i, j + 1, k)] +
                    phi[id3(n, i, j, k - 1)] + phi[id3(n, i, j, k + 1)];
        long q = id3(n, i, j, k);
        tmp[q] = (1.0 - omega) * phi[q] + (omega / 6.0) * (nb - h2 * F[q]);
      }
  memcpy(phi, tmp, sizeof(double) * n * n * n);
}

/* one red-black Gauss-Seidel sweep (Sec. 6.2.1 names it as the alternative
 * smoother): first every red cell (i + j + k even), then every black cell,
 * each set to the value that zeroes its own residual given its neighbours,
 * phi = (sum of the six neighbours - h^2 F) / 6, in place.  The grids it
 * smooths have an even n, so the colouring is consistent across the periodic
 * wrap and the cells of one colour only read the other colour. */
static void rbgs(long n, double h, double *phi, const double *F) {
  double h2 = h * h;
  for (long colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k)
      for (long j = 0; j < n; ++j)
        for (long i = 0; i < n; ++i) {
          if ((i + j + k) % 2 != colour) continue;
          double nb = phi[id3(n, i - 1, j, k)] + phi[id3(n, i + 1, j, k)] +
                      phi[id3(n, i, j - 1, k)] + phi[id3(n, i, j + 1, k)] +
                      phi[id3(n, i, j, k - 1)] + phi[id3(n, i, j, k + 1)];
          phi[id3(n, i, j, k)] = (nb - h2 * F[id3(n, i, j, k)]) / 6.0;
        }
  }
}

/* one sweep of the configured smoother */
static void smooth(const or_config *c, long n, double h, double *phi, const double *F,
                   double *tmp) {
  if (c->mg_smoother == OR_SMOOTH_RBGS) rbgs(n, h, phi, F);
  else jacobi(n, h, phi, F, tmp);
}

void or_mg_smooth(const or_config *c, int n, double h, double *phi, const double *F) {
  double *tmp = (double *)malloc(sizeof(double) * (long)n * n * n);
  smooth(c, n, h, phi, F, tmp);
  free(tmp);
}

static void residual(long n, double h, const double *phi, const double *F,
                     double *r) {
  or_laplacian((int)n, h, phi, r);
  long N = n * n * n;
  for (long q = 0; q < N; ++q) r[q] = F[q] - r[q];
}

/* r^{2h}_{IJK} = (1/8) sum over the 8 children (Sec. 6.2.2) */
static void restrict8(long nc, const double *rf, double *rc) {
  long nf = 2 * nc;
#pragma omp parallel for schedule(static)
  for (long K = 0; K < nc; ++K)
    for (long J = 0; J < nc; ++J)
      for (long I = 0; I < nc; ++I) {
        double s = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              s += rf[id3(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
        rc[id3(nc, I, J, K)] = 0.125 * s;
      }
}

/* cell-centred trilinear prolongation-and-add (Sec. 6.2.3): a fine cell sits a
 * quarter coarse cell from its parent's centre, so per axis it takes 3/4 of
 * the parent and 1/4 of the parent's neighbour on the child's side */
static void prolong_add(long nc, const double *ec, double *phif) {
  long nf = 2 * nc;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nf; ++k)
    for (long j = 0; j < nf; ++j)
      for (long i = 0; i < nf; ++i) {
        long I = i / 2, J = j / 2, K = k / 2;
        long si = (i % 2) ? 1 : -1, sj = (j % 2) ? 1 : -1, sk = (k % 2) ? 1 : -1;
        double e = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
              e += w * ec[id3(nc, I + a * si, J + b * sj, K + c * sk)];
            }
        phif[id3(nf, i, j, k)] += e;
      }
}

static int is_coarsest(const or_config *c, long n) {
  return n <= c->mg_coarsest || (n % 2) != 0;
}

void or_mg_vcycle(const or_config *c, int n_, double h, double *phi,
                  const double *F) {
  long n = n_, N = n * n * n;
  double *tmp = (double *)malloc(sizeof(double) * N);
  if (is_coarsest(c, n)) {
    for (int s = 0; s < c->mg_coarse_sweeps; ++s) jacobi(n, h, phi, F, tmp);
    remove_mean(n, phi);
    free(tmp);
    return;
  }
  for (int s = 0; s < c->mg_pre; ++s) smooth(c, n, h, phi, F, tmp);
  double *r = (double *)malloc(sizeof(double) * N);
  residual(n, h, phi, F, r);
  long nc = n / 2, Nc = nc * nc * nc;
  double *rc = (double *)malloc(sizeof(double) * Nc);
  double *ec = (double *)calloc(Nc, sizeof(double));
  restrict8(nc, r, rc);
  remove_mean(nc, rc);
  /* V: one cycle of the error equation; W: two (one on the coarsest) */
  int mu = (c->mg_cycle == OR_MG_W && !is_coarsest(c, nc)) ? 2 : 1;
  for (int m = 0; m < mu; ++m) or_mg_vcycle(c, (int)nc, 2.0 * h, ec, rc);
  prolong_add(nc, ec, phi);
  for (int s = 0; s < c->mg_post; ++s) smooth(c, n, h, phi, F, tmp);
  free(r);
  free(rc);
  free(ec);
  free(tmp);
}

/* Cycles (V or W) from the warm start in phi until ||F - A phi||_2 <= tol ||F||_2 or
 * mg_max_cycles cycles; the mean of phi is removed after every cycle.
 * Returns the number of cycles run. */
int or_mg_solve(const or_config *c, int n_, double h, double *phi,
                const double *F) {
  long n = n_, N = n * n * n;
  double *r = (double *)malloc(sizeof(double) * N);
  double fn = sqrt(fixed_sumsq(n, F));
  int cyc = 0;
  double prev = INFINITY;
  remove_mean(n, phi);
  for (;;) {
    residual(n, h, phi, F, r);
    double rn = sqrt(fixed_sumsq(n, r));
    if (rn <= c->mg_tol * fn || cyc >= c->mg_max_cycles) break;
    /* with a tolerance, stop once a cycle cuts the residual by less than 10 %:
       the residual has reached the round-off floor of the arithmetic */
    if (c->mg_tol > 0.0 && rn > 0.9 * prev) break;
    prev = rn;
    or_mg_vcycle(c, n_, h, phi, F);
    remove_mean(n, phi);
    ++cyc;
  }
  free(r);
  return cyc;
}

/* F = 4 pi G (rho - <rho>), solve A phi = F, g = -grad phi by central
 * differences g_a = -(phi_{i+1} - phi_{i-1}) / (2h)  (Sec. 6, "the usual
 * finite-difference gradient").  Needs a periodic cube with equal spacing. */
int or_gravity_accel(const or_config *c, const double *U, double *phi,
                     double *acc) {
  long n = c->n[0], N = n * n * n;
  if (c->grav_solver == OR_GRAV_FFT) {
    /* the spectral solve and gradient of Sec. 6.1 (oracle_fft.c) */
    or_fft_gravity(c, U, phi, acc);
    return 0;
  }
  double h = c->h[0];
  double *F = (double *)malloc(sizeof(double) * N);
  double mean = fixed_sum(n, U) / (double)N;
  double fourpiG = 4.0 * M_PI * c->grav_G;
  for (long q = 0; q < N; ++q) F[q] = fourpiG * (U[q] - mean);
  int cyc = or_mg_solve(c, (int)n, h, phi, F);
  double i2h = 1.0 / (2.0 * h);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k)
    for (long j = 0; j < n; ++j)
      for (long i = 0; i < n; ++i) {
        long q = id3(n, i, j, k);
        acc[q] = -(phi[id3(n, i + 1, j, k)] - phi[id3(n, i - 1, j, k)]) * i2h;
        acc[N + q] = -(phi[id3(n, i, j + 1, k)] - phi[id3(n, i, j - 1, k)]) * i2h;
        acc[2 * N + q] = -(phi[id3(n, i, j, k + 1)] - phi[id3(n, i, j, k - 1)]) * i2h;
      }
  free(F);
  return cyc;
}
