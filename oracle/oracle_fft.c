/*
 * oracle_fft.c -- spectral self-gravity of the oracle (paper Sec. 6.1: the
 * Fourier-space Poisson solve, the spectral acceleration, and the adjoint of
 * both).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * The transform is the discrete Fourier transform by its definition, applied
 * along x, then y, then z (the 3D transform is separable):
 *   X_k = sum_j x_j exp(-2 pi i j k / n),
 *   x_j = (1/n) sum_k X_k exp(+2 pi i j k / n),
 * each phase factor read from a table of cos and sin of 2 pi m / n with
 * m = j k mod n.  That is n operations per output value: slow and plain, for
 * test sizes.
 *
 * On a periodic cube of n cells of size h (box length L = n h), the
 * wavenumber of index q along an axis is kappa = 2 pi m / L with the integer
 * m = q for q <= n/2 and m = q - n above.  Then (Sec. 6.1)
 *   Phi_hat = -4 pi G rho_hat / |kappa|^2   (0 for kappa = 0),
 *   a_hat   = -i kappa~ Phi_hat,
 * where kappa~ is kappa with the Nyquist index q = n/2 (even n) set to 0: the
 * derivative of that mode has no real-valued counterpart, so the spectral
 * gradient drops it (|kappa|^2 keeps it).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* DFT of every line along one axis of the n^3 complex array (re, im) */
static void dft_axis(int n, int axis, int inverse, double *re, double *im) {
  long nn = n, N = nn * nn * nn;
  long stride = axis == 0 ? 1 : (axis == 1 ? nn : nn * nn);
  double *cs = (double *)malloc(sizeof(double) * nn);
  double *sn = (double *)malloc(sizeof(double) * nn);
  for (long m = 0; m < nn; ++m) {
    cs[m] = cos(2.0 * M_PI * (double)m / (double)nn);
    sn[m] = sin(2.0 * M_PI * (double)m / (double)nn);
  }
  double sgn = inverse ? 1.0 : -1.0;
  double scale = inverse ? 1.0 / (double)nn : 1.0;
#pragma omp parallel for schedule(static)
  for (long line = 0; line < N / nn; ++line) {
    /* first element of the line: the other two coordinates of `line` */
    long a = line % nn, b = line / nn, base;
    if (axis == 0) base = line * nn;
    else if (axis == 1) base = b * nn * nn + a;
    else base = b * nn + a;
    double *xr = (double *)malloc(sizeof(double) * nn);
    double *xi = (double *)malloc(sizeof(double) * nn);
    for (long j = 0; j < nn; ++j) {
      xr[j] = re[base + j * stride];
      xi[j] = im[base + j * stride];
    }
    for (long k = 0; k < nn; ++k) {
      double sr = 0.0, si = 0.0;
      for (long j = 0; j < nn; ++j) {
        long m = (j * k) % nn;
        double c = cs[m], s = sgn * sn[m]; /* exp(sgn 2 pi i j k / n) */
        sr += xr[j] * c - xi[j] * s;
        si += xr[j] * s + xi[j] * c;
      }
      re[base + k * stride] = scale * sr;
      im[base + k * stride] = scale * si;
    }
    free(xr);
    free(xi);
  }
  free(cs);
  free(sn);
}

void or_dft3(int n, int inverse, double *re, double *im) {
  for (int axis = 0; axis < 3; ++axis) dft_axis(n, axis, inverse, re, im);
}

/* integer wavenumber of index q, and its derivative version (Nyquist -> 0) */
static double wavenumber(long q, long n) { return q <= n / 2 ? (double)q : (double)(q - n); }
static double deriv_wavenumber(long q, long n) {
  return (n % 2 == 0 && q == n / 2) ? 0.0 : wavenumber(q, n);
}

/* rho: [n^3] density.  phi: [n^3] potential (out).  acc: [3][n^3] (out). */
void or_fft_gravity(const or_config *c, const double *rho, double *phi, double *acc) {
  long n = c->n[0], N = n * n * n;
  double L = (double)n * c->h[0], tk = 2.0 * M_PI / L;
  double fourpiG = 4.0 * M_PI * c->grav_G;
  double *pr = (double *)malloc(sizeof(double) * N), *pi = (double *)malloc(sizeof(double) * N);
  double mean = 0.0;
  for (long q = 0; q < N; ++q) mean += rho[q];
  mean /= (double)N;
  for (long q = 0; q < N; ++q) {
    pr[q] = rho[q] - mean;
    pi[q] = 0.0;
  }
  or_dft3((int)n, 0, pr, pi);
  /* Phi_hat = -4 pi G rho_hat / |kappa|^2 */
  for (long kz = 0; kz < n; ++kz)
    for (long ky = 0; ky < n; ++ky)
      for (long kx = 0; kx < n; ++kx) {
        long q = (kz * n + ky) * n + kx;
        double k2 = tk * tk * (wavenumber(kx, n) * wavenumber(kx, n) +
                               wavenumber(ky, n) * wavenumber(ky, n) +
                               wavenumber(kz, n) * wavenumber(kz, n));
        double f = k2 > 0.0 ? -fourpiG / k2 : 0.0;
        pr[q] *= f;
        pi[q] *= f;
      }
  double *ar = (double *)malloc(sizeof(double) * N), *ai = (double *)malloc(sizeof(double) * N);
  for (int a = 0; a < 3; ++a) {
    /* a_hat = -i kappa~_a Phi_hat: (re, im) -> (kappa~ im, -kappa~ re) */
    for (long kz = 0; kz < n; ++kz)
      for (long ky = 0; ky < n; ++ky)
        for (long kx = 0; kx < n; ++kx) {
          long q = (kz * n + ky) * n + kx;
          long idx = a == 0 ? kx : (a == 1 ? ky : kz);
          double ka = tk * deriv_wavenumber(idx, n);
          ar[q] = ka * pi[q];
          ai[q] = -ka * pr[q];
        }
    or_dft3((int)n, 1, ar, ai);
    memcpy(acc + a * N, ar, sizeof(double) * N);
  }
  or_dft3((int)n, 1, pr, pi);
  memcpy(phi, pr, sizeof(double) * N);
  free(pr); free(pi); free(ar); free(ai);
}

/* Adjoint of rho -> acc above (the potential output carries no gradient
 * here): acc_a = F^-1[m_a F[rho - <rho>]] with m_a = 4 pi G i kappa~_a /
 * |kappa|^2, so rho_b = P0 sum_a F^-1[conj(m_a) F[acc_b,a]] (P0 removes the
 * mean; m_a is 0 at kappa = 0).  This is the paper's adjoint: the potential
 * adjoint sum_a i kappa_a g_hat_a, scaled by -4 pi G / kappa^2.  Writes rhob. */
void or_fft_gravity_vjp(const or_config *c, const double *accb, double *rhob) {
  long n = c->n[0], N = n * n * n;
  double L = (double)n * c->h[0], tk = 2.0 * M_PI / L;
  double fourpiG = 4.0 * M_PI * c->grav_G;
  double *sr = (double *)calloc(N, sizeof(double)), *si = (double *)calloc(N, sizeof(double));
  double *gr = (double *)malloc(sizeof(double) * N), *gi = (double *)malloc(sizeof(double) * N);
  for (int a = 0; a < 3; ++a) {
    for (long q = 0; q < N; ++q) {
      gr[q] = accb[a * N + q];
      gi[q] = 0.0;
    }
    or_dft3((int)n, 0, gr, gi);
    for (long kz = 0; kz < n; ++kz)
      for (long ky = 0; ky < n; ++ky)
        for (long kx = 0; kx < n; ++kx) {
          long q = (kz * n + ky) * n + kx;
          long idx = a == 0 ? kx : (a == 1 ? ky : kz);
          double k2 = tk * tk * (wavenumber(kx, n) * wavenumber(kx, n) +
                                 wavenumber(ky, n) * wavenumber(ky, n) +
                                 wavenumber(kz, n) * wavenumber(kz, n));
          /* conj(m_a) = -4 pi G i kappa~_a / k2; times (gr + i gi) */
          double f = k2 > 0.0 ? -fourpiG * tk * deriv_wavenumber(idx, n) / k2 : 0.0;
          sr[q] += -f * gi[q];
          si[q] += f * gr[q];
        }
  }
  or_dft3((int)n, 1, sr, si);
  double mean = 0.0;
  for (long q = 0; q < N; ++q) mean += sr[q];
  mean /= (double)N;
  for (long q = 0; q < N; ++q) rhob[q] = sr[q] - mean;
  free(sr); free(si); free(gr); free(gi);
}
