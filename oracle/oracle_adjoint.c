/*
 * oracle_adjoint.c -- FP64 reverse-mode derivative (vector-Jacobian product)
 * of the oracle's time step, written by hand, statement by statement, as the
 * reverse of the forward code in oracle.c and oracle_mg.c.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * The paper obtains gradients by reverse-mode differentiation through the
 * time loop with checkpointing (Sec. 2.3), with custom adjoints for the
 * elliptic solve (Sec. 6.2.4: for the symmetric Poisson operator the adjoint
 * is another solve with the same operator).  Here the time step dt is held
 * fixed (the optional gradient stop of App. A.4), and at every non-smooth
 * point the derivative of the branch the forward took is used: minmod takes
 * the derivative of the argument it returned (0 when it returned 0), min/max
 * of the wave speeds that of the argument selected (the first on ties), the
 * HLLC region that of the region selected, the cooling branch and floor those
 * of the branch taken.  The other limiters (van Leer, MC, superbee) and
 * solvers (HLL, Rusanov) follow the same rule; the branch orders are given
 * at lim_partials and at the solvers' reverse functions.
 *
 * All vectors are laid out like the state: [5][nz][ny][nx].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static inline long cells(const or_config *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }
static inline long idx(const or_config *c, long i, long j, long k) {
  return (k * c->n[1] + j) * c->n[0] + i;
}
static inline long bcmap(long i, long n, int bc) {
  if (bc == OR_BC_PERIODIC) {
    long r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* ------------------------------------------------------------------------- */
/* minmod and its subgradient                                                */
/* ------------------------------------------------------------------------- */

/* forward minmod with the selection it made: 1 = returned a, 2 = returned b,
 * 0 = returned 0 (same rule as the forward: a tie |a| = |b| takes a) */
static double minmod_sel(double a, double b, int *sel) {
  if (a * b <= 0.0) {
    *sel = 0;
    return 0.0;
  }
  if (fabs(a) <= fabs(b)) {
    *sel = 1;
    return a;
  }
  *sel = 2;
  return b;
}

/* A limited slope phi(a, b) of App. A.1 (a = W_{i+1} - W_i, b = W_i -
 * W_{i-1}), computed like oracle.c, with its partial derivatives pa =
 * dphi/da, pb = dphi/db on the branch taken.  Every limiter is 0 (pa = pb =
 * 0) when ab <= 0.  Otherwise:
 *   minmod   a if |a| <= |b| (1, 0), else b (0, 1);
 *   van Leer 2ab/(a+b): (2b^2/(a+b)^2, 2a^2/(a+b)^2);
 *   MC       the smallest of |a+b|/2, 2|a|, 2|b| with the sign of a, ties in
 *            that order: (a+b)/2 (1/2, 1/2), 2a (2, 0), 2b (0, 2);
 *   superbee max(min(2|a|, |b|), min(|a|, 2|b|)) with the sign of a: the
 *            first min on ties, each min its first argument on ties:
 *            2a (2, 0), b (0, 1), a (1, 0), 2b (0, 2). */
static double lim_partials(int limiter, double a, double b, double *pa, double *pb) {
  *pa = 0.0;
  *pb = 0.0;
  if (limiter == OR_LIM_NONE || a * b <= 0.0) return 0.0;
  if (limiter == OR_LIM_MINMOD) {
    int sel;
    double m = minmod_sel(a, b, &sel);
    *pa = sel == 1 ? 1.0 : 0.0;
    *pb = sel == 2 ? 1.0 : 0.0;
    return m;
  }
  if (limiter == OR_LIM_VANLEER) {
    double s = a + b;
    *pa = 2.0 * b * b / (s * s);
    *pb = 2.0 * a * a / (s * s);
    return 2.0 * a * b / (a + b);
  }
  if (limiter == OR_LIM_MC) {
    double cen = fabs(0.5 * (a + b)), ta = 2.0 * fabs(a), tb = 2.0 * fabs(b);
    double m = fmin(cen, fmin(ta, tb));
    if (cen <= fmin(ta, tb)) { *pa = 0.5; *pb = 0.5; }
    else if (ta <= tb) *pa = 2.0;
    else *pb = 2.0;
    return a > 0.0 ? m : -m;
  }
  /* superbee */
  double s1 = fmin(2.0 * fabs(a), fabs(b));
  double s2 = fmin(fabs(a), 2.0 * fabs(b));
  double m = fmax(s1, s2);
  if (s1 >= s2) {
    if (2.0 * fabs(a) <= fabs(b)) *pa = 2.0;
    else *pb = 1.0;
  } else {
    if (fabs(a) <= 2.0 * fabs(b)) *pa = 1.0;
    else *pb = 2.0;
  }
  return a > 0.0 ? m : -m;
}

/* ------------------------------------------------------------------------- */
/* HLLC: forward recomputation and reverse sweep                             */
/* ------------------------------------------------------------------------- */

/* Reverse of the four-region HLLC flux of oracle.c for face states
 * wl, wr = (rho, v_n, v_t1, v_t2, P) in the face frame.  Given Fb = dL/dF,
 * adds dL/dwl to wlb and dL/dwr to wrb. */
void or_hllc_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                 double wlb[5], double wrb[5]) {
  const double gm1 = g - 1.0;
  /* forward */
  double rl = wl[0], ul = wl[1], vl = wl[2], tl = wl[3], pl = wl[4];
  double rr = wr[0], ur = wr[1], vr = wr[2], tr = wr[3], pr = wr[4];
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  int minL = (ul - cl) <= (ur - cr);
  double SL = minL ? ul - cl : ur - cr;
  int maxL = (ul + cl) >= (ur + cr);
  double SR = maxL ? ul + cl : ur + cr;
  double El = pl / gm1 + 0.5 * rl * (ul * ul + vl * vl + tl * tl);
  double Er = pr / gm1 + 0.5 * rr * (ur * ur + vr * vr + tr * tr);
  double dl = rl * (SL - ul), dr = rr * (SR - ur);
  double num = pr - pl + ul * dl - ur * dr;
  double den = dl - dr;
  double ss = num / den;
  int region = (0.0 <= SL) ? 1 : (0.0 <= ss) ? 2 : (0.0 < SR) ? 3 : 4;

  /* adjoint accumulators */
  double rlb = 0, ulb = 0, vlb = 0, tlb = 0, plb = 0, Elb = 0;
  double rrb = 0, urb = 0, vrb = 0, trb = 0, prb = 0, Erb = 0;
  double SLb = 0, SRb = 0, dlb = 0, drb = 0, ssb = 0;

  if (region == 1 || region == 2 || region == 3 || region == 4) {
    /* pick side K and its data */
    int left = (region <= 2);
    double rK = left ? rl : rr, uK = left ? ul : ur, vK = left ? vl : vr, tK = left ? tl : tr;
    double pK = left ? pl : pr, EK = left ? El : Er, SK = left ? SL : SR, dK = left ? dl : dr;
    double rKb = 0, uKb = 0, vKb = 0, tKb = 0, pKb = 0, EKb = 0, SKb = 0, dKb = 0;
    double FKb[5] = {Fb[0], Fb[1], Fb[2], Fb[3], Fb[4]};
    if (region == 2 || region == 3) {
      /* F = F_K + S_K (U*_K - U_K) */
      double fac = dK / (SK - ss);
      double Y = ss + pK / dK;
      double X = EK / rK + (ss - uK) * Y;
      double Us[5] = {fac, fac * ss, fac * vK, fac * tK, fac * X};
      double UK[5] = {rK, rK * uK, rK * vK, rK * tK, EK};
      double Usb[5], UKb[5];
      for (int f = 0; f < 5; ++f) {
        SKb += Fb[f] * (Us[f] - UK[f]);
        Usb[f] = SK * Fb[f];
        UKb[f] = -SK * Fb[f];
      }
      /* Us = fac [1, ss, vK, tK, X] */
      double facb = Usb[0] + Usb[1] * ss + Usb[2] * vK + Usb[3] * tK + Usb[4] * X;
      ssb += Usb[1] * fac;
      vKb += Usb[2] * fac;
      tKb += Usb[3] * fac;
      double Xb = Usb[4] * fac;
      /* X = EK/rK + (ss - uK) Y */
      EKb += Xb / rK;
      rKb -= Xb * EK / (rK * rK);
      ssb += Xb * Y;
      uKb -= Xb * Y;
      double Yb = Xb * (ss - uK);
      /* Y = ss + pK/dK */
      ssb += Yb;
      pKb += Yb / dK;
      dKb -= Yb * pK / (dK * dK);
      /* fac = dK / (SK - ss) */
      double Z = SK - ss;
      dKb += facb / Z;
      double Zb = -facb * dK / (Z * Z);
      SKb += Zb;
      ssb -= Zb;
      /* U_K = [rK, rK uK, rK vK, rK tK, EK] */
      rKb += UKb[0] + UKb[1] * uK + UKb[2] * vK + UKb[3] * tK;
      uKb += UKb[1] * rK;
      vKb += UKb[2] * rK;
      tKb += UKb[3] * rK;
      EKb += UKb[4];
    }
    /* F_K = [rK uK, rK uK^2 + pK, rK uK vK, rK uK tK, uK (EK + pK)] */
    rKb += FKb[0] * uK + FKb[1] * uK * uK + FKb[2] * uK * vK + FKb[3] * uK * tK;
    uKb += FKb[0] * rK + FKb[1] * 2.0 * rK * uK + FKb[2] * rK * vK + FKb[3] * rK * tK +
           FKb[4] * (EK + pK);
    vKb += FKb[2] * rK * uK;
    tKb += FKb[3] * rK * uK;
    pKb += FKb[1] + FKb[4] * uK;
    EKb += FKb[4] * uK;
    /* scatter side-K adjoints back */
    if (left) {
      rlb += rKb; ulb += uKb; vlb += vKb; tlb += tKb; plb += pKb; Elb += EKb;
      SLb += SKb; dlb += dKb;
    } else {
      rrb += rKb; urb += uKb; vrb += vKb; trb += tKb; prb += pKb; Erb += EKb;
      SRb += SKb; drb += dKb;
    }
  }
  /* ss = num / den */
  double numb = ssb / den;
  double denb = -ssb * ss / den;
  /* num = pr - pl + ul dl - ur dr */
  prb += numb;
  plb -= numb;
  ulb += numb * dl;
  dlb += numb * ul;
  urb -= numb * dr;
  drb -= numb * ur;
  /* den = dl - dr */
  dlb += denb;
  drb -= denb;
  /* dl = rl (SL - ul), dr = rr (SR - ur) */
  rlb += dlb * (SL - ul);
  SLb += dlb * rl;
  ulb -= dlb * rl;
  rrb += drb * (SR - ur);
  SRb += drb * rr;
  urb -= drb * rr;
  /* E_K = P/(g-1) + rho |v|^2 / 2 */
  plb += Elb / gm1;
  rlb += Elb * 0.5 * (ul * ul + vl * vl + tl * tl);
  ulb += Elb * rl * ul;
  vlb += Elb * rl * vl;
  tlb += Elb * rl * tl;
  prb += Erb / gm1;
  rrb += Erb * 0.5 * (ur * ur + vr * vr + tr * tr);
  urb += Erb * rr * ur;
  vrb += Erb * rr * vr;
  trb += Erb * rr * tr;
  /* SL = min(ul - cl, ur - cr), SR = max(ul + cl, ur + cr) */
  double clb = 0, crb = 0;
  if (minL) { ulb += SLb; clb -= SLb; } else { urb += SLb; crb -= SLb; }
  if (maxL) { ulb += SRb; clb += SRb; } else { urb += SRb; crb += SRb; }
  /* c = sqrt(g P / rho): dc/dP = g/(2 c rho), dc/drho = -c/(2 rho) */
  plb += clb * g / (2.0 * cl * rl);
  rlb -= clb * cl / (2.0 * rl);
  prb += crb * g / (2.0 * cr * rr);
  rrb -= crb * cr / (2.0 * rr);

  wlb[0] += rlb; wlb[1] += ulb; wlb[2] += vlb; wlb[3] += tlb; wlb[4] += plb;
  wrb[0] += rrb; wrb[1] += urb; wrb[2] += vrb; wrb[3] += trb; wrb[4] += prb;
}

/* ------------------------------------------------------------------------- */
/* HLL and Rusanov: reverse sweeps                                            */
/* ------------------------------------------------------------------------- */

/* conserved state U and flux F of a face-frame primitive state (oracle.c's
 * flux_of), and the reverse: adds dL/dw given Ub = dL/dU, Fb = dL/dF */
static void state_flux(const double w[5], double g, double U[5], double F[5]) {
  double rho = w[0], vn = w[1], t1 = w[2], t2 = w[3], p = w[4];
  double E = p / (g - 1.0) + 0.5 * rho * (vn * vn + t1 * t1 + t2 * t2);
  U[0] = rho; U[1] = rho * vn; U[2] = rho * t1; U[3] = rho * t2; U[4] = E;
  F[0] = rho * vn; F[1] = rho * vn * vn + p; F[2] = rho * vn * t1; F[3] = rho * vn * t2;
  F[4] = vn * (E + p);
}

static void state_flux_vjp(const double w[5], double g, const double Ub[5], const double Fb[5],
                           double wb[5]) {
  double rho = w[0], vn = w[1], t1 = w[2], t2 = w[3], p = w[4];
  double E = p / (g - 1.0) + 0.5 * rho * (vn * vn + t1 * t1 + t2 * t2);
  double Eb = Ub[4] + Fb[4] * vn;
  wb[0] += Ub[0] + Ub[1] * vn + Ub[2] * t1 + Ub[3] * t2 + Fb[0] * vn + Fb[1] * vn * vn +
           Fb[2] * vn * t1 + Fb[3] * vn * t2 + Eb * 0.5 * (vn * vn + t1 * t1 + t2 * t2);
  wb[1] += Ub[1] * rho + Fb[0] * rho + Fb[1] * 2.0 * rho * vn + Fb[2] * rho * t1 +
           Fb[3] * rho * t2 + Fb[4] * (E + p) + Eb * rho * vn;
  wb[2] += Ub[2] * rho + Fb[2] * rho * vn + Eb * rho * t1;
  wb[3] += Ub[3] * rho + Fb[3] * rho * vn + Eb * rho * t2;
  wb[4] += Fb[1] + Fb[4] * vn + Eb / (g - 1.0);
}

/* c = sqrt(g P / rho) reversed: adds cb dc/dw to wb */
static void sound_vjp(const double w[5], double g, double c, double cb, double wb[5]) {
  wb[4] += cb * g / (2.0 * c * w[0]);
  wb[0] -= cb * c / (2.0 * w[0]);
}

/* Reverse of oracle.c's HLL flux.  Regions: F_L when 0 <= S_L, else F_R when
 * S_R <= 0, else the HLL average
 *   F = (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L),
 * whose partials are dF/dS_L = (S_R (U_R - U_L) - F_R + F)/(S_R - S_L),
 * dF/dS_R = (F_L + S_L (U_R - U_L) - F)/(S_R - S_L).  The Davis min/max
 * take the left argument on ties, as in or_hllc_vjp. */
void or_hll_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                double wlb[5], double wrb[5]) {
  double UL[5], FL[5], UR[5], FR[5];
  state_flux(wl, g, UL, FL);
  state_flux(wr, g, UR, FR);
  double cl = sqrt(g * wl[4] / wl[0]), cr = sqrt(g * wr[4] / wr[0]);
  int minL = (wl[1] - cl) <= (wr[1] - cr);
  int maxL = (wl[1] + cl) >= (wr[1] + cr);
  double SL = minL ? wl[1] - cl : wr[1] - cr;
  double SR = maxL ? wl[1] + cl : wr[1] + cr;
  double ULb[5] = {0}, FLb[5] = {0}, URb[5] = {0}, FRb[5] = {0};
  double SLb = 0.0, SRb = 0.0;
  if (0.0 <= SL) {
    for (int f = 0; f < 5; ++f) FLb[f] = Fb[f];
  } else if (SR <= 0.0) {
    for (int f = 0; f < 5; ++f) FRb[f] = Fb[f];
  } else {
    double D = SR - SL;
    for (int f = 0; f < 5; ++f) {
      double F = (SR * FL[f] - SL * FR[f] + SL * SR * (UR[f] - UL[f])) / D;
      FLb[f] = Fb[f] * SR / D;
      FRb[f] = -Fb[f] * SL / D;
      URb[f] = Fb[f] * SL * SR / D;
      ULb[f] = -URb[f];
      SLb += Fb[f] * (SR * (UR[f] - UL[f]) - FR[f] + F) / D;
      SRb += Fb[f] * (FL[f] + SL * (UR[f] - UL[f]) - F) / D;
    }
  }
  double clb = 0.0, crb = 0.0;
  if (minL) { wlb[1] += SLb; clb -= SLb; } else { wrb[1] += SLb; crb -= SLb; }
  if (maxL) { wlb[1] += SRb; clb += SRb; } else { wrb[1] += SRb; crb += SRb; }
  sound_vjp(wl, g, cl, clb, wlb);
  sound_vjp(wr, g, cr, crb, wrb);
  state_flux_vjp(wl, g, ULb, FLb, wlb);
  state_flux_vjp(wr, g, URb, FRb, wrb);
}

/* Reverse of the Rusanov flux F = (F_L + F_R)/2 - s (U_R - U_L)/2 with
 * s = max(|v_L| + c_L, |v_R| + c_R): the left argument on ties, and
 * d|v|/dv = -1 for v < 0, else +1. */
void or_rusanov_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                    double wlb[5], double wrb[5]) {
  double UL[5], FL[5], UR[5], FR[5];
  state_flux(wl, g, UL, FL);
  state_flux(wr, g, UR, FR);
  double cl = sqrt(g * wl[4] / wl[0]), cr = sqrt(g * wr[4] / wr[0]);
  int maxL = (fabs(wl[1]) + cl) >= (fabs(wr[1]) + cr);
  double s = maxL ? fabs(wl[1]) + cl : fabs(wr[1]) + cr;
  double ULb[5], FLb[5], URb[5], FRb[5];
  double sb = 0.0;
  for (int f = 0; f < 5; ++f) {
    FLb[f] = 0.5 * Fb[f];
    FRb[f] = 0.5 * Fb[f];
    URb[f] = -0.5 * s * Fb[f];
    ULb[f] = 0.5 * s * Fb[f];
    sb -= 0.5 * Fb[f] * (UR[f] - UL[f]);
  }
  double clb = 0.0, crb = 0.0;
  if (maxL) {
    wlb[1] += sb * (wl[1] < 0.0 ? -1.0 : 1.0);
    clb = sb;
  } else {
    wrb[1] += sb * (wr[1] < 0.0 ? -1.0 : 1.0);
    crb = sb;
  }
  sound_vjp(wl, g, cl, clb, wlb);
  sound_vjp(wr, g, cr, crb, wrb);
  state_flux_vjp(wl, g, ULb, FLb, wlb);
  state_flux_vjp(wr, g, URb, FRb, wrb);
}

/* ------------------------------------------------------------------------- */
/* J(U)^T v for L = or_rhs                                                    */
/* ------------------------------------------------------------------------- */

/* Reverse of or_rhs: out = (dL/dU)^T v.  For each pencil, the face adjoints
 * Fb_f = dL/dF_f come from the differencing (face f adds +F_f/h to cell f and
 * -F_f/h to cell f-1 when those are real cells), each face's HLLC reverse
 * gives the face-state adjoints, the MUSCL reconstruction is reversed onto the
 * ghost-extended pencil, ghost positions fold onto the cells they copy, and
 * finally dW/dU is applied per cell. */
void or_rhs_vjp(const or_config *c, const double *U, const double *v, double *out) {
  long N = cells(c);
  double *W = (double *)malloc(sizeof(double) * 5 * N);
  double *Wb = (double *)calloc(5 * N, sizeof(double));
  or_primitives(c, U, W);
  for (int a = 0; a < 3; ++a) {
    long n = c->n[a];
    int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    long npencil = (long)c->n[b1] * c->n[b2];
    double inv_h = 1.0 / c->h[a];
    int vn = 1 + a, vt1 = 1 + b1, vt2 = 1 + b2;
    int perm[5] = {0, vn, vt1, vt2, 4}; /* face-frame slot -> state field */
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npencil; ++p) {
      long j1 = p % c->n[b1], j2 = p / c->n[b1];
      double (*wg)[5] = malloc(sizeof(double[5]) * (n + 4));
      double (*wgb)[5] = calloc(n + 4, sizeof(double[5]));
      double (*slope)[5] = malloc(sizeof(double[5]) * (n + 2));
      double (*pa)[5] = malloc(sizeof(double[5]) * (n + 2));
      double (*pb)[5] = malloc(sizeof(double[5]) * (n + 2));
      long *q = malloc(sizeof(long) * (n + 4)); /* cell of each position */
      long cq[3];
      for (long i = -2; i < n + 2; ++i) {
        cq[a] = bcmap(i, n, c->bc[a]);
        cq[b1] = j1;
        cq[b2] = j2;
        q[i + 2] = idx(c, cq[0], cq[1], cq[2]);
        for (int s = 0; s < 5; ++s) wg[i + 2][s] = W[perm[s] * N + q[i + 2]];
      }
      for (long i = -1; i <= n; ++i)
        for (int s = 0; s < 5; ++s) {
          double av = wg[i + 3][s] - wg[i + 2][s], bv = wg[i + 2][s] - wg[i + 1][s];
          slope[i + 1][s] = lim_partials(c->limiter, av, bv, &pa[i + 1][s], &pb[i + 1][s]);
        }
      for (long fidx = 0; fidx <= n; ++fidx) {
        double wl[5], wr[5], Fb[5], wlb[5] = {0}, wrb[5] = {0};
        for (int s = 0; s < 5; ++s) {
          wl[s] = wg[fidx + 1][s] + 0.5 * slope[fidx][s];
          wr[s] = wg[fidx + 2][s] - 0.5 * slope[fidx + 1][s];
        }
        for (int s = 0; s < 5; ++s) {
          double right = (fidx <= n - 1) ? v[perm[s] * N + q[fidx + 2]] : 0.0;
          double left = (fidx - 1 >= 0) ? v[perm[s] * N + q[fidx + 1]] : 0.0;
          Fb[s] = (right - left) * inv_h;
        }
        if (c->riemann == OR_RS_HLL) or_hll_vjp(wl, wr, c->gamma, Fb, wlb, wrb);
        else if (c->riemann == OR_RS_RUSANOV) or_rusanov_vjp(wl, wr, c->gamma, Fb, wlb, wrb);
        else or_hllc_vjp(wl, wr, c->gamma, Fb, wlb, wrb);
        /* wl = W_{i} + slope_i/2 (i = fidx-1, position fidx+1), with
         * slope_i = phi(W_{i+1} - W_i, W_i - W_{i-1}) */
        for (int s = 0; s < 5; ++s) {
          wgb[fidx + 1][s] += wlb[s];
          double sb = 0.5 * wlb[s];
          wgb[fidx + 2][s] += sb * pa[fidx][s];
          wgb[fidx + 1][s] += sb * (pb[fidx][s] - pa[fidx][s]);
          wgb[fidx][s] -= sb * pb[fidx][s];
          /* wr = W_{i+1} - slope_{i+1}/2 (position fidx+2) */
          wgb[fidx + 2][s] += wrb[s];
          double tb = -0.5 * wrb[s];
          wgb[fidx + 3][s] += tb * pa[fidx + 1][s];
          wgb[fidx + 2][s] += tb * (pb[fidx + 1][s] - pa[fidx + 1][s]);
          wgb[fidx + 1][s] -= tb * pb[fidx + 1][s];
        }
      }
      /* fold positions onto cells (the pencil is private to this thread) */
      for (long i = -2; i < n + 2; ++i)
        for (int s = 0; s < 5; ++s) Wb[perm[s] * N + q[i + 2]] += wgb[i + 2][s];
      free(wg); free(wgb); free(slope); free(pa); free(pb); free(q);
    }
  }
  /* W = (rho, v, P) from U = (rho, m, E):
   * rho_b += Wb_rho - sum_a Wb_va v_a / rho + Wb_P (g-1) |v|^2 / 2
   * m_a_b = Wb_va / rho - Wb_P (g-1) v_a,  E_b = Wb_P (g-1) */
  double gm1 = c->gamma - 1.0;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; ++k) {
    double rho = U[k];
    double vx = U[N + k] / rho, vy = U[2 * N + k] / rho, vz = U[3 * N + k] / rho;
    double wr = Wb[k], wx = Wb[N + k], wy = Wb[2 * N + k], wz = Wb[3 * N + k], wp = Wb[4 * N + k];
    out[k] = wr - (wx * vx + wy * vy + wz * vz) / rho + wp * gm1 * 0.5 * (vx * vx + vy * vy + vz * vz);
    out[N + k] = wx / rho - wp * gm1 * vx;
    out[2 * N + k] = wy / rho - wp * gm1 * vy;
    out[3 * N + k] = wz / rho - wp * gm1 * vz;
    out[4 * N + k] = wp * gm1;
  }
  free(W);
  free(Wb);
}

/* ------------------------------------------------------------------------- */
/* RK2                                                                        */
/* ------------------------------------------------------------------------- */

/* Reverse of U1 = U + dt L(U), U2 = U/2 + (U1 + dt L(U1))/2:
 *   lam1 = lam2/2 + (dt/2) J(U1)^T lam2,
 *   lam  = lam2/2 + lam1 + dt J(U)^T lam1. */
/* gflux (or NULL): += the adjoint of the flux-correction field, which enters
 * every stage's L with the stage's dt weight (or_flux_corr_vjp) */
static void rk2_vjp(const or_config *c, const double *U, double dt, const double *lam2,
                    double *lam, double *gflux) {
  long N5 = 5 * cells(c);
  double *U1 = (double *)malloc(sizeof(double) * N5);
  double *L = (double *)malloc(sizeof(double) * N5);
  double *lam1 = (double *)malloc(sizeof(double) * N5);
  double *tmp = (double *)malloc(sizeof(double) * N5);
  or_rhs(c, U, L);
  for (long q = 0; q < N5; ++q) U1[q] = U[q] + dt * L[q];
  or_rhs_vjp(c, U1, lam2, tmp);
  for (long q = 0; q < N5; ++q) lam1[q] = 0.5 * lam2[q] + 0.5 * dt * tmp[q];
  or_rhs_vjp(c, U, lam1, tmp);
  for (long q = 0; q < N5; ++q) lam[q] = 0.5 * lam2[q] + lam1[q] + dt * tmp[q];
  if (gflux) {
    or_flux_corr_vjp(c, lam2, 0.5 * dt, gflux); /* U_new = U/2 + (U1 + dt L(U1))/2 */
    or_flux_corr_vjp(c, lam1, dt, gflux);       /* U1 = U + dt L(U) */
  }
  free(U1); free(L); free(lam1); free(tmp);
}

void or_rk2_vjp(const or_config *c, const double *U, double dt, const double *lam2,
                double *lam) {
  rk2_vjp(c, U, dt, lam2, lam, NULL);
}

/* Reverse of forward Euler: lam = lam1 + dt J(U)^T lam1. */
static void euler_vjp(const or_config *c, const double *U, double dt, const double *lam1,
                      double *lam, double *gflux) {
  long N5 = 5 * cells(c);
  double *tmp = (double *)malloc(sizeof(double) * N5);
  or_rhs_vjp(c, U, lam1, tmp);
  for (long q = 0; q < N5; ++q) lam[q] = lam1[q] + dt * tmp[q];
  if (gflux) or_flux_corr_vjp(c, lam1, dt, gflux);
  free(tmp);
}

void or_euler_vjp(const or_config *c, const double *U, double dt, const double *lam1,
                  double *lam) {
  euler_vjp(c, U, dt, lam1, lam, NULL);
}

/* Reverse of SSPRK3 (or_ssprk3), stage by stage from the last one, with lam3
 * the adjoint of U_new:
 *   lam2 = 2/3 (lam3 + dt J(U2)^T lam3)            (adjoint of U2)
 *   lam1 = 1/4 (lam2 + dt J(U1)^T lam2)            (adjoint of U1)
 *   lam  = lam3/3 + 3/4 lam2 + lam1 + dt J(U)^T lam1 */
static void ssprk3_vjp(const or_config *c, const double *U, double dt, const double *lam3,
                       double *lam, double *gflux) {
  long N5 = 5 * cells(c);
  double *L = (double *)malloc(sizeof(double) * N5);
  double *U1 = (double *)malloc(sizeof(double) * N5);
  double *U2 = (double *)malloc(sizeof(double) * N5);
  double *lam1 = (double *)malloc(sizeof(double) * N5);
  double *lam2 = (double *)malloc(sizeof(double) * N5);
  double *tmp = (double *)malloc(sizeof(double) * N5);
  or_rhs(c, U, L);
  for (long q = 0; q < N5; ++q) U1[q] = U[q] + dt * L[q];
  or_rhs(c, U1, L);
  for (long q = 0; q < N5; ++q) U2[q] = 0.75 * U[q] + 0.25 * (U1[q] + dt * L[q]);
  or_rhs_vjp(c, U2, lam3, tmp);
  for (long q = 0; q < N5; ++q) lam2[q] = 2.0 / 3.0 * (lam3[q] + dt * tmp[q]);
  or_rhs_vjp(c, U1, lam2, tmp);
  for (long q = 0; q < N5; ++q) lam1[q] = 0.25 * (lam2[q] + dt * tmp[q]);
  or_rhs_vjp(c, U, lam1, tmp);
  for (long q = 0; q < N5; ++q)
    lam[q] = lam3[q] / 3.0 + 0.75 * lam2[q] + lam1[q] + dt * tmp[q];
  if (gflux) {
    or_flux_corr_vjp(c, lam3, 2.0 / 3.0 * dt, gflux); /* the last stage's L(U2) */
    or_flux_corr_vjp(c, lam2, 0.25 * dt, gflux);       /* U2's L(U1) */
    or_flux_corr_vjp(c, lam1, dt, gflux);              /* U1's L(U) */
  }
  free(L); free(U1); free(U2); free(lam1); free(lam2); free(tmp);
}

void or_ssprk3_vjp(const or_config *c, const double *U, double dt, const double *lam3,
                   double *lam) {
  ssprk3_vjp(c, U, dt, lam3, lam, NULL);
}

/* reverse of or_integrate; gflux (or NULL) += the adjoint of the flux
 * correction */
void or_integrate_vjp_flux(const or_config *c, const double *U, double dt, const double *lamp,
                           double *lam, double *gflux) {
  if (c->integrator == OR_RK_SSP3) ssprk3_vjp(c, U, dt, lamp, lam, gflux);
  else if (c->integrator == OR_RK_EULER) euler_vjp(c, U, dt, lamp, lam, gflux);
  else rk2_vjp(c, U, dt, lamp, lam, gflux);
}

void or_integrate_vjp(const or_config *c, const double *U, double dt, const double *lamp,
                      double *lam) {
  or_integrate_vjp_flux(c, U, dt, lamp, lam, NULL);
}

/* g += weight (dL/dflux_corr)^T v for L = or_rhs: the correction at cell i
 * is the flux of its +a face on every axis a; a face's flux enters L of the
 * cell on its left with -1/h_a and of the cell on its right with +1/h_a
 * (cells that exist: with outflow the lowest face, mapped to cell 0, has
 * only its right cell and the highest face only its left one). */
void or_flux_corr_vjp(const or_config *c, const double *v, double weight, double *g) {
  long N = cells(c);
  for (int a = 0; a < 3; ++a) {
    long n = c->n[a];
    int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    long npencil = (long)c->n[b1] * c->n[b2];
    double w = weight / c->h[a];
    for (long p = 0; p < npencil; ++p) {
      long j1 = p % c->n[b1], j2 = p / c->n[b1];
      long cq[3];
      cq[b1] = j1;
      cq[b2] = j2;
      for (long fidx = 0; fidx <= n; ++fidx) {
        cq[a] = bcmap(fidx - 1, n, c->bc[a]);
        long qc = idx(c, cq[0], cq[1], cq[2]);
        for (int f = 0; f < 5; ++f) {
          double d = 0.0;
          if (fidx <= n - 1) {
            cq[a] = fidx;
            d += v[f * N + idx(c, cq[0], cq[1], cq[2])];
          }
          if (fidx >= 1) {
            cq[a] = fidx - 1;
            d -= v[f * N + idx(c, cq[0], cq[1], cq[2])];
          }
          g[f * N + qc] += w * d;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* sources                                                                    */
/* ------------------------------------------------------------------------- */

/* Reverse of the kick m' = m + rho a dt, E' = E + (m . a) dt at fixed a;
 * with accb != NULL also returns dL/da (for gravity, whose a depends on rho). */
void or_kick_vjp(const or_config *c, const double *U, const double *acc, double dt,
                 const double *lamp, double *lam, double *accb) {
  long N = cells(c);
#pragma omp parallel for schedule(static)
  for (long q = 0; q < N; ++q) {
    double rb = lamp[q], Eb = lamp[4 * N + q];
    double rho = U[q];
    for (int a = 0; a < 3; ++a) {
      double mb = lamp[(1 + a) * N + q];
      double av = acc[a * N + q];
      rb += mb * av * dt;
      lam[(1 + a) * N + q] = mb + Eb * av * dt;
      if (accb) accb[a * N + q] = mb * rho * dt + Eb * U[(1 + a) * N + q] * dt;
    }
    lam[q] = rb;
    lam[4 * N + q] = Eb;
  }
}

/* Derivatives of the exact cooling map T -> Tn(rho, T) of or_cool_temperature,
 * branch by branch (0 once floored). */
static void cool_partials(double rho, double T, double dt, double gamma, double L0, double Tc,
                          double Ts, double Tfloor, double *dT, double *drho) {
  double c2 = (gamma - 1.0) * L0 / Ts;
  double k2 = c2 * rho;
  double Tn;
  if (T >= Tc) {
    double c1 = (gamma - 1.0) * L0 / (2.0 * sqrt(Tc));
    double k1 = c1 * rho;
    double st = sqrt(T);
    double t1 = (st - sqrt(Tc)) / k1;
    if (dt <= t1) {
      double s = st - k1 * dt;
      Tn = s * s;
      *dT = s / st;
      *drho = -2.0 * s * c1 * dt;
    } else {
      double w = 1.0 + k2 * (dt - t1);
      Tn = Tc - Ts * log(w);
      /* dt1/dT = 1/(2 sqrt(T) k1), dt1/drho = -t1/rho */
      *dT = Ts * k2 / w / (2.0 * st * k1);
      *drho = -Ts / w * (c2 * (dt - t1) + k2 * t1 / rho);
    }
  } else {
    double e = exp(-(T - Tc) / Ts);
    double w = e + k2 * dt;
    Tn = Tc - Ts * log(w);
    *dT = e / w;
    *drho = -Ts / w * c2 * dt;
  }
  if (Tn < Tfloor) {
    *dT = 0.0;
    *drho = 0.0;
  }
}

/* Reverse of or_cool: E' = ek + rho Tn(rho, T)/(g-1), T = (g-1)(E - ek)/rho,
 * ek = |m|^2/(2 rho); rho and m pass through. */
void or_cool_vjp(const or_config *c, const double *U, double dt, const double *lamp,
                 double *lam) {
  long N = cells(c);
  double g = c->gamma, gm1 = g - 1.0;
  if (c->cool_model == OR_COOL_TABLE) {
    /* E' = ek + C(rho, E - ek), ek = |m|^2/(2 rho), with C the tabulated
     * model's step and its partials C_E, C_rho (oracle_cool.c) */
#pragma omp parallel for schedule(static)
    for (long q = 0; q < N; ++q) {
      double rho = U[q], mx = U[N + q], my = U[2 * N + q], mz = U[3 * N + q], E = U[4 * N + q];
      double ek = 0.5 * (mx * mx + my * my + mz * mz) / rho;
      double CE, Cr;
      or_cool_eth_step_d(c, rho, E - ek, dt, &CE, &Cr);
      double Eb = lamp[4 * N + q];
      double ekb = Eb * (1.0 - CE); /* dE'/dek */
      lam[q] = lamp[q] + Eb * Cr - ekb * ek / rho;
      lam[N + q] = lamp[N + q] + ekb * mx / rho;
      lam[2 * N + q] = lamp[2 * N + q] + ekb * my / rho;
      lam[3 * N + q] = lamp[3 * N + q] + ekb * mz / rho;
      lam[4 * N + q] = Eb * CE;
    }
    return;
  }
#pragma omp parallel for schedule(static)
  for (long q = 0; q < N; ++q) {
    double rho = U[q], mx = U[N + q], my = U[2 * N + q], mz = U[3 * N + q], E = U[4 * N + q];
    double ek = 0.5 * (mx * mx + my * my + mz * mz) / rho;
    double T = gm1 * (E - ek) / rho;
    double dT, drho;
    cool_partials(rho, T, dt, g, c->cool_lambda0, c->cool_tc, c->cool_ts, c->cool_tfloor, &dT,
                  &drho);
    double Eb = lamp[4 * N + q];
    double Tn = or_cool_temperature(rho, T, dt, g, c->cool_lambda0, c->cool_tc, c->cool_ts,
                                    c->cool_tfloor);
    /* E' = ek + rho Tn / gm1 */
    double ekb = Eb;
    double rhob = lamp[q] + Eb * Tn / gm1;
    double Tnb = Eb * rho / gm1;
    double Tb = Tnb * dT;
    rhob += Tnb * drho;
    /* T = gm1 (E - ek) / rho */
    double Ein_b = Tb * gm1 / rho;
    ekb -= Tb * gm1 / rho;
    rhob -= Tb * T / rho;
    /* ek = |m|^2 / (2 rho) */
    rhob -= ekb * ek / rho;
    lam[q] = rhob;
    lam[N + q] = lamp[N + q] + ekb * mx / rho;
    lam[2 * N + q] = lamp[2 * N + q] + ekb * my / rho;
    lam[3 * N + q] = lamp[3 * N + q] + ekb * mz / rho;
    lam[4 * N + q] = Ein_b;
  }
}

/* Reverse of the gravity step (oracle_mg.c): U' = kick(U, g(rho)), with
 * g = -grad phi, phi = A^+ F, F = 4 pi G (rho - <rho>).  The adjoint of the
 * solve is a solve with the same symmetric operator (Sec. 6.2.4), run with the
 * same multigrid settings from a zero start.  phi_scratch holds the forward
 * solution on entry (warm start for recomputing g). */
int or_gravity_vjp(const or_config *c, const double *U, double dt, double *phi,
                   const double *lamp, double *lam) {
  long n = c->n[0], N = n * n * n;
  double h = c->h[0];
  double *acc = (double *)malloc(sizeof(double) * 3 * N);
  double *accb = (double *)malloc(sizeof(double) * 3 * N);
  int cyc = or_gravity_accel(c, U, phi, acc);
  or_kick_vjp(c, U, acc, dt, lamp, lam, accb);
  if (c->grav_solver == OR_GRAV_FFT) {
    double *rhob = (double *)malloc(sizeof(double) * N);
    or_fft_gravity_vjp(c, accb, rhob);
    for (long q = 0; q < N; ++q) lam[q] += rhob[q];
    free(rhob); free(acc); free(accb);
    return cyc;
  }
  /* g_a,i = -(phi_{i+1} - phi_{i-1}) / (2h)  =>  phib_j = sum_a (gb_{a,j+1} - gb_{a,j-1}) / (2h) */
  double *phib = (double *)malloc(sizeof(double) * N);
  double i2h = 1.0 / (2.0 * h);
  for (long k = 0; k < n; ++k)
    for (long j = 0; j < n; ++j)
      for (long i = 0; i < n; ++i) {
        long ip = (i + 1) % n, im = (i + n - 1) % n, jp = (j + 1) % n, jm = (j + n - 1) % n;
        long kp = (k + 1) % n, km = (k + n - 1) % n;
        phib[(k * n + j) * n + i] =
            ((accb[(k * n + j) * n + ip] - accb[(k * n + j) * n + im]) +
             (accb[N + (k * n + jp) * n + i] - accb[N + (k * n + jm) * n + i]) +
             (accb[2 * N + (kp * n + j) * n + i] - accb[2 * N + (km * n + j) * n + i])) * i2h;
      }
  /* Fb = P0 A^+ P0 phib, then rho_b += 4 pi G P0 Fb (P0: remove the mean) */
  double *Fb = (double *)calloc(N, sizeof(double));
  double m = 0.0;
  for (long q = 0; q < N; ++q) m += phib[q];
  m /= (double)N;
  for (long q = 0; q < N; ++q) phib[q] -= m;
  or_mg_solve(c, (int)n, h, Fb, phib);
  m = 0.0;
  for (long q = 0; q < N; ++q) m += Fb[q];
  m /= (double)N;
  double fourpiG = 4.0 * M_PI * c->grav_G;
  for (long q = 0; q < N; ++q) lam[q] += fourpiG * (Fb[q] - m);
  free(acc); free(accb); free(phib); free(Fb);
  return cyc;
}

/* ------------------------------------------------------------------------- */
/* one full step                                                              */
/* ------------------------------------------------------------------------- */

/* lam_n = (dU^{n+1}/dU^n)^T lam_np1 for the step or_step(U^n, dt) taken with
 * a fixed dt, global step index `step`, the OU mode state ou_ahat *before* the
 * step (not modified) and the potential phi before the step (warm start;
 * modified). */
void or_step_vjp(const or_config *c, const double *Un, double dt, int64_t step, int nmodes,
                 const int32_t *nvec, const double *ou_ahat, double *phi,
                 const double *lam_np1, double *lam_n) {
  or_step_vjp_flux(c, Un, dt, step, nmodes, nvec, ou_ahat, phi, lam_np1, lam_n, NULL);
}

/* or_step_vjp that also accumulates the flux-correction adjoint into gflux
 * (when not NULL) */
void or_step_vjp_flux(const or_config *c, const double *Un, double dt, int64_t step, int nmodes,
                      const int32_t *nvec, const double *ou_ahat, double *phi,
                      const double *lam_np1, double *lam_n, double *gflux) {
  long N = cells(c), N5 = 5 * N;
  double *Ua = (double *)malloc(sizeof(double) * N5); /* after the RK update */
  double *Ub = (double *)malloc(sizeof(double) * N5); /* after forcing */
  double *Uc = (double *)malloc(sizeof(double) * N5); /* after gravity */
  double *acc = (double *)malloc(sizeof(double) * 3 * N);
  double *la = (double *)malloc(sizeof(double) * N5);
  double *lb = (double *)malloc(sizeof(double) * N5);
  double *ahat = (double *)malloc(sizeof(double) * 6 * (nmodes > 0 ? nmodes : 1));
  double *phi0 = (double *)malloc(sizeof(double) * N);
  memcpy(Ua, Un, sizeof(double) * N5);
  or_integrate(c, Ua, dt);
  memcpy(Ub, Ua, sizeof(double) * N5);
  int force = (c->flags & OR_SRC_FORCING) && nmodes > 0;
  if (force) {
    memcpy(ahat, ou_ahat, sizeof(double) * 6 * nmodes);
    int every = c->ou_every > 0 ? c->ou_every : 1;
    if (step % every == 0) or_ou_advance(c, nmodes, nvec, ahat, step / every, dt * every);
    or_ou_accel(c, nmodes, nvec, ahat, acc);
    or_kick(c, Ub, acc, dt);
  }
  memcpy(Uc, Ub, sizeof(double) * N5);
  if (c->flags & OR_SRC_GRAVITY) {
    memcpy(phi0, phi, sizeof(double) * N);
    double *gacc = (double *)malloc(sizeof(double) * 3 * N);
    or_gravity_accel(c, Uc, phi, gacc);
    or_kick(c, Uc, gacc, dt);
    free(gacc);
  }
  /* reverse */
  memcpy(lb, lam_np1, sizeof(double) * N5);
  if (c->flags & OR_SRC_COOLING) or_cool_vjp(c, Uc, dt, lam_np1, lb);
  memcpy(la, lb, sizeof(double) * N5);
  if (c->flags & OR_SRC_GRAVITY) or_gravity_vjp(c, Ub, dt, phi0, lb, la);
  memcpy(lb, la, sizeof(double) * N5);
  if (force) or_kick_vjp(c, Ua, acc, dt, la, lb, NULL);
  or_integrate_vjp_flux(c, Un, dt, lb, lam_n, gflux);
  free(Ua); free(Ub); free(Uc); free(acc); free(la); free(lb); free(ahat); free(phi0);
}
