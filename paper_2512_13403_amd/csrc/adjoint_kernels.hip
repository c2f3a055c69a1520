// adjoint_kernels.hip -- reverse-mode derivative of the finite-volume step
// (arXiv 2512.13403, Sec. 2.3 and 6.2.4) for gfx950.
//
// With dt held fixed, the derivative of one step U^n -> U^{n+1} is applied in
// transposed form, lam^n = (dU^{n+1}/dU^n)^T lam^{n+1}, source by source in
// reverse order and then through the two RK stages:
//   lam1 = lam_a/2 + (dt/2) J(U1)^T lam_a,   lam^n = lam_a/2 + lam1 + dt J(U^n)^T lam1.
// J(U)^T v for L(U) = -sum_a (F_{a,i+1/2} - F_{a,i-1/2}) / h_a runs in two
// deterministic passes per axis (no floating-point atomics):
//   k_face_vjp    one thread per face: Fb = (v_right - v_left)/h, the HLLC
//                 reverse sweep gives the face-state adjoints W^L_b, W^R_b, and
//                 the minmod selections of the two slopes the face used;
//   k_cell_gather one thread per cell: sums, over the (at most four) faces
//                 whose stencil reads the cell, the reverse of
//                 W^L = W_i + minmod(..)/2, W^R = W_{i+1} - minmod(..)/2;
// and k_jtv_finish applies (dW/dU)^T per cell.  At every kink the derivative
// of the branch the forward took is used (minmod: the returned argument, or 0;
// wave-speed min/max: the selected argument, the first on ties; HLLC: the
// side and fan the face fell in).  The other limiters and solvers run in
// k_face_vjp_rt, which takes them at run time and writes each face's four
// stencil contributions instead of the minmod selections: the slope partials
// dphi/da, dphi/db of van Leer (2b^2/(a+b)^2, 2a^2/(a+b)^2), MC ((1/2, 1/2),
// (2, 0) or (0, 2), ties in that order) and superbee ((2, 0), (0, 1), (1, 0)
// or (0, 2)), and the HLL / Rusanov reverse sweeps.
#include "mg.h"
#include "mh_adjoint.h"
#include "mh_device.h"

namespace mh {

namespace {

__device__ __forceinline__ int minmod_sel(float a, float b) {
  return (a * b <= 0.0f) ? 0 : (fabsf(a) <= fabsf(b) ? 1 : 2);
}
__device__ __forceinline__ int minmod_sel(double a, double b) {
  return (a * b <= 0.0) ? 0 : (fabs(a) <= fabs(b) ? 1 : 2);
}
template <typename T>
__device__ __forceinline__ T sel_value(int s, T a, T b) {
  return s == 1 ? a : (s == 2 ? b : T(0));
}

// primitive variables of cell q, with the arithmetic of the stage kernels
// (so every limiter and wave-speed branch is taken as in the forward step)
template <typename T>
__device__ __forceinline__ void prim_at(const T* __restrict__ U, long long N, long long q, T gm1,
                                        T (&w)[5]) {
  T u[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f] = U[f * N + q];
  to_prim(u, gm1, w);
}

// Reverse of the one-sided HLLC assembly of the stage kernel, for face states
// wl, wr = (rho, v_n, v_t1, v_t2, P) in the face frame.  Fb = dL/dF; writes
// dL/dwl and dL/dwr.  The forward quantities are recomputed with the stage
// kernel's own arithmetic (c = gP rsq(gP rho), S* through one reciprocal of
// rho_L(S_L - u_L) - rho_R(S_R - u_R)), so the side, fan and wave-speed
// branches are the ones the step took; the derivatives use the same
// reciprocals (dc/dP = g rsq(gP rho) / 2, dc/drho = -c / (2 rho) with
// 1/rho = gP rsq^2) instead of divisions.
template <typename T>
__device__ void hllc_reverse(const T (&wl)[5], const T (&wr)[5], T g, T gm1inv, const T (&Fb)[5],
                             T (&wlb)[5], T (&wrb)[5]) {
  const T rl = wl[0], ul = wl[1], al = wl[2], bl = wl[3], pl = wl[4];
  const T rr = wr[0], ur = wr[1], ar = wr[2], br = wr[3], pr = wr[4];
  const T gpl = g * pl, gpr = g * pr;
  const T rsl = dev_rsq(gpl * rl), rsr = dev_rsq(gpr * rr);
  const T cl = gpl * rsl, cr = gpr * rsr;
  const bool minL = (ul - cl) <= (ur - cr);
  const bool maxL = (ul + cl) >= (ur + cr);
  const T SL = minL ? ul - cl : ur - cr;
  const T SR = maxL ? ul + cl : ur + cr;
  const T kl = fmad(ul, ul, fmad(al, al, bl * bl)), kr = fmad(ur, ur, fmad(ar, ar, br * br));
  const T El = fmad(pl, gm1inv, (T(0.5) * rl) * kl);
  const T Er = fmad(pr, gm1inv, (T(0.5) * rr) * kr);
  const T dl = rl * (SL - ul), dr = rr * (SR - ur);
  const T num = fmad(-ur, dr, fmad(ul, dl, pr - pl));
  const T iden = dev_rcp(dl - dr);
  const T ss = num * iden;
  const bool left = (SL >= T(0)) || (ss >= T(0));
  const bool fan = (left ? -SL : SR) > T(0);
  const T rK = left ? rl : rr, uK = left ? ul : ur, aK = left ? al : ar, bK = left ? bl : br;
  const T pK = left ? pl : pr, EK = left ? El : Er, SK = left ? SL : SR, dK = left ? dl : dr;
  const T mK = rK * uK;

  T rKb = 0, uKb = 0, aKb = 0, bKb = 0, pKb = 0, EKb = 0, SKb = 0, dKb = 0, mKb = 0, ssb = 0;
  if (fan) {
    const T q = dev_rcp(SK - ss);
    const T qd = q * dK;
    const T H = fmad(dK, ss, pK);
    const T G4 = fmad(SK - uK, EK, (ss - uK) * H);
    const T s[5] = {qd, qd * ss, qd * aK, qd * bK, q * G4};
    const T UK[5] = {rK, mK, rK * aK, rK * bK, EK};
    T sb[5], UKb[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      SKb = fmad(Fb[f], s[f] - UK[f], SKb);
      sb[f] = SK * Fb[f];
      UKb[f] = -SK * Fb[f];
    }
    T qb = sb[4] * G4;
    const T G4b = sb[4] * q;
    SKb = fmad(G4b, EK, SKb);
    uKb = fmad(-G4b, EK, uKb);
    EKb = fmad(G4b, SK - uK, EKb);
    ssb = fmad(G4b, H, ssb);
    uKb = fmad(-G4b, H, uKb);
    const T Hb = G4b * (ss - uK);
    dKb = fmad(Hb, ss, dKb);
    ssb = fmad(Hb, dK, ssb);
    pKb += Hb;
    const T qdb = fmad(sb[3], bK, fmad(sb[2], aK, fmad(sb[1], ss, sb[0])));
    ssb = fmad(sb[1], qd, ssb);
    aKb = fmad(sb[2], qd, aKb);
    bKb = fmad(sb[3], qd, bKb);
    qb = fmad(qdb, dK, qb);
    dKb = fmad(qdb, q, dKb);
    const T Zb = -(qb * q) * q;  // q = 1/Z, Z = SK - ss
    SKb += Zb;
    ssb -= Zb;
    rKb += fmad(UKb[3], bK, fmad(UKb[2], aK, UKb[0]));
    mKb += UKb[1];
    aKb = fmad(UKb[2], rK, aKb);
    bKb = fmad(UKb[3], rK, bKb);
    EKb += UKb[4];
  }
  // F_K = (mK, mK uK + pK, mK aK, mK bK, uK (EK + pK))
  mKb += fmad(Fb[3], bK, fmad(Fb[2], aK, fmad(Fb[1], uK, Fb[0])));
  uKb += fmad(Fb[4], EK + pK, Fb[1] * mK);
  pKb += fmad(Fb[4], uK, Fb[1]);
  aKb = fmad(Fb[2], mK, aKb);
  bKb = fmad(Fb[3], mK, bKb);
  EKb = fmad(Fb[4], uK, EKb);
  rKb = fmad(mKb, uK, rKb);
  uKb = fmad(mKb, rK, uKb);

  T rlb = 0, ulb = 0, alb = 0, blb = 0, plb = 0, Elb = 0, SLb = 0, dlb = 0;
  T rrb = 0, urb = 0, arb = 0, brb = 0, prb = 0, Erb = 0, SRb = 0, drb = 0;
  if (left) {
    rlb = rKb; ulb = uKb; alb = aKb; blb = bKb; plb = pKb; Elb = EKb; SLb = SKb; dlb = dKb;
  } else {
    rrb = rKb; urb = uKb; arb = aKb; brb = bKb; prb = pKb; Erb = EKb; SRb = SKb; drb = dKb;
  }
  // ss = num / den
  const T numb = ssb * iden, denb = -(ssb * ss) * iden;
  prb += numb;
  plb -= numb;
  ulb = fmad(numb, dl, ulb);
  dlb = fmad(numb, ul, dlb);
  urb = fmad(-numb, dr, urb);
  drb = fmad(-numb, ur, drb);
  dlb += denb;
  drb -= denb;
  rlb = fmad(dlb, SL - ul, rlb);
  SLb = fmad(dlb, rl, SLb);
  ulb = fmad(-dlb, rl, ulb);
  rrb = fmad(drb, SR - ur, rrb);
  SRb = fmad(drb, rr, SRb);
  urb = fmad(-drb, rr, urb);
  plb = fmad(Elb, gm1inv, plb);
  rlb = fmad(Elb * T(0.5), kl, rlb);
  const T Elr = Elb * rl;
  ulb = fmad(Elr, ul, ulb);
  alb = fmad(Elr, al, alb);
  blb = fmad(Elr, bl, blb);
  prb = fmad(Erb, gm1inv, prb);
  rrb = fmad(Erb * T(0.5), kr, rrb);
  const T Err = Erb * rr;
  urb = fmad(Err, ur, urb);
  arb = fmad(Err, ar, arb);
  brb = fmad(Err, br, brb);
  T clb = 0, crb = 0;
  if (minL) { ulb += SLb; clb -= SLb; } else { urb += SLb; crb -= SLb; }
  if (maxL) { ulb += SRb; clb += SRb; } else { urb += SRb; crb += SRb; }
  // c = sqrt(gP / rho): dc/dP = g rsq / 2, dc/drho = -c / (2 rho), 1/rho = gP rsq^2
  plb = fmad(clb, T(0.5) * g * rsl, plb);
  rlb = fmad(-clb, (T(0.5) * cl) * (gpl * rsl * rsl), rlb);
  prb = fmad(crb, T(0.5) * g * rsr, prb);
  rrb = fmad(-crb, (T(0.5) * cr) * (gpr * rsr * rsr), rrb);
  wlb[0] = rlb; wlb[1] = ulb; wlb[2] = alb; wlb[3] = blb; wlb[4] = plb;
  wrb[0] = rrb; wrb[1] = urb; wrb[2] = arb; wrb[3] = brb; wrb[4] = prb;
}

// limited slope phi(a, b) of a run-time limiter with its partials on the
// branch taken (0 when ab <= 0)
template <typename T>
__device__ __forceinline__ T slope_partials(int lim, T a, T b, T& pa, T& pb) {
  pa = T(0);
  pb = T(0);
  if (lim == LIM_NONE || !(a * b > T(0))) return T(0);
  const T aa = fabs(a), ab = fabs(b);
  T m;
  if (lim == LIM_MINMOD) {
    if (aa <= ab) { pa = T(1); return a; }
    pb = T(1);
    return b;
  }
  if (lim == LIM_VANLEER) {
    const T s = a + b;
    const T is2 = T(1) / (s * s);
    pa = T(2) * b * b * is2;
    pb = T(2) * a * a * is2;
    return T(2) * a * b / s;
  }
  if (lim == LIM_MC) {
    const T cen = fabs(T(0.5) * (a + b)), t2 = fmin(T(2) * aa, T(2) * ab);
    if (cen <= t2) { pa = T(0.5); pb = T(0.5); m = cen; }
    else if (aa <= ab) { pa = T(2); m = T(2) * aa; }
    else { pb = T(2); m = T(2) * ab; }
  } else {  // superbee
    const T s1 = fmin(T(2) * aa, ab), s2 = fmin(aa, T(2) * ab);
    if (s1 >= s2) {
      if (T(2) * aa <= ab) pa = T(2); else pb = T(1);
      m = s1;
    } else {
      if (aa <= T(2) * ab) pa = T(1); else pb = T(2);
      m = s2;
    }
  }
  return a > T(0) ? m : -m;
}

// conserved state and flux of a face-frame primitive state (rho, v_n, v_t1,
// v_t2, P), and the reverse: wb += (dU/dw)^T Ub + (dF/dw)^T Fb
template <typename T>
__device__ __forceinline__ void frame_state_flux(const T (&w)[5], T gm1, T (&U)[5], T (&F)[5]) {
  const T r = w[0], u = w[1], a = w[2], b = w[3], p = w[4];
  const T E = p / gm1 + T(0.5) * r * (u * u + a * a + b * b);
  U[0] = r; U[1] = r * u; U[2] = r * a; U[3] = r * b; U[4] = E;
  F[0] = r * u; F[1] = r * u * u + p; F[2] = r * u * a; F[3] = r * u * b; F[4] = u * (E + p);
}
template <typename T>
__device__ __forceinline__ void frame_state_flux_reverse(const T (&w)[5], T gm1, const T (&Ub)[5],
                                                         const T (&Fb)[5], T (&wb)[5]) {
  const T r = w[0], u = w[1], a = w[2], b = w[3], p = w[4];
  const T q2 = u * u + a * a + b * b;
  const T E = p / gm1 + T(0.5) * r * q2;
  const T Eb = Ub[4] + Fb[4] * u;  // E enters U[4] and F[4]
  wb[0] += Ub[0] + Ub[1] * u + Ub[2] * a + Ub[3] * b +
           u * (Fb[0] + Fb[1] * u + Fb[2] * a + Fb[3] * b) + Eb * T(0.5) * q2;
  wb[1] += r * (Ub[1] + Fb[0] + T(2) * Fb[1] * u + Fb[2] * a + Fb[3] * b + Eb * u) +
           Fb[4] * (E + p);
  wb[2] += r * (Ub[2] + Fb[2] * u + Eb * a);
  wb[3] += r * (Ub[3] + Fb[3] * u + Eb * b);
  wb[4] += Fb[1] + Fb[4] * u + Eb / gm1;
}
// c = sqrt(g P / rho): wb += cb dc/dw
template <typename T>
__device__ __forceinline__ void sound_reverse(const T (&w)[5], T g, T c, T cb, T (&wb)[5]) {
  wb[4] += cb * g / (T(2) * c * w[0]);
  wb[0] -= cb * c / (T(2) * w[0]);
}

// Reverse of the HLL flux (F_L for 0 <= S_L, F_R for S_R <= 0, else the HLL
// average); Davis min/max take the left argument on ties.  Writes wlb, wrb.
template <typename T>
__device__ void hll_reverse(const T (&wl)[5], const T (&wr)[5], T g, const T (&Fb)[5],
                            T (&wlb)[5], T (&wrb)[5]) {
  const T gm1 = g - T(1);
  T UL[5], FL[5], UR[5], FR[5];
  frame_state_flux(wl, gm1, UL, FL);
  frame_state_flux(wr, gm1, UR, FR);
  const T cl = sqrt(g * wl[4] / wl[0]), cr = sqrt(g * wr[4] / wr[0]);
  const bool minL = (wl[1] - cl) <= (wr[1] - cr);
  const bool maxL = (wl[1] + cl) >= (wr[1] + cr);
  const T SL = minL ? wl[1] - cl : wr[1] - cr;
  const T SR = maxL ? wl[1] + cl : wr[1] + cr;
  T ULb[5], FLb[5], URb[5], FRb[5];
  T SLb = T(0), SRb = T(0);
  const bool lo = T(0) <= SL, hi = !lo && SR <= T(0);
  const T iD = T(1) / (SR - SL);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    wlb[f] = T(0);
    wrb[f] = T(0);
    if (lo || hi) {
      FLb[f] = lo ? Fb[f] : T(0);
      FRb[f] = hi ? Fb[f] : T(0);
      ULb[f] = URb[f] = T(0);
    } else {
      const T dU = UR[f] - UL[f];
      const T Fm = (SR * FL[f] - SL * FR[f] + SL * SR * dU) * iD;
      FLb[f] = Fb[f] * SR * iD;
      FRb[f] = -Fb[f] * SL * iD;
      URb[f] = Fb[f] * SL * SR * iD;
      ULb[f] = -URb[f];
      SLb += Fb[f] * (SR * dU - FR[f] + Fm) * iD;
      SRb += Fb[f] * (FL[f] + SL * dU - Fm) * iD;
    }
  }
  T clb = T(0), crb = T(0);
  if (minL) { wlb[1] += SLb; clb -= SLb; } else { wrb[1] += SLb; crb -= SLb; }
  if (maxL) { wlb[1] += SRb; clb += SRb; } else { wrb[1] += SRb; crb += SRb; }
  sound_reverse(wl, g, cl, clb, wlb);
  sound_reverse(wr, g, cr, crb, wrb);
  frame_state_flux_reverse(wl, gm1, ULb, FLb, wlb);
  frame_state_flux_reverse(wr, gm1, URb, FRb, wrb);
}

// Reverse of the Rusanov flux (F_L + F_R)/2 - s (U_R - U_L)/2, s = max(|v_L|
// + c_L, |v_R| + c_R): the left argument on ties, d|v|/dv = -1 for v < 0,
// else +1.  Writes wlb, wrb.
template <typename T>
__device__ void rusanov_reverse(const T (&wl)[5], const T (&wr)[5], T g, const T (&Fb)[5],
                                T (&wlb)[5], T (&wrb)[5]) {
  const T gm1 = g - T(1);
  T UL[5], FL[5], UR[5], FR[5];
  frame_state_flux(wl, gm1, UL, FL);
  frame_state_flux(wr, gm1, UR, FR);
  const T cl = sqrt(g * wl[4] / wl[0]), cr = sqrt(g * wr[4] / wr[0]);
  const bool maxL = (fabs(wl[1]) + cl) >= (fabs(wr[1]) + cr);
  const T s = maxL ? fabs(wl[1]) + cl : fabs(wr[1]) + cr;
  T ULb[5], FLb[5], URb[5], FRb[5];
  T sb = T(0);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    wlb[f] = T(0);
    wrb[f] = T(0);
    FLb[f] = FRb[f] = T(0.5) * Fb[f];
    URb[f] = -T(0.5) * s * Fb[f];
    ULb[f] = -URb[f];
    sb -= T(0.5) * Fb[f] * (UR[f] - UL[f]);
  }
  T clb = T(0), crb = T(0);
  if (maxL) {
    wlb[1] += wl[1] < T(0) ? -sb : sb;
    clb = sb;
  } else {
    wrb[1] += wr[1] < T(0) ? -sb : sb;
    crb = sb;
  }
  sound_reverse(wl, g, cl, clb, wlb);
  sound_reverse(wr, g, cr, crb, wrb);
  frame_state_flux_reverse(wl, gm1, ULb, FLb, wlb);
  frame_state_flux_reverse(wr, gm1, URb, FRb, wrb);
}

struct AxisGeom {
  int n[3];   // cells along x, y, z
  int bc;     // boundary kind of the axis
  int nf;     // faces along the axis: n (periodic) or n + 1 (outflow)
};

// cell index of (along-axis coordinate c, the other two coordinates) and the
// face record index of (face f along the axis, the other two coordinates)
template <int AX>
__device__ __forceinline__ long long cell_of(const AxisGeom& g, int c, int o1, int o2) {
  if (AX == 0) return ((long long)o2 * g.n[1] + o1) * g.n[0] + c;
  if (AX == 1) return ((long long)o2 * g.n[1] + c) * g.n[0] + o1;
  return ((long long)c * g.n[1] + o2) * g.n[0] + o1;
}
template <int AX>
__device__ __forceinline__ long long face_of(const AxisGeom& g, int f, int o1, int o2) {
  if (AX == 0) return ((long long)o2 * g.n[1] + o1) * g.nf + f;
  if (AX == 1) return ((long long)o2 * g.nf + f) * g.n[0] + o1;
  return ((long long)f * g.n[1] + o2) * g.n[0] + o1;
}
// the inverses: thread t takes face record t and cell t, so that consecutive
// lanes touch consecutive addresses (x fastest) along every axis
template <int AX>
__device__ __forceinline__ void face_coords(const AxisGeom& g, long long t, int& f, int& o1,
                                            int& o2) {
  if (AX == 0) {
    f = (int)(t % g.nf);
    const long long r = t / g.nf;
    o1 = (int)(r % g.n[1]);
    o2 = (int)(r / g.n[1]);
  } else if (AX == 1) {
    o1 = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    f = (int)(r % g.nf);
    o2 = (int)(r / g.nf);
  } else {
    o1 = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    o2 = (int)(r % g.n[1]);
    f = (int)(r / g.n[1]);
  }
}
template <int AX>
__device__ __forceinline__ void cell_coords(const AxisGeom& g, long long t, int& c, int& o1,
                                            int& o2) {
  if (AX == 0) {
    c = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    o1 = (int)(r % g.n[1]);
    o2 = (int)(r / g.n[1]);
  } else if (AX == 1) {
    o1 = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    c = (int)(r % g.n[1]);
    o2 = (int)(r / g.n[1]);
  } else {
    o1 = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    o2 = (int)(r % g.n[1]);
    c = (int)(r / g.n[1]);
  }
}
// the two other coordinates of axis AX: AX=0 -> (y, z), AX=1 -> (x, z), AX=2 -> (x, y)
template <int AX>
__device__ __forceinline__ void other_dims(const AxisGeom& g, int& d1, int& d2) {
  d1 = AX == 0 ? g.n[1] : g.n[0];
  d2 = AX == 2 ? g.n[1] : g.n[2];
}

template <typename T, int LIM, int AX>
__global__ __launch_bounds__(256) void k_face_vjp(const T* __restrict__ U, const T* __restrict__ v,
                                                  AxisGeom g, T gamma, T ih, T* __restrict__ wbar,
                                                  int* __restrict__ flags, long long nfaces) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nfaces) return;
  int d1, d2;
  other_dims<AX>(g, d1, d2);
  int f, o1, o2;
  face_coords<AX>(g, t, f, o1, o2);
  const int n = g.n[AX];
  const int i = g.bc == BC_PERIODIC ? f : f - 1;  // left cell position of the face
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const T gm1 = gamma - T(1);
  const T gm1inv = T(1) / gm1;
  constexpr int vn = 1 + AX, t1 = 1 + (AX + 1) % 3, t2 = 1 + (AX + 2) % 3;
  const int perm[5] = {0, vn, t1, t2, 4};
  T w[4][5];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T wc[5];
    prim_at(U, N, cell_of<AX>(g, bc_map(i - 1 + k, n, g.bc), o1, o2), gm1, wc);
#pragma unroll
    for (int s = 0; s < 5; ++s) w[k][s] = wc[perm[s]];
  }
  T wl[5], wr[5];
  int fl = 0;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const T a0 = w[2][s] - w[1][s], b0 = w[1][s] - w[0][s];
    const T a1 = w[3][s] - w[2][s], b1 = w[2][s] - w[1][s];
    const int s0 = LIM == LIM_NONE ? 0 : minmod_sel(a0, b0);
    const int s1 = LIM == LIM_NONE ? 0 : minmod_sel(a1, b1);
    wl[s] = w[1][s] + T(0.5) * sel_value(s0, a0, b0);
    wr[s] = w[2][s] - T(0.5) * sel_value(s1, a1, b1);
    fl |= (s0 << (2 * s)) | (s1 << (10 + 2 * s));
  }
  // Fb = (v of the face's right cell - v of its left cell) / h, real cells only
  const bool has_right = g.bc == BC_PERIODIC || i + 1 <= n - 1;
  const bool has_left = g.bc == BC_PERIODIC || i >= 0;
  const long long qr = cell_of<AX>(g, bc_map(i + 1, n, g.bc), o1, o2);
  const long long ql = cell_of<AX>(g, bc_map(i, n, g.bc), o1, o2);
  T Fb[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const T vr = has_right ? v[perm[s] * N + qr] : T(0);
    const T vl = has_left ? v[perm[s] * N + ql] : T(0);
    Fb[s] = (vr - vl) * ih;
  }
  T wlb[5], wrb[5];
  hllc_reverse<T>(wl, wr, gamma, gm1inv, Fb, wlb, wrb);
  const long long rec = face_of<AX>(g, f, o1, o2);
  const long long NF = (long long)g.nf * d1 * d2;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    wbar[s * NF + rec] = wlb[s];
    wbar[(5 + s) * NF + rec] = wrb[s];
  }
  flags[rec] = fl;
}

// The same for a run-time limiter `lim` and solver `rs`: writes the face's
// contributions to the W adjoint of its four stencil cells i-1+k (k = 0..3),
// per face-frame field s, to slots[(5 k + s) NF + rec]:
//   k = 0: -pb0 WLb/2
//   k = 1: WLb (1 + (pb0 - pa0)/2) + pb1 WRb/2
//   k = 2: pa0 WLb/2 + WRb (1 - (pb1 - pa1)/2)
//   k = 3: -pa1 WRb/2
// from W^L = W_i + phi(a0, b0)/2, W^R = W_{i+1} - phi(a1, b1)/2.
template <typename T, int AX>
__global__ __launch_bounds__(256) void k_face_vjp_rt(const T* __restrict__ U,
                                                     const T* __restrict__ v, AxisGeom g, T gamma,
                                                     T ih, int lim, int rs,
                                                     T* __restrict__ slots, long long nfaces) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nfaces) return;
  int d1, d2;
  other_dims<AX>(g, d1, d2);
  int f, o1, o2;
  face_coords<AX>(g, t, f, o1, o2);
  const int n = g.n[AX];
  const int i = g.bc == BC_PERIODIC ? f : f - 1;
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const T gm1 = gamma - T(1);
  const T gm1inv = T(1) / gm1;
  constexpr int vn = 1 + AX, t1 = 1 + (AX + 1) % 3, t2 = 1 + (AX + 2) % 3;
  const int perm[5] = {0, vn, t1, t2, 4};
  T w[4][5];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T wc[5];
    prim_at(U, N, cell_of<AX>(g, bc_map(i - 1 + k, n, g.bc), o1, o2), gm1, wc);
#pragma unroll
    for (int s = 0; s < 5; ++s) w[k][s] = wc[perm[s]];
  }
  T wl[5], wr[5], pa0[5], pb0[5], pa1[5], pb1[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const T d0 = slope_partials(lim, w[2][s] - w[1][s], w[1][s] - w[0][s], pa0[s], pb0[s]);
    const T d1 = slope_partials(lim, w[3][s] - w[2][s], w[2][s] - w[1][s], pa1[s], pb1[s]);
    wl[s] = w[1][s] + T(0.5) * d0;
    wr[s] = w[2][s] - T(0.5) * d1;
  }
  const bool has_right = g.bc == BC_PERIODIC || i + 1 <= n - 1;
  const bool has_left = g.bc == BC_PERIODIC || i >= 0;
  const long long qr = cell_of<AX>(g, bc_map(i + 1, n, g.bc), o1, o2);
  const long long ql = cell_of<AX>(g, bc_map(i, n, g.bc), o1, o2);
  T Fb[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const T vr = has_right ? v[perm[s] * N + qr] : T(0);
    const T vl = has_left ? v[perm[s] * N + ql] : T(0);
    Fb[s] = (vr - vl) * ih;
  }
  T wlb[5], wrb[5];
  if (rs == RS_HLL) hll_reverse<T>(wl, wr, gamma, Fb, wlb, wrb);
  else if (rs == RS_RUSANOV) rusanov_reverse<T>(wl, wr, gamma, Fb, wlb, wrb);
  else hllc_reverse<T>(wl, wr, gamma, gm1inv, Fb, wlb, wrb);
  const long long rec = face_of<AX>(g, f, o1, o2);
  const long long NF = (long long)g.nf * d1 * d2;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const T L = wlb[s], R = wrb[s];
    slots[(0 + s) * NF + rec] = -T(0.5) * pb0[s] * L;
    slots[(5 + s) * NF + rec] = L + T(0.5) * (pb0[s] - pa0[s]) * L + T(0.5) * pb1[s] * R;
    slots[(10 + s) * NF + rec] = T(0.5) * pa0[s] * L + R - T(0.5) * (pb1[s] - pa1[s]) * R;
    slots[(15 + s) * NF + rec] = -T(0.5) * pa1[s] * R;
  }
}

// contribution of the face with left cell position i to the stencil slot k
// (position i - 1 + k), field s (face frame), from the reverse of
// W^L = W_i + minmod_i/2 and W^R = W_{i+1} - minmod_{i+1}/2
template <typename T>
__device__ __forceinline__ T slot_contrib(int k, int fl, int s, T WLb, T WRb) {
  // selection codes of the two slopes (1: forward difference, 2: backward,
  // 0: none); every term is a signed half of WLb or WRb or zero, so selects
  // give the same sums as multiplying by the 0/1 indicators
  const int s0 = (fl >> (2 * s)) & 3, s1 = (fl >> (10 + 2 * s)) & 3;
  const T hl = T(0.5) * WLb, hr = T(0.5) * WRb;
  switch (k) {
    case 0: return s0 == 2 ? -hl : T(0);
    case 1: return (WLb + (s0 == 2 ? hl : (s0 == 1 ? -hl : T(0)))) + (s1 == 2 ? hr : T(0));
    case 2: return ((s0 == 1 ? hl : T(0)) + WRb) + (s1 == 2 ? -hr : (s1 == 1 ? hr : T(0)));
    default: return s1 == 1 ? -hr : T(0);
  }
}

// out = c0 x0 + c1 x1 + c2 x2 + beta (dW/dU)^T w at cell q, W = (rho, v, P)
// of U (the last step of J(U)^T v)
template <typename T>
struct FinishArgs {
  T gm1, beta, c0, c1, c2;
  const T *x0, *x1, *x2;
  T* out;
};
template <typename T>
__device__ __forceinline__ void finish_cell(const T* __restrict__ U, const T (&w)[5], long long q,
                                            long long N, const FinishArgs<T>& fa) {
  const T rho = U[q];
  const T ir = dev_rcp(rho);
  const T vx = U[N + q] * ir, vy = U[2 * N + q] * ir, vz = U[3 * N + q] * ir;
  const T wr = w[0], wx = w[1], wy = w[2], wz = w[3], wp = w[4];
  const T gm1 = fa.gm1;
  T g[5];
  g[0] = wr - (wx * vx + wy * vy + wz * vz) * ir + wp * gm1 * T(0.5) * (vx * vx + vy * vy + vz * vz);
  g[1] = wx * ir - wp * gm1 * vx;
  g[2] = wy * ir - wp * gm1 * vy;
  g[3] = wz * ir - wp * gm1 * vz;
  g[4] = wp * gm1;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    T o = fa.beta * g[f];
    if (fa.x0) o += fa.c0 * fa.x0[f * N + q];
    if (fa.x1) o += fa.c1 * fa.x1[f * N + q];
    if (fa.x2) o += fa.c2 * fa.x2[f * N + q];
    fa.out[f * N + q] = o;
  }
}

// what a gather does with its sum: add it to Wacc, store it to Wacc (the
// first axis), or add Wacc and finish the cell (the last axis; FIRST_LAST when
// it is the only one)
enum : int { GATHER_ADD = 0, GATHER_FIRST = 1, GATHER_LAST = 2, GATHER_FIRST_LAST = 3 };

// SLOTS: the face records are the four stencil contributions written by
// k_face_vjp_rt; otherwise (W^L_b, W^R_b) and the minmod selections
template <typename T, int AX, bool SLOTS, int MODE>
__global__ __launch_bounds__(256) void k_cell_gather(const T* __restrict__ wbar,
                                                     const int* __restrict__ flags, AxisGeom g,
                                                     T* __restrict__ Wacc,
                                                     const T* __restrict__ U, FinishArgs<T> fa) {
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  int d1, d2;
  other_dims<AX>(g, d1, d2);
  const int n = g.n[AX];
  int c, o1, o2;
  cell_coords<AX>(g, t, c, o1, o2);
  const long long NF = (long long)g.nf * d1 * d2;
  constexpr int vn = 1 + AX, t1 = 1 + (AX + 1) % 3, t2 = 1 + (AX + 2) % 3;
  const int perm[5] = {0, vn, t1, t2, 4};
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
  auto add_face = [&](int f, int i) {  // record f, left cell position i
    const long long rec = face_of<AX>(g, f, o1, o2);
    const int fl = SLOTS ? 0 : flags[rec];
    for (int k = 0; k < 4; ++k) {
      if (bc_map(i - 1 + k, n, g.bc) != c) continue;
#pragma unroll
      for (int s = 0; s < 5; ++s)
        acc[s] += SLOTS ? wbar[(5 * k + s) * NF + rec]
                        : slot_contrib<T>(k, fl, s, wbar[s * NF + rec], wbar[(5 + s) * NF + rec]);
    }
  };
  if (g.bc == BC_PERIODIC && n >= 4) {
    // face c - 2 + m (wrapped) holds this cell in stencil slot k = 3 - m, so
    // every record is loaded before any sum (the slot known at compile time);
    // slot 3 reads only W^R_b, slot 0 only W^L_b; sums in face order
    long long rec[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = c - 2 + m;
      rec[m] = face_of<AX>(g, i < 0 ? i + n : (i >= n ? i - n : i), o1, o2);
    }
    int fl[4];
    T wl[4][5], wr[4][5];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      fl[m] = SLOTS ? 0 : flags[rec[m]];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        if (SLOTS) {
          wl[m][s] = wbar[(5 * (3 - m) + s) * NF + rec[m]];
          wr[m][s] = T(0);
        } else {
          wl[m][s] = m >= 1 ? wbar[s * NF + rec[m]] : T(0);
          wr[m][s] = m <= 2 ? wbar[(5 + s) * NF + rec[m]] : T(0);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int s = 0; s < 5; ++s)
        acc[s] += SLOTS ? wl[m][s] : slot_contrib<T>(3 - m, fl[m], s, wl[m][s], wr[m][s]);
  } else if (g.bc == BC_PERIODIC) {
    for (int f = 0; f < n; ++f) add_face(f, f);
  } else {
    for (int i = max(-1, c - 2); i <= min(n - 1, c + 1); ++i) add_face(i + 1, i);
  }
  const long long q = cell_of<AX>(g, c, o1, o2);
  if (MODE == GATHER_ADD) {
#pragma unroll
    for (int s = 0; s < 5; ++s) Wacc[perm[s] * N + q] += acc[s];
  } else if (MODE == GATHER_FIRST) {
#pragma unroll
    for (int s = 0; s < 5; ++s) Wacc[perm[s] * N + q] = acc[s];
  } else {
    T w[5];
#pragma unroll
    for (int s = 0; s < 5; ++s)
      w[perm[s]] = MODE == GATHER_LAST ? Wacc[perm[s] * N + q] + acc[s] : acc[s];
    finish_cell(U, w, q, N, fa);
  }
}

// J(U)^T v along axis AX = 1 or 2 for periodic boundaries (n >= 4) and the
// minmod (or first-order) HLLC scheme, face reverse and gather fused: one
// thread per (x, other) column and segment of `seg` cells along the axis
// marches the faces c0 - 2 .. c1 in order, reverses each with the arithmetic
// of k_face_vjp and adds its four stencil contributions (slot_contrib) to a
// ring of four cell accumulators.  Once face f is done, cell f - 1 has all of
// its faces (f - 3 .. f, the order in which k_cell_gather sums them, so the
// result is bitwise the same) and leaves the ring: stored, added to or
// finished as in k_cell_gather's MODE.  Lanes take consecutive x, so every
// load and store of a wave is contiguous, and the face records never leave
// registers (the two-kernel path writes and reads 44 B per face).
template <typename T, int LIM, int AX, int MODE>
__global__ __launch_bounds__(256) void k_axis_jtv(const T* __restrict__ U, const T* __restrict__ v,
                                                  AxisGeom g, T gamma, T ih, int seg,
                                                  T* __restrict__ Wacc, FinishArgs<T> fa) {
  static_assert(AX == 1 || AX == 2, "columns along y or z");
  int d1, d2;
  other_dims<AX>(g, d1, d2);
  const int n = g.n[AX];
  const int nseg = (n + seg - 1) / seg;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)d1 * d2 * nseg) return;
  const int o1 = (int)(t % d1);
  const long long r = t / d1;
  const int o2 = (int)(r % d2), sg = (int)(r / d2);
  const int c0 = sg * seg, c1 = min(c0 + seg, n);
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const T gm1 = gamma - T(1);
  const T gm1inv = T(1) / gm1;
  constexpr int vn = 1 + AX, t1 = 1 + (AX + 1) % 3, t2 = 1 + (AX + 2) % 3;
  const int perm[5] = {0, vn, t1, t2, 4};
  auto wrapc = [&](int c) { return c < 0 ? c + n : (c >= n ? c - n : c); };
  auto load_w = [&](int c, T (&out)[5]) {
    T wc[5];
    prim_at(U, N, cell_of<AX>(g, wrapc(c), o1, o2), gm1, wc);
#pragma unroll
    for (int s = 0; s < 5; ++s) out[s] = wc[perm[s]];
  };
  auto load_v = [&](int c, T (&out)[5]) {
    const long long q = cell_of<AX>(g, wrapc(c), o1, o2);
#pragma unroll
    for (int s = 0; s < 5; ++s) out[s] = v[perm[s] * N + q];
  };
  // stencil of face f: cells f - 1 .. f + 2; v of its left and right cells
  T w[4][5], vl[5], vr[5];
#pragma unroll
  for (int k = 0; k < 4; ++k) load_w(c0 - 3 + k, w[k]);
  load_v(c0 - 2, vl);
  load_v(c0 - 1, vr);
  // accumulators of cells f - 1 .. f + 2
  T acc[4][5];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int s = 0; s < 5; ++s) acc[k][s] = T(0);
  for (int f = c0 - 2; f <= c1; ++f) {
    T wl[5], wr[5];
    int fl = 0;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const T a0 = w[2][s] - w[1][s], b0 = w[1][s] - w[0][s];
      const T a1 = w[3][s] - w[2][s], b1 = w[2][s] - w[1][s];
      const int s0 = LIM == LIM_NONE ? 0 : minmod_sel(a0, b0);
      const int s1 = LIM == LIM_NONE ? 0 : minmod_sel(a1, b1);
      wl[s] = w[1][s] + T(0.5) * sel_value(s0, a0, b0);
      wr[s] = w[2][s] - T(0.5) * sel_value(s1, a1, b1);
      fl |= (s0 << (2 * s)) | (s1 << (10 + 2 * s));
    }
    T Fb[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) Fb[s] = (vr[s] - vl[s]) * ih;
    T wlb[5], wrb[5];
    hllc_reverse<T>(wl, wr, gamma, gm1inv, Fb, wlb, wrb);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int s = 0; s < 5; ++s) acc[k][s] += slot_contrib<T>(k, fl, s, wlb[s], wrb[s]);
    // cell f - 1 is complete
    if (f - 1 >= c0) {
      const long long q = cell_of<AX>(g, f - 1, o1, o2);
      if (MODE == GATHER_ADD) {
#pragma unroll
        for (int s = 0; s < 5; ++s) Wacc[perm[s] * N + q] += acc[0][s];
      } else if (MODE == GATHER_FIRST) {
#pragma unroll
        for (int s = 0; s < 5; ++s) Wacc[perm[s] * N + q] = acc[0][s];
      } else {
        T wc[5];
#pragma unroll
        for (int s = 0; s < 5; ++s)
          wc[perm[s]] = MODE == GATHER_LAST ? Wacc[perm[s] * N + q] + acc[0][s] : acc[0][s];
        finish_cell(U, wc, q, N, fa);
      }
    }
    if (f == c1) break;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      acc[0][s] = acc[1][s];
      acc[1][s] = acc[2][s];
      acc[2][s] = acc[3][s];
      acc[3][s] = T(0);
      w[0][s] = w[1][s];
      w[1][s] = w[2][s];
      w[2][s] = w[3][s];
      vl[s] = vr[s];
    }
    load_w(f + 3, w[3]);
    load_v(f + 2, vr);
  }
}

// J(U)^T v along x for periodic boundaries (nx >= 4) and the minmod (or
// first-order) HLLC scheme, face reverse and gather fused: each wave takes a
// segment of XSEG = 61 cells of one x row; lane L reverses the face between
// cells x0 - 2 + L and x0 - 1 + L (the arithmetic of k_face_vjp) and puts its
// four stencil contributions (slot_contrib) in LDS, and lane L = 2 .. 62
// sums, for cell x0 + L - 2, the contributions of the faces on lanes L - 2 ..
// L + 1 in that order (the order of k_cell_gather: bitwise the same result)
// and stores, adds or finishes it as in k_cell_gather's MODE.  Three faces in
// 64 are computed twice (by two segments); the face records stay in LDS.
constexpr int XSEG = 61;

template <typename T, int LIM, int MODE>
__global__ __launch_bounds__(256) void k_x_jtv(const T* __restrict__ U, const T* __restrict__ v,
                                               AxisGeom g, T gamma, T ih, T* __restrict__ Wacc,
                                               FinishArgs<T> fa) {
  __shared__ T sc[4][20][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = g.n[0];
  const int nseg = (n + XSEG - 1) / XSEG;
  const long long wave = (long long)blockIdx.x * 4 + wv;
  const long long nrows = (long long)g.n[1] * g.n[2];
  const bool active = wave < nrows * nseg;
  const int sg = (int)(wave % nseg);
  const long long row = active ? wave / nseg : 0;
  const int o1 = (int)(row % g.n[1]), o2 = (int)(row / g.n[1]);
  const int x0 = sg * XSEG;
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const T gm1 = gamma - T(1);
  const T gm1inv = T(1) / gm1;
  auto wrapc = [&](int c) {
    c %= n;
    return c < 0 ? c + n : c;
  };
  if (active) {
    const int f = x0 - 2 + lane;  // the face between cells f and f + 1
    T w[4][5];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      prim_at(U, N, cell_of<0>(g, wrapc(f - 1 + k), o1, o2), gm1, w[k]);
    T wl[5], wr[5];
    int fl = 0;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const T a0 = w[2][s] - w[1][s], b0 = w[1][s] - w[0][s];
      const T a1 = w[3][s] - w[2][s], b1 = w[2][s] - w[1][s];
      const int s0 = LIM == LIM_NONE ? 0 : minmod_sel(a0, b0);
      const int s1 = LIM == LIM_NONE ? 0 : minmod_sel(a1, b1);
      wl[s] = w[1][s] + T(0.5) * sel_value(s0, a0, b0);
      wr[s] = w[2][s] - T(0.5) * sel_value(s1, a1, b1);
      fl |= (s0 << (2 * s)) | (s1 << (10 + 2 * s));
    }
    const long long ql = cell_of<0>(g, wrapc(f), o1, o2);
    const long long qr = cell_of<0>(g, wrapc(f + 1), o1, o2);
    T Fb[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) Fb[s] = (v[s * N + qr] - v[s * N + ql]) * ih;
    T wlb[5], wrb[5];
    hllc_reverse<T>(wl, wr, gamma, gm1inv, Fb, wlb, wrb);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int s = 0; s < 5; ++s) sc[wv][5 * k + s][lane] = slot_contrib<T>(k, fl, s, wlb[s], wrb[s]);
  }
  __syncthreads();
  const int c = x0 + lane - 2;
  if (!active || lane < 2 || lane > 62 || c >= n) return;
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int s = 0; s < 5; ++s) acc[s] += sc[wv][5 * (3 - m) + s][lane - 2 + m];
  const long long q = cell_of<0>(g, c, o1, o2);
  if (MODE == GATHER_ADD) {
#pragma unroll
    for (int s = 0; s < 5; ++s) Wacc[s * N + q] += acc[s];
  } else if (MODE == GATHER_FIRST) {
#pragma unroll
    for (int s = 0; s < 5; ++s) Wacc[s * N + q] = acc[s];
  } else {
    T wc[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) wc[s] = MODE == GATHER_LAST ? Wacc[s * N + q] + acc[s] : acc[s];
    finish_cell(U, wc, q, N, fa);
  }
}

// out = c0 x0 + c1 x1 + c2 x2 + beta (dW/dU)^T Wacc, W = (rho, v, P) of U
template <typename T>
__global__ __launch_bounds__(256) void k_jtv_finish(const T* __restrict__ U,
                                                    const T* __restrict__ Wacc, long long N,
                                                    FinishArgs<T> fa) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  T w[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) w[f] = Wacc[f * N + q];
  finish_cell(U, w, q, N, fa);
}

// g += weight (dL/dB)^T v for the flux-correction field B (B at a cell is
// added to the flux through its upper face on each axis a; a face's flux
// leaves the cell below with -1/h_a and enters the cell above with +1/h_a):
// per axis, d = v(i+1) - v(i), with v beyond the last cell 0 for outflow
// (periodic: wrapped), plus v(0) at the first cell with outflow, whose B
// also sits on the face below it
template <typename T>
__global__ __launch_bounds__(256) void k_flux_corr_vjp(const T* __restrict__ v, int nx, int ny,
                                                       int nz, int bcx, int bcy, int bcz, T wx,
                                                       T wy, T wz, T* g) {
  const long long N = (long long)nx * ny * nz;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
  const long long sx = 1, sy = nx, sz = (long long)nx * ny;
  const int n[3] = {nx, ny, nz}, c[3] = {i, j, k}, bc[3] = {bcx, bcy, bcz};
  const long long st[3] = {sx, sy, sz};
  const T w[3] = {wx, wy, wz};
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T* vf = v + f * N;
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T up;
      if (c[a] + 1 < n[a]) up = vf[q + st[a]];
      else up = bc[a] == BC_PERIODIC ? vf[q - (long long)(n[a] - 1) * st[a]] : T(0);
      T d = up - vf[q];
      if (bc[a] != BC_PERIODIC && c[a] == 0) d += vf[q];
      acc += w[a] * d;
    }
    g[f * N + q] += acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* y, long long n, T v) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) y[q] = v;
}

// ---------------------------------------------------------------- sources

// OU acceleration at (x, y, z) from the row records and X phase factors,
// the same separable sum the stage kernel evaluates
template <typename T>
__device__ __forceinline__ void ou_accel(const T* __restrict__ rows, const T* __restrict__ tabx,
                                         int R, int nx, int ny, int x, int y, int z, T (&a)[3]) {
  const T* pq = rows + ((long long)z * ny + y) * 6 * (R + 1);
#pragma unroll
  for (int c = 0; c < 3; ++c) a[c] = pq[2 * c];
  for (int n = 1; n <= R; ++n) {
    const T xr = tabx[2 * ((long long)n * nx + x)], xi = tabx[2 * ((long long)n * nx + x) + 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] += xr * pq[6 * n + 2 * c] - xi * pq[6 * n + 2 * c + 1];
  }
}

// reverse of the kick m += rho a dt, E += (m_old . a) dt (the acceleration
// does not depend on the state): lam_rho += sum_c lam_m_c a_c dt,
// lam_m_c += lam_E a_c dt
template <typename T>
__device__ __forceinline__ void kick_vjp_cell(const T (&a)[3], T dt, const T (&li)[5],
                                              T (&lo)[5]) {
  const T Eb = li[4];
  T rb = li[0];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T mb = li[1 + c];
    rb += mb * a[c] * dt;
    lo[1 + c] = mb + Eb * a[c] * dt;
  }
  lo[0] = rb;
  lo[4] = Eb;
}

template <typename T>
__global__ __launch_bounds__(256) void k_force_kick_vjp(const T* __restrict__ rows,
                                                        const T* __restrict__ tabx, int R, int nx,
                                                        int ny, int nz, T dt,
                                                        const T* __restrict__ lin, T* lout) {
  const long long N = (long long)nx * ny * nz;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int x = (int)(q % nx), y = (int)((q / nx) % ny), z = (int)(q / ((long long)nx * ny));
  T a[3];
  ou_accel(rows, tabx, R, nx, ny, x, y, z, a);
  T li[5], lo[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) li[f] = lin[f * N + q];
  kick_vjp_cell(a, dt, li, lo);
#pragma unroll
  for (int f = 0; f < 5; ++f) lout[f * N + q] = lo[f];
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// reverse of the gravity kick at U (before the kick) with g = -grad phi:
// lam as for any kick, and accb_c = lam_m_c rho dt + lam_E m_c dt
template <typename T>
__global__ __launch_bounds__(256) void k_grav_kick_vjp(const T* __restrict__ U,
                                                       const T* __restrict__ phi, int n, T i2h,
                                                       T dt, const T* __restrict__ lin, T* lout,
                                                       T* __restrict__ accb) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((long long)n * n));
  const long long n2 = (long long)n * n;
  const long long row = (long long)k * n2 + (long long)j * n;
  T a[3];
  a[0] = -(phi[row + wrapi(i + 1, n)] - phi[row + wrapi(i - 1, n)]) * i2h;
  a[1] = -(phi[(long long)k * n2 + (long long)wrapi(j + 1, n) * n + i] -
           phi[(long long)k * n2 + (long long)wrapi(j - 1, n) * n + i]) * i2h;
  a[2] = -(phi[(long long)wrapi(k + 1, n) * n2 + (long long)j * n + i] -
           phi[(long long)wrapi(k - 1, n) * n2 + (long long)j * n + i]) * i2h;
  const T rho = U[q], Eb = lin[4 * N + q];
  T rb = lin[q];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T mb = lin[(1 + c) * N + q];
    rb += mb * a[c] * dt;
    lout[(1 + c) * N + q] = mb + Eb * a[c] * dt;
    accb[c * N + q] = mb * rho * dt + Eb * U[(1 + c) * N + q] * dt;
  }
  lout[q] = rb;
  lout[4 * N + q] = Eb;
}

// reverse of g_c,i = -(phi_{i+1} - phi_{i-1}) / (2h): phib_j = sum_c (accb_c,j+1 - accb_c,j-1) / (2h)
template <typename T>
__global__ __launch_bounds__(256) void k_grad_adjoint(const T* __restrict__ accb, int n, T i2h,
                                                      T* __restrict__ phib) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((long long)n * n));
  const long long n2 = (long long)n * n;
  const long long row = (long long)k * n2 + (long long)j * n;
  phib[q] = ((accb[row + wrapi(i + 1, n)] - accb[row + wrapi(i - 1, n)]) +
             (accb[N + (long long)k * n2 + (long long)wrapi(j + 1, n) * n + i] -
              accb[N + (long long)k * n2 + (long long)wrapi(j - 1, n) * n + i]) +
             (accb[2 * N + (long long)wrapi(k + 1, n) * n2 + (long long)j * n + i] -
              accb[2 * N + (long long)wrapi(k - 1, n) * n2 + (long long)j * n + i])) * i2h;
}

// lam_rho += s x
template <typename T>
__global__ __launch_bounds__(256) void k_axpy(T* y, const T* __restrict__ x, long long n, T s) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) y[q] += s * x[q];
}

// reverse of exact cooling E' = ek + rho Tn(rho, T)/(g-1), T = (g-1)(E - ek)/rho,
// ek = |m|^2/(2 rho), using the partial derivatives of the branch taken
template <typename T>
__device__ __forceinline__ void cool_vjp_cell(const T* __restrict__ U, long long N, long long q,
                                              T gm1, T dt, const CoolParams<T>& c,
                                              const T (&li)[5], T (&lo)[5]) {
  const T rho = U[q], mx = U[N + q], my = U[2 * N + q], mz = U[3 * N + q], E = U[4 * N + q];
  const T ek = T(0.5) * (mx * mx + my * my + mz * mz) / rho;
  const T Tin = gm1 * (E - ek) / rho;
  // the forward map (same branch decisions as the forward kernel) and its partials
  const T k2 = c.k2r * rho;
  T Tn, dT, dr;
  if (Tin >= c.tc) {
    const T k1 = c.k1r * rho;
    const T st = sqrt(Tin);
    const T t1 = (st - c.sqrt_tc) / k1;
    if (dt <= t1) {
      const T s = st - k1 * dt;
      Tn = s * s;
      dT = s / st;
      dr = -T(2) * s * c.k1r * dt;
    } else {
      const T w = T(1) + k2 * (dt - t1);
      Tn = c.tc - c.ts * log(w);
      dT = c.ts * k2 / (w * T(2) * st * k1);
      dr = -c.ts / w * (c.k2r * (dt - t1) + k2 * t1 / rho);
    }
  } else {
    const T e = exp((c.tc - Tin) * c.its);
    const T w = e + k2 * dt;
    Tn = c.tc - c.ts * log(w);
    dT = e / w;
    dr = -c.ts / w * c.k2r * dt;
  }
  if (Tn < c.tfloor) {
    Tn = c.tfloor;
    dT = T(0);
    dr = T(0);
  }
  const T Eb = li[4];
  T ekb = Eb;
  T rhob = li[0] + Eb * Tn / gm1;
  const T Tnb = Eb * rho / gm1;
  const T Tb = Tnb * dT;
  rhob += Tnb * dr;
  const T Einb = Tb * gm1 / rho;
  ekb -= Tb * gm1 / rho;
  rhob -= Tb * Tin / rho;
  rhob -= ekb * ek / rho;
  lo[0] = rhob;
  lo[1] = li[1] + ekb * mx / rho;
  lo[2] = li[2] + ekb * my / rho;
  lo[3] = li[3] + ekb * mz / rho;
  lo[4] = Einb;
}


template <typename T>
__global__ __launch_bounds__(256) void k_cool_vjp(const T* __restrict__ U, long long N, T gm1, T dt,
                                                  CoolParams<T> c, const T* __restrict__ lin,
                                                  T* lout) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  T li[5], lo[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) li[f] = lin[f * N + q];
  cool_vjp_cell(U, N, q, gm1, dt, c, li, lo);
#pragma unroll
  for (int f = 0; f < 5; ++f) lout[f * N + q] = lo[f];
}

// cooling reverse then forcing-kick reverse in one pass (the order of the
// reverse sweep without gravity): the intermediate adjoint stays in registers
template <typename T>
__global__ __launch_bounds__(256) void k_cool_force_vjp(const T* __restrict__ U, T gm1, T dt,
                                                        CoolParams<T> c,
                                                        const T* __restrict__ rows,
                                                        const T* __restrict__ tabx, int R, int nx,
                                                        int ny, int nz, const T* __restrict__ lin,
                                                        T* lout) {
  const long long N = (long long)nx * ny * nz;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int x = (int)(q % nx), y = (int)((q / nx) % ny), z = (int)(q / ((long long)nx * ny));
  T li[5], lm[5], lo[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) li[f] = lin[f * N + q];
  cool_vjp_cell(U, N, q, gm1, dt, c, li, lm);
  T a[3];
  ou_accel(rows, tabx, R, nx, ny, x, y, z, a);
  kick_vjp_cell(a, dt, lm, lo);
#pragma unroll
  for (int f = 0; f < 5; ++f) lout[f * N + q] = lo[f];
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// J(U)^T v into out = c0 x0 + c1 x1 + beta J^T v (x0, x1 may be NULL)
// cells per column segment of the fused march (k_axis_jtv)
constexpr int ADJ_SEG = 64;

template <typename T>
hipError_t adj_jtv(const AdjointBuffers<T>& B, const StageGeom& geom, int limiter, int riemann,
                   T gamma,
                   const double* h, const T* U, const T* v, T beta, T c0, const T* x0, T c1,
                   const T* x1, T c2, const T* x2, T* out, hipStream_t s) {
  const long long N = (long long)geom.nx * geom.ny * geom.nz;
  const int nn[3] = {geom.nx, geom.ny, geom.nz};
  const bool rt = adj_runtime_scheme(limiter, riemann);
  const FinishArgs<T> fa{gamma - T(1), beta, c0, c1, c2, x0, x1, x2, out};
  // the axes with fluxes (a periodic axis of one cell has none: its fluxes
  // cancel exactly); the first one's gather stores the W adjoint, the last
  // one's adds the others and finishes the cell
  int active[3], na = 0;
  for (int ax = 0; ax < 3; ++ax)
    if (!(geom.bc[ax] == BC_PERIODIC && nn[ax] == 1)) active[na++] = ax;
  if (na == 0) {
    hipLaunchKernelGGL((k_fill<T>), dim3(nblk(5 * N)), dim3(256), 0, s, B.Wacc, 5 * N, T(0));
    hipLaunchKernelGGL((k_jtv_finish<T>), dim3(nblk(N)), dim3(256), 0, s, U, B.Wacc, N, fa);
    return hipGetLastError();
  }
  for (int ia = 0; ia < na; ++ia) {
    const int ax = active[ia];
    const int mode = na == 1 ? GATHER_FIRST_LAST
                             : (ia == 0 ? GATHER_FIRST : (ia == na - 1 ? GATHER_LAST : GATHER_ADD));
    AxisGeom ag{{geom.nx, geom.ny, geom.nz}, geom.bc[ax], 0};
    ag.nf = geom.bc[ax] == BC_PERIODIC ? nn[ax] : nn[ax] + 1;
    const long long nfaces = (long long)ag.nf * (N / nn[ax]);
    const T ih = (T)(1.0 / h[ax]);
#define MH_GATHER(AX, SL)                                                                     \
  do {                                                                                        \
    if (mode == GATHER_ADD)                                                                   \
      hipLaunchKernelGGL((k_cell_gather<T, AX, SL, GATHER_ADD>), dim3(nblk(N)), dim3(256), 0, \
                         s, B.wbar, B.flags, ag, B.Wacc, U, fa);                              \
    else if (mode == GATHER_FIRST)                                                            \
      hipLaunchKernelGGL((k_cell_gather<T, AX, SL, GATHER_FIRST>), dim3(nblk(N)), dim3(256),  \
                         0, s, B.wbar, B.flags, ag, B.Wacc, U, fa);                           \
    else if (mode == GATHER_LAST)                                                             \
      hipLaunchKernelGGL((k_cell_gather<T, AX, SL, GATHER_LAST>), dim3(nblk(N)), dim3(256),   \
                         0, s, B.wbar, B.flags, ag, B.Wacc, U, fa);                           \
    else                                                                                      \
      hipLaunchKernelGGL((k_cell_gather<T, AX, SL, GATHER_FIRST_LAST>), dim3(nblk(N)),        \
                         dim3(256), 0, s, B.wbar, B.flags, ag, B.Wacc, U, fa);                \
  } while (0)
#define MH_FACE(AX)                                                                           \
  do {                                                                                        \
    if (rt) {                                                                                 \
      hipLaunchKernelGGL((k_face_vjp_rt<T, AX>), dim3(nblk(nfaces)), dim3(256), 0, s, U, v,   \
                         ag, gamma, ih, limiter, riemann, B.wbar, nfaces);                    \
      MH_GATHER(AX, true);                                                                    \
    } else {                                                                                  \
      if (limiter == LIM_NONE)                                                                \
        hipLaunchKernelGGL((k_face_vjp<T, LIM_NONE, AX>), dim3(nblk(nfaces)), dim3(256), 0,   \
                           s, U, v, ag, gamma, ih, B.wbar, B.flags, nfaces);                  \
      else                                                                                    \
        hipLaunchKernelGGL((k_face_vjp<T, LIM_MINMOD, AX>), dim3(nblk(nfaces)), dim3(256), 0, \
                           s, U, v, ag, gamma, ih, B.wbar, B.flags, nfaces);                  \
      MH_GATHER(AX, false);                                                                   \
    }                                                                                         \
  } while (0)
    // y and z, periodic with at least four cells, minmod or first order:
    // the fused column march
    const bool march = !rt && geom.bc[ax] == BC_PERIODIC && nn[ax] >= 4;
    if (march && ax == 0) {
      const long long waves = (N / nn[0]) * ((nn[0] + XSEG - 1) / XSEG);
      const unsigned blocks = (unsigned)((waves + 3) / 4);
#define MH_XJTV(LM)                                                                           \
  do {                                                                                        \
    if (mode == GATHER_ADD)                                                                   \
      hipLaunchKernelGGL((k_x_jtv<T, LM, GATHER_ADD>), dim3(blocks), dim3(256), 0, s, U, v,  \
                         ag, gamma, ih, B.Wacc, fa);                                          \
    else if (mode == GATHER_FIRST)                                                            \
      hipLaunchKernelGGL((k_x_jtv<T, LM, GATHER_FIRST>), dim3(blocks), dim3(256), 0, s, U, v, \
                         ag, gamma, ih, B.Wacc, fa);                                          \
    else if (mode == GATHER_LAST)                                                             \
      hipLaunchKernelGGL((k_x_jtv<T, LM, GATHER_LAST>), dim3(blocks), dim3(256), 0, s, U, v,  \
                         ag, gamma, ih, B.Wacc, fa);                                          \
    else                                                                                      \
      hipLaunchKernelGGL((k_x_jtv<T, LM, GATHER_FIRST_LAST>), dim3(blocks), dim3(256), 0, s,  \
                         U, v, ag, gamma, ih, B.Wacc, fa);                                    \
  } while (0)
      if (limiter == LIM_NONE) MH_XJTV(LIM_NONE);
      else MH_XJTV(LIM_MINMOD);
#undef MH_XJTV
    } else if (march) {
      const int seg = nn[ax] < ADJ_SEG ? nn[ax] : ADJ_SEG;
      const long long threads = (N / nn[ax]) * ((nn[ax] + seg - 1) / seg);
#define MH_MARCH(AX, LM)                                                                      \
  do {                                                                                        \
    if (mode == GATHER_ADD)                                                                   \
      hipLaunchKernelGGL((k_axis_jtv<T, LM, AX, GATHER_ADD>), dim3(nblk(threads)), dim3(256), \
                         0, s, U, v, ag, gamma, ih, seg, B.Wacc, fa);                         \
    else if (mode == GATHER_FIRST)                                                            \
      hipLaunchKernelGGL((k_axis_jtv<T, LM, AX, GATHER_FIRST>), dim3(nblk(threads)),          \
                         dim3(256), 0, s, U, v, ag, gamma, ih, seg, B.Wacc, fa);              \
    else if (mode == GATHER_LAST)                                                             \
      hipLaunchKernelGGL((k_axis_jtv<T, LM, AX, GATHER_LAST>), dim3(nblk(threads)),           \
                         dim3(256), 0, s, U, v, ag, gamma, ih, seg, B.Wacc, fa);              \
    else                                                                                      \
      hipLaunchKernelGGL((k_axis_jtv<T, LM, AX, GATHER_FIRST_LAST>), dim3(nblk(threads)),     \
                         dim3(256), 0, s, U, v, ag, gamma, ih, seg, B.Wacc, fa);              \
  } while (0)
      if (ax == 1) {
        if (limiter == LIM_NONE) MH_MARCH(1, LIM_NONE);
        else MH_MARCH(1, LIM_MINMOD);
      } else {
        if (limiter == LIM_NONE) MH_MARCH(2, LIM_NONE);
        else MH_MARCH(2, LIM_MINMOD);
      }
#undef MH_MARCH
    } else if (ax == 0) MH_FACE(0);
    else if (ax == 1) MH_FACE(1);
    else MH_FACE(2);
#undef MH_FACE
#undef MH_GATHER
  }
  return hipGetLastError();
}

template <typename T>
hipError_t adj_flux_corr_vjp(const T* v, const StageGeom& g, const double* h, double weight,
                             T* grad, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL((k_flux_corr_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, v, g.nx, g.ny, g.nz,
                     g.bc[0], g.bc[1], g.bc[2], (T)(weight / h[0]), (T)(weight / h[1]),
                     (T)(weight / h[2]), grad);
  return hipGetLastError();
}

template <typename T>
hipError_t adj_force_kick_vjp(const T* rows, const T* tabx, int R, const StageGeom& g, T dt,
                              const T* lin, T* lout, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL((k_force_kick_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, rows, tabx, R, g.nx,
                     g.ny, g.nz, dt, lin, lout);
  return hipGetLastError();
}

template <typename T>
hipError_t adj_cool_vjp(const T* U, long long N, T gm1, T dt, const CoolParams<T>& c, const T* lin,
                        T* lout, hipStream_t s) {
  hipLaunchKernelGGL((k_cool_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, U, N, gm1, dt, c, lin, lout);
  return hipGetLastError();
}

template <typename T>
hipError_t adj_cool_force_vjp(const T* U, T gm1, T dt, const CoolParams<T>& c, const T* rows,
                              const T* tabx, int R, const StageGeom& g, const T* lin, T* lout,
                              hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL((k_cool_force_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, U, gm1, dt, c, rows,
                     tabx, R, g.nx, g.ny, g.nz, lin, lout);
  return hipGetLastError();
}

// reverse of the gravity step at Ub (the state the kick acted on), with the
// potential phi solved from Ub: lout from lin, using a second multigrid solve
// with the same operator for the adjoint of A^+ (Sec. 6.2.4)
template <typename T>
hipError_t adj_gravity_vjp(const AdjointBuffers<T>& B, MGLayout& mgL, char* mgws,
                           const mh_physics_desc& p, const T* Ub, const T* phi, int n, double h,
                           T dt, const T* lin, T* lout, DevClock* clk, hipStream_t s) {
  const long long N = (long long)n * n * n;
  if (mgL.fft) return fft_gravity_vjp<T>(mgws, mgL, h, p.grav_G, Ub, dt, lin, lout, B.accb, s);
  const T i2h = (T)(1.0 / (2.0 * h));
  hipLaunchKernelGGL((k_grav_kick_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, Ub, phi, n, i2h, dt,
                     lin, lout, B.accb);
  hipLaunchKernelGGL((k_grad_adjoint<T>), dim3(nblk(N)), dim3(256), 0, s, B.accb, n, i2h, B.phib);
  hipError_t e = mg_set_rhs<T>(mgws, mgL, B.phib, 1.0, clk, s);
  if (e != hipSuccess) return e;
  e = mg_set_guess<T>(mgws, mgL, (const T*)nullptr, s);
  if (e != hipSuccess) return e;
  e = mg_solve<T>(mgws, mgL, p, clk, nullptr, s);
  if (e != hipSuccess) return e;
  const T* x = reinterpret_cast<const T*>(mgws + mg_phi_offset(mgL));
  hipLaunchKernelGGL((k_axpy<T>), dim3(nblk(N)), dim3(256), 0, s, lout, x, N,
                     (T)(4.0 * M_PI * p.grav_G));
  return hipGetLastError();
}

#define ADJ_INSTANTIATE(T)                                                                       \
  template hipError_t adj_jtv<T>(const AdjointBuffers<T>&, const StageGeom&, int, int, T,        \
                                 const double*, const T*, const T*, T, T, const T*, T, const T*, \
                                 T, const T*, T*, hipStream_t);                                  \
  template hipError_t adj_flux_corr_vjp<T>(const T*, const StageGeom&, const double*, double,   \
                                           T*, hipStream_t);                                   \
  template hipError_t adj_force_kick_vjp<T>(const T*, const T*, int, const StageGeom&, T,        \
                                            const T*, T*, hipStream_t);                          \
  template hipError_t adj_cool_vjp<T>(const T*, long long, T, T, const CoolParams<T>&, const T*, \
                                      T*, hipStream_t);                                          \
  template hipError_t adj_cool_force_vjp<T>(const T*, T, T, const CoolParams<T>&, const T*,     \
                                            const T*, int, const StageGeom&, const T*, T*,     \
                                            hipStream_t);                                      \
  template hipError_t adj_gravity_vjp<T>(const AdjointBuffers<T>&, MGLayout&, char*,             \
                                         const mh_physics_desc&, const T*, const T*, int, double, \
                                         T, const T*, T*, DevClock*, hipStream_t);
ADJ_INSTANTIATE(float)
ADJ_INSTANTIATE(double)
#undef ADJ_INSTANTIATE

}  // namespace mh
