// hydro_kernels.hip -- fused finite-volume stage kernels for gfx950.
//
// One launch of k_stage performs one Runge-Kutta stage of the unsplit
// method-of-lines update of diffhydro (arXiv 2512.13403, App. A.3):
//   stage 1:  U1 = U^n + dt L(U^n)
//   stage 3:  U' = ca U^n + cb (Uk + dt L(Uk))            (an inner stage)
//   stage 2:  U^{n+1} = ca U^n + cb (Uk + dt L(Uk)), then the sources
// -- (ca, cb) = (1/2, 1/2) after stage 1 for the two-stage SSP-RK2; (3/4, 1/4)
// for the inner stage and (1/3, 2/3) for the last one in SSPRK3; (0, 1) for
// forward Euler, a lone final stage -- with L(U) = -sum_a (F_{a,i+1/2} - F_{a,i-1/2}) / dx_a, the face fluxes F
// from HLLC (App. A.2) on MUSCL face states of the primitive variables with a
// minmod-limited slope (App. A.1).  Stage 2 also applies, per cell and in
// registers, the operator-split sources in the order forcing -> cooling
// (Sec. 3.1.1, Sec. 4), flags unphysical cells, and reduces the CFL signal
// speed max_a (|v_a| + c_s)/dx_a of the new state (App. A.4) into the device
// clock, so the next step's dt never leaves the GPU.
//
// Data movement per stage (fp32): each cell is read once from HBM for its own
// column and written once; the x/y stencil halos of a 64 x 8 tile come from
// neighbouring tiles through L2 (the outputs and the last stage's U^n, which
// no other tile reads, go through non-temporal stores and loads so as not to
// displace them).  Primitive variables of the current z-plane
// live in LDS (with a 2-cell x/y halo); the z-stencil is a register ring of
// four planes per thread, so the kernel marches along z and touches each
// plane once.  Every face flux is computed exactly once per tile: x faces by
// the thread on their left, which takes the limited x slope of the cell on
// the right from the next lane of its wave (the tile's left and right edges by
// lanes of one wave), y faces by the thread below (plus the tile's lower
// edge), z faces by the column's thread, carried from one plane to the next.
// Floating-point contraction is off in this file and every fused multiply-add
// is written out: the compiler may not fuse a product into a sum at one call
// site of the face flux and not at another, so each face gets bit-identical
// arithmetic wherever it is computed (interior faces, the tile's edge faces,
// the first z face of a column), and a state that is uniform along an axis
// stays exactly uniform.
#pragma clang fp contract(off)

#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

// minmod(a, b): the smaller magnitude when a and b share a sign, else 0 --
// which is the median of (a, b, 0): one v_med3_f32 in fp32.
__device__ __forceinline__ float minmod(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// limited slope of W_i from W_{i-1}, W_i, W_{i+1} (App. A.1): limiter(a, b)
// of the forward and backward differences a = W_{i+1} - W_i, b = W_i - W_{i-1};
// every limiter is 0 when a and b disagree in sign.  The LIM_GENERIC kernel
// takes the limiter `rl` at run time.
template <typename T>
__device__ __forceinline__ T slope_of(int rl, T a, T b) {
  if (rl == LIM_MINMOD) return minmod(a, b);
  if (rl == LIM_NONE) return T(0);
  const bool same = a * b > T(0);
  T m;
  if (rl == LIM_VANLEER) {
    m = T(2) * a * b * dev_rcp(a + b);  // harmonic mean
  } else {
    const T aa = fabs(a), ab = fabs(b);
    T mag;
    if (rl == LIM_MC) mag = fmin(fabs(T(0.5) * (a + b)), fmin(T(2) * aa, T(2) * ab));
    else mag = fmax(fmin(T(2) * aa, ab), fmin(aa, T(2) * ab));  // superbee
    m = a > T(0) ? mag : -mag;
  }
  return same ? m : T(0);
}

template <typename T, int LIM>
__device__ __forceinline__ T limited_slope(T wm, T w0, T wp, int rl = 0) {
  if (LIM == LIM_NONE) return T(0);
  if (LIM == LIM_GENERIC) return slope_of(rl, wp - w0, w0 - wm);
  if (LIM == LIM_VANLEER || LIM == LIM_MC || LIM == LIM_SUPERBEE)
    return slope_of(LIM, wp - w0, w0 - wm);
  return minmod(wp - w0, w0 - wm);
}

// c = sqrt(gamma P / rho) from gp = gamma P, as gp * rsq(gp rho): one
// reciprocal square root instead of a division and a square root
__device__ __forceinline__ float sound_speed(float gp, float rho) { return gp * dev_rsq(gp * rho); }
__device__ __forceinline__ double sound_speed(double gp, double rho) { return gp * dev_rsq(gp * rho); }

// HLLC flux through a face with normal velocity component `n` (0, 1, 2) of
// the primitive face states wl, wr = (rho, vx, vy, vz, P).  Davis speeds
// S_L = min(vL - cL, vR - cR), S_R = max(vL + cL, vR + cR); contact speed
// S* and star states as in the standard HLLC construction.  Only the side
// K that the face falls on is assembled: F = F_K + S_K (U*_K - U_K) inside
// the star fan, F = F_K outside it, with
//   U*_K = q (d_K, d_K S*, d_K vt1, d_K vt2, (S_K - v_K) E_K + (S* - v_K)(d_K S* + P_K)),
//   d_K = rho_K (S_K - v_K), q = 1 / (S_K - S*),
// which is the usual star state with the common factor rho_K (S_K - v_K) /
// (S_K - S*) multiplied through (one reciprocal instead of three divides).
template <typename T, int N>
__device__ __forceinline__ void hllc_flux(const T (&wl)[5], const T (&wr)[5], T gamma, T gm1inv,
                                          T (&F)[5]) {
  constexpr int t1 = 1 + (N + 1) % 3, t2 = 1 + (N + 2) % 3, vn = 1 + N;
  const T rl = wl[0], ul = wl[vn], pl = wl[4];
  const T rr = wr[0], ur = wr[vn], pr = wr[4];
  const T cl = sound_speed(gamma * pl, rl), cr = sound_speed(gamma * pr, rr);
  const T SL = fmin(ul - cl, ur - cr), SR = fmax(ul + cl, ur + cr);
  const T dl = rl * (SL - ul), dr = rr * (SR - ur);
  const T sstar = fmad(-ur, dr, fmad(ul, dl, pr - pl)) * dev_rcp(dl - dr);
  // side: the oracle's region order (0 <= S_L, 0 <= S*, 0 < S_R, else R)
  const bool left = (SL >= T(0)) || (sstar >= T(0));
  const T rK = left ? rl : rr, uK = left ? ul : ur, pK = left ? pl : pr;
  const T aK = left ? wl[t1] : wr[t1], bK = left ? wl[t2] : wr[t2];
  const T SK = left ? SL : SR, dK = left ? dl : dr;
  // total energy of the selected side only (the other side's is never used)
  const T EK = fmad(pK, gm1inv, (T(0.5) * rK) * fmad(uK, uK, fmad(aK, aK, bK * bK)));
  // inside the star fan: S_L < 0 on the left side, S_R > 0 on the right
  const bool fan = (left ? -SL : SR) > T(0);
  const T mK = rK * uK;
  const T FK0 = mK, FK1 = fmad(mK, uK, pK), FK2 = mK * aK, FK3 = mK * bK, FK4 = uK * (EK + pK);
  const T q = dev_rcp(SK - sstar);
  const T qd = q * dK;
  const T s0 = qd, s1 = qd * sstar, s2 = qd * aK, s3 = qd * bK;
  const T s4 = q * fmad(SK - uK, EK, (sstar - uK) * fmad(dK, sstar, pK));
  const T f0 = fmad(SK, s0 - rK, FK0);
  const T f1 = fmad(SK, s1 - mK, FK1);
  const T f2 = fmad(SK, fmad(-rK, aK, s2), FK2);
  const T f3 = fmad(SK, fmad(-rK, bK, s3), FK3);
  const T f4 = fmad(SK, s4 - EK, FK4);
  F[0] = fan ? f0 : FK0;
  F[vn] = fan ? f1 : FK1;
  F[t1] = fan ? f2 : FK2;
  F[t2] = fan ? f3 : FK3;
  F[4] = fan ? f4 : FK4;
}

// conserved state and physical flux of a primitive face state, in the
// component order of the grid (normal momentum at 1 + N)
template <typename T, int N>
__device__ __forceinline__ void state_flux(const T (&w)[5], T gm1inv, T (&U)[5], T (&F)[5]) {
  constexpr int vn = 1 + N;
  const T rho = w[0], u = w[vn], p = w[4];
  const T E = fmad(p, gm1inv, (T(0.5) * rho) * fmad(w[1], w[1], fmad(w[2], w[2], w[3] * w[3])));
  const T m = rho * u;
  U[0] = rho;
  U[1] = rho * w[1];
  U[2] = rho * w[2];
  U[3] = rho * w[3];
  U[4] = E;
  F[0] = m;
  F[1] = m * w[1];
  F[2] = m * w[2];
  F[3] = m * w[3];
  F[vn] = fmad(m, u, p);
  F[4] = u * (E + p);
}

// HLL (two-wave) flux with the Davis speeds (App. A.2 lists it with Rusanov
// as alternatives to HLLC): F_L for 0 <= S_L, F_R for S_R <= 0, else
// (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L)
template <typename T, int N>
__device__ __forceinline__ void hll_flux(const T (&wl)[5], const T (&wr)[5], T gamma, T gm1inv,
                                         T (&F)[5]) {
  constexpr int vn = 1 + N;
  const T cl = sound_speed(gamma * wl[4], wl[0]), cr = sound_speed(gamma * wr[4], wr[0]);
  const T SL = fmin(wl[vn] - cl, wr[vn] - cr), SR = fmax(wl[vn] + cl, wr[vn] + cr);
  T UL[5], FL[5], UR[5], FR[5];
  state_flux<T, N>(wl, gm1inv, UL, FL);
  state_flux<T, N>(wr, gm1inv, UR, FR);
  const T q = dev_rcp(SR - SL);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T fm = (fmad(SR, FL[f], -SL * FR[f]) + SL * SR * (UR[f] - UL[f])) * q;
    F[f] = SL >= T(0) ? FL[f] : (SR <= T(0) ? FR[f] : fm);
  }
}

// Rusanov (local Lax-Friedrichs): (F_L + F_R)/2 - s (U_R - U_L)/2 with
// s = max(|v_L| + c_L, |v_R| + c_R)
template <typename T, int N>
__device__ __forceinline__ void rusanov_flux(const T (&wl)[5], const T (&wr)[5], T gamma,
                                             T gm1inv, T (&F)[5]) {
  constexpr int vn = 1 + N;
  const T cl = sound_speed(gamma * wl[4], wl[0]), cr = sound_speed(gamma * wr[4], wr[0]);
  const T smax = fmax(fabs(wl[vn]) + cl, fabs(wr[vn]) + cr);
  T UL[5], FL[5], UR[5], FR[5];
  state_flux<T, N>(wl, gm1inv, UL, FL);
  state_flux<T, N>(wr, gm1inv, UR, FR);
#pragma unroll
  for (int f = 0; f < 5; ++f)
    F[f] = fmad(T(0.5), FL[f] + FR[f], -(T(0.5) * smax) * (UR[f] - UL[f]));
}

// the face flux of the scheme: HLLC in the specialised kernels, the solver
// `rs` chosen at run time in the LIM_GENERIC kernel
template <typename T, int N, int LIM>
__device__ __forceinline__ void riemann_flux(const T (&wl)[5], const T (&wr)[5], T gamma, T gm1inv,
                                             int rs, T (&F)[5]) {
  if (LIM == LIM_GENERIC && rs == RS_HLL) hll_flux<T, N>(wl, wr, gamma, gm1inv, F);
  else if (LIM == LIM_GENERIC && rs == RS_RUSANOV) rusanov_flux<T, N>(wl, wr, gamma, gm1inv, F);
  else hllc_flux<T, N>(wl, wr, gamma, gm1inv, F);
}

// flux through the face between cells i and i+1 from W_{i-1}, W_i, W_{i+1},
// W_{i+2}: W^L = W_i + dW_i/2, W^R = W_{i+1} - dW_{i+1}/2 (App. A.1)
template <typename T, int LIM, int N>
__device__ __forceinline__ void face_flux(const T (&wm)[5], const T (&w0)[5], const T (&w1)[5],
                                          const T (&w2)[5], T gamma, T gm1inv, int rl, int rs,
                                          T (&F)[5]) {
  T wl[5], wr[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    wl[f] = fmad(T(0.5), limited_slope<T, LIM>(wm[f], w0[f], w1[f], rl), w0[f]);
    wr[f] = fmad(T(-0.5), limited_slope<T, LIM>(w0[f], w1[f], w2[f], rl), w1[f]);
  }
  riemann_flux<T, N, LIM>(wl, wr, gamma, gm1inv, rs, F);
}

// the same flux from precomputed limited slopes d0 of W_i and d1 of W_{i+1}
template <typename T, int N, int LIM>
__device__ __forceinline__ void face_flux_sl(const T (&w0)[5], const T (&d0)[5], const T (&w1)[5],
                                             const T (&d1)[5], T gamma, T gm1inv, int rs,
                                             T (&F)[5]) {
  T wl[5], wr[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    wl[f] = fmad(T(0.5), d0[f], w0[f]);
    wr[f] = fmad(T(-0.5), d1[f], w1[f]);
  }
  riemann_flux<T, N, LIM>(wl, wr, gamma, gm1inv, rs, F);
}

// learned flux correction (the solver-in-the-loop flux term): the field's
// value at a cell is added to the flux through each of its upper faces
template <typename T>
__device__ __forceinline__ void add_dflux(const T* __restrict__ d, long long N, long long q,
                                          T (&F)[5]) {
#pragma unroll
  for (int f = 0; f < 5; ++f) F[f] += d[f * N + q];
}

// the 5 fields of one lane's cell in a z-plane: `base` is field 0 of the
// plane (the same for the whole wave) and `off` the lane's byte offset
// within the plane.  The empty asm statements make the offset and each
// field's plane base opaque at the access, the base in scalar registers, so
// the compiler neither folds the offset into per-lane 64-bit pointers nor
// shares one base among the fields: every access is one scalar base + one
// 32-bit vector offset, without 64-bit vector address arithmetic.
__device__ __forceinline__ uint32_t lane_off(uint32_t off) {
  asm volatile("" : "+v"(off));
  return off;
}
// STREAM: a non-temporal load, for data read once (U^n of the last stage),
// so that it does not displace from L2 the halo rows the neighbouring tiles
// read again
template <typename T, bool STREAM = false>
__device__ __forceinline__ void load_lane(const T* __restrict__ base, long long N, uint32_t off,
                                          T (&u)[5]) {
  typedef __attribute__((address_space(1))) const char gchar;
  typedef __attribute__((address_space(1))) const T gT;
  const uint32_t o = lane_off(off);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    gchar* b = (gchar*)(base + f * N);
    asm volatile("" : "+s"(b));
    if (STREAM) u[f] = __builtin_nontemporal_load((gT*)(b + o));
    else u[f] = *(gT*)(b + o);
  }
}
// the stage's output, written once and not read again by this launch:
// non-temporal stores, which keep L2 for the halo rows
template <typename T>
__device__ __forceinline__ void store_lane(T* __restrict__ base, long long N, uint32_t off,
                                           const T (&u)[5]) {
  typedef __attribute__((address_space(1))) char gchar;
  typedef __attribute__((address_space(1))) T gT;
  const uint32_t o = lane_off(off);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    gchar* b = (gchar*)(base + f * N);
    asm volatile("" : "+s"(b));
    __builtin_nontemporal_store(u[f], (gT*)(b + o));
  }
}

// the value this quantity has in lane + 1 of the wave (a DPP wave shift
// left by one lane); lane 63 receives 0
__device__ __forceinline__ float from_next_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_next_lane(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x130, 0xf, 0xf, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x130, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Each row of the tile (fixed ty) is exactly one wave, so a lane's x
// neighbour is the next lane and the edge faces below can be given to whole
// waves.
static_assert(TX == 64 && 2 * TY <= TX, "one wave per tile row; the edge wave takes 2 TY x faces");

template <typename T, int STAGE, int LIM, bool FORCE, bool COOL>
__global__ __launch_bounds__(NTHREADS, sizeof(T) == 4 ? 4 : 2) void k_stage(const StageArgs<T> a) {
  __shared__ T sW[5][TY + 4][TX + 4];
  __shared__ T sFx[5][TY][TX + 1];
  __shared__ T sFy[5][TY + 1][TX];
  __shared__ T sRed[NTHREADS / 64];
  // separable forcing: the row sums P_n, Q_n (see k_force_rows) of the tile's
  // rows, three planes in flight, and the x phase factors X_n of its columns
  __shared__ T sPQ[FORCE ? 3 : 1][TY][FORCE ? 6 * (MAX_R + 1) : 1];
  __shared__ T sX[FORCE ? MAX_R + 1 : 1][2][TX];

  // XCD-aware tile order: consecutive hardware workgroups go round-robin to
  // the 8 XCDs, so give each XCD a contiguous range of tiles (x fastest, then
  // y, then z) and the x/y halos of neighbouring tiles stay in one L2.
  const int b = blockIdx.x;
  const int logical = (b & 7) * a.nb_per_xcd + (b >> 3);
  if (logical >= a.nbx * a.nby * a.nbz) return;
  const int bx = logical % a.nbx;
  const int rest = logical / a.nbx;
  const int by = rest % a.nby, bz = rest / a.nby;

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.zc;
  const int zend = min(z0 + a.zc, a.nz);
  const int gx = x0 + tx, gy = y0 + ty;
  const bool inside = gx < a.nx && gy < a.ny;
  const long long N = a.ncell;
  const long long plane = (long long)a.nx * a.ny;
  const long long col = (long long)bc_map(gy, a.ny, a.bcy) * a.nx + bc_map(gx, a.nx, a.bcx);
  const T gamma = a.gamma, gm1 = a.gm1, gm1inv = a.gm1inv;
  const T dt = (T)a.clk->dt;
  // byte offsets of this lane's column within a z-plane (all in-loop loads
  // and stores address a plane base plus such an offset)
  const uint32_t col_b = (uint32_t)col * (uint32_t)sizeof(T);

  // halo cells of the current plane this thread loads into LDS (if any):
  // 4 columns x TY rows left/right of the tile, TX columns x 4 rows below/above
  int h_lx = -1, h_ly = -1;
  long long h_col = 0;
  if (tid < 4 * TY) {
    const int hy = tid >> 2, hi = tid & 3;
    h_lx = hi < 2 ? hi : TX + hi;
    h_ly = hy + 2;
    h_col = (long long)bc_map(y0 + hy, a.ny, a.bcy) * a.nx + bc_map(x0 - 2 + h_lx, a.nx, a.bcx);
  } else if (tid < 4 * TY + 4 * TX) {
    const int t2 = tid - 4 * TY;
    const int hx = t2 % TX, hj = t2 / TX;
    h_ly = hj < 2 ? hj : TY + hj;
    h_lx = hx + 2;
    h_col = (long long)bc_map(y0 - 2 + h_ly, a.ny, a.bcy) * a.nx + bc_map(x0 + hx, a.nx, a.bcx);
  }

  const uint32_t h_b = (uint32_t)h_col * (uint32_t)sizeof(T);

  // forcing rows: thread tid < TY * 6(R+1) owns element `pq_e` of its row's
  // record; the record of plane z+1 is loaded during plane z-1 and stored to
  // LDS during plane z (slot (z - z0) mod 3), read during plane z+1
  const int nr6 = FORCE ? 6 * (a.ou_R + 1) : 1;
  const bool pq_thread = FORCE && tid < TY * nr6;
  const int pq_r = pq_thread ? tid / nr6 : 0, pq_e = pq_thread ? tid % nr6 : 0;
  const long long pq_row = (y0 + pq_r) < a.ny ? (y0 + pq_r) : 0;
  T pq_ahead = T(0);
  if (FORCE) {
    if (ty == 0) {
      const int ix = gx < a.nx ? gx : 0;
      for (int n = 0; n <= a.ou_R; ++n) {
        sX[n][0][tx] = a.ou_tab[0][2 * ((long long)n * a.nx + ix)];
        sX[n][1][tx] = a.ou_tab[0][2 * ((long long)n * a.nx + ix) + 1];
      }
    }
    if (pq_thread) {
      sPQ[0][pq_r][pq_e] = a.ou_rows[((long long)z0 * a.ny + pq_row) * nr6 + pq_e];
      if (z0 + 1 < zend)
        pq_ahead = a.ou_rows[((long long)(z0 + 1) * a.ny + pq_row) * nr6 + pq_e];
    }
    __syncthreads();
  }
  int pq_slot = 0;

  // z ring: W at z-1, z, z+1, z+2; U at z, z+1, z+2; z-flux at z-1/2; the
  // limited z slope of W at z (each cell's slope is computed once)
  T w[4][5], u[3][5], fzm[5], dz1[5];
  {
    T tmp[5], wz[5], dz0[5];
    load_cell(a.uin, N, (long long)bc_map(z0 - 2, a.nz, a.bcz) * plane + col, tmp);
    to_prim(tmp, gm1, wz);
    load_cell(a.uin, N, (long long)bc_map(z0 - 1, a.nz, a.bcz) * plane + col, tmp);
    to_prim(tmp, gm1, w[0]);
    load_cell(a.uin, N, (long long)bc_map(z0, a.nz, a.bcz) * plane + col, u[0]);
    to_prim(u[0], gm1, w[1]);
    load_cell(a.uin, N, (long long)bc_map(z0 + 1, a.nz, a.bcz) * plane + col, u[1]);
    to_prim(u[1], gm1, w[2]);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      dz0[f] = limited_slope<T, LIM>(wz[f], w[0][f], w[1][f], a.lim);
      dz1[f] = limited_slope<T, LIM>(w[0][f], w[1][f], w[2][f], a.lim);
    }
    face_flux_sl<T, 2, LIM>(w[0], dz0, w[1], dz1, gamma, gm1inv, a.rs, fzm);
    if (LIM == LIM_GENERIC && a.dflux)
      add_dflux(a.dflux, N, (long long)bc_map(z0 - 1, a.nz, a.bcz) * plane + col, fzm);
  }

  T smax = T(0);
  unsigned long long nbad = 0, first_bad = ~0ull;

  // software pipeline: the column cell two planes ahead and this thread's halo
  // cell of the current plane are loaded one iteration early
  T u_ahead[5], h_ahead[5] = {T(0), T(0), T(0), T(0), T(0)};
  load_cell(a.uin, N, (long long)bc_map(z0 + 2, a.nz, a.bcz) * plane + col, u_ahead);
  if (h_lx >= 0) load_cell(a.uin, N, (long long)z0 * plane + h_col, h_ahead);

  for (int z = z0; z < zend; ++z) {
    T hu[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      u[2][f] = u_ahead[f];
      hu[f] = h_ahead[f];
    }
    if (z + 1 < zend) {
      load_lane(a.uin + (long long)bc_map(z + 3, a.nz, a.bcz) * plane, N, col_b, u_ahead);
      if (h_lx >= 0) load_lane(a.uin + (long long)(z + 1) * plane, N, h_b, h_ahead);
    }
    to_prim(u[2], gm1, w[3]);
#pragma unroll
    for (int f = 0; f < 5; ++f) sW[f][ty + 2][tx + 2] = w[1][f];
    if (h_lx >= 0) {
      T hw[5];
      to_prim(hu, gm1, hw);
#pragma unroll
      for (int f = 0; f < 5; ++f) sW[f][h_ly][h_lx] = hw[f];
    }
    if (pq_thread) {
      if (z + 1 < zend) sPQ[pq_slot == 2 ? 0 : pq_slot + 1][pq_r][pq_e] = pq_ahead;
      if (z + 2 < zend)
        pq_ahead = a.ou_rows[((long long)(z + 2) * a.ny + pq_row) * nr6 + pq_e];
    }
    __syncthreads();

    {
      T c0[5], c1[5], c2[5], c3[5], F[5];
      // x face at x + 1/2: the limited x slope of this lane's cell (its W is
      // w[1]), and that of the next cell taken from lane + 1, which computed it
      // as its own; lane 63's face is the tile's right edge, taken below
      {
        T dx0[5], dx1[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          c0[f] = sW[f][ty + 2][tx + 1];
          c2[f] = sW[f][ty + 2][tx + 3];
          dx0[f] = limited_slope<T, LIM>(c0[f], w[1][f], c2[f], a.lim);
          dx1[f] = LIM == LIM_NONE ? T(0) : from_next_lane(dx0[f]);
        }
        face_flux_sl<T, 0, LIM>(w[1], dx0, c2, dx1, gamma, gm1inv, a.rs, F);
      }
      if (LIM == LIM_GENERIC && a.dflux) add_dflux(a.dflux, N, (long long)z * plane + col, F);
      if (tx < TX - 1) {
#pragma unroll
        for (int f = 0; f < 5; ++f) sFx[f][ty][tx + 1] = F[f];
      }
      // y face at y + 1/2
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        c0[f] = sW[f][ty + 1][tx + 2];
        c2[f] = sW[f][ty + 3][tx + 2];
        c3[f] = sW[f][ty + 4][tx + 2];
      }
      face_flux<T, LIM, 1>(c0, w[1], c2, c3, gamma, gm1inv, a.lim, a.rs, F);
      if (LIM == LIM_GENERIC && a.dflux) add_dflux(a.dflux, N, (long long)z * plane + col, F);
#pragma unroll
      for (int f = 0; f < 5; ++f) sFy[f][ty + 1][tx] = F[f];
      // the tile's edge faces: the TX y faces at y0 - 1/2 by the wave of row
      // 0; the TY x faces at x0 - 1/2 and the TY at x0 + TX - 1/2 by lanes of
      // the wave of row 1, so two waves (not every wave) carry the extra flux
      if (ty == 0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          c0[f] = sW[f][0][tx + 2];
          c1[f] = sW[f][1][tx + 2];
          c2[f] = sW[f][2][tx + 2];
          c3[f] = sW[f][3][tx + 2];
        }
        face_flux<T, LIM, 1>(c0, c1, c2, c3, gamma, gm1inv, a.lim, a.rs, F);
        if (LIM == LIM_GENERIC && a.dflux)
          add_dflux(a.dflux, N,
                    (long long)z * plane + (long long)bc_map(y0 - 1, a.ny, a.bcy) * a.nx +
                        bc_map(gx, a.nx, a.bcx),
                    F);
#pragma unroll
        for (int f = 0; f < 5; ++f) sFy[f][0][tx] = F[f];
      } else if (ty == 1 && tx < 2 * TY) {
        // lane r < TY: row r's face at x0 - 1/2 (LDS columns 0..3); lane
        // TY + r: its face at x0 + TX - 1/2 (columns TX..TX+3)
        const int r = tx < TY ? tx : tx - TY, xc = tx < TY ? 0 : TX;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          c0[f] = sW[f][r + 2][xc];
          c1[f] = sW[f][r + 2][xc + 1];
          c2[f] = sW[f][r + 2][xc + 2];
          c3[f] = sW[f][r + 2][xc + 3];
        }
        face_flux<T, LIM, 0>(c0, c1, c2, c3, gamma, gm1inv, a.lim, a.rs, F);
        if (LIM == LIM_GENERIC && a.dflux)
          add_dflux(a.dflux, N,
                    (long long)z * plane + (long long)bc_map(y0 + r, a.ny, a.bcy) * a.nx +
                        bc_map(x0 - 1 + xc, a.nx, a.bcx),
                    F);
#pragma unroll
        for (int f = 0; f < 5; ++f) sFx[f][r][xc] = F[f];
      }
    }
    T fzp[5], dz2[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) dz2[f] = limited_slope<T, LIM>(w[1][f], w[2][f], w[3][f], a.lim);
    face_flux_sl<T, 2, LIM>(w[1], dz1, w[2], dz2, gamma, gm1inv, a.rs, fzp);
    if (LIM == LIM_GENERIC && a.dflux) add_dflux(a.dflux, N, (long long)z * plane + col, fzp);
    __syncthreads();

    T un[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      T L = -(sFx[f][ty][tx + 1] - sFx[f][ty][tx]) * a.ihx;
      L = fmad(-(sFy[f][ty + 1][tx] - sFy[f][ty][tx]), a.ihy, L);
      L = fmad(-(fzp[f] - fzm[f]), a.ihz, L);
      un[f] = fmad(dt, L, u[0][f]);
    }
    const long long q = (long long)z * plane + col;
    if (STAGE != 1) {
      T u0[5];
      if (inside) load_lane<T, true>(a.un + (long long)z * plane, N, col_b, u0);
      else {
#pragma unroll
        for (int f = 0; f < 5; ++f) u0[f] = u[0][f];
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) un[f] = fmad(a.ca, u0[f], a.cb * un[f]);
    }
    if (STAGE != 2) {
      if (inside) {
        store_lane(a.uout + (long long)z * plane, N, col_b, un);
      }
    } else {
      if (FORCE) {
        // a(x) = scale sum_m 2 Re(ahat_m exp(2 pi i n_m . x / L)) at the cell
        // centre; coef = 2 scale ahat (T), phase tables per axis for n >= 0,
        // complex conjugate for n < 0.
        // separable form: a_c = P_0 + sum_{n>=1} (Re X_n P_n - Im X_n Q_n)
        const T* pq = sPQ[pq_slot][ty];
        T acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = pq[2 * c];
        for (int n = 1; n <= a.ou_R; ++n) {
          const T xr = sX[n][0][tx], xi = sX[n][1][tx];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            acc[c] += fmad(xr, pq[6 * n + 2 * c], -xi * pq[6 * n + 2 * c + 1]);
        }
        // m += rho a dt, E += (m_old . a) dt  (Sec. 3.1.1, Sec. 2.1 listing)
        const T dE = fmad(un[1], acc[0], fmad(un[2], acc[1], un[3] * acc[2]));
#pragma unroll
        for (int c = 0; c < 3; ++c) un[1 + c] = fmad(un[0] * acc[c], dt, un[1 + c]);
        un[4] = fmad(dE, dt, un[4]);
      }
      const T ir = dev_rcp(un[0]);
      const T vx = un[1] * ir, vy = un[2] * ir, vz = un[3] * ir;
      const T ek = (T(0.5) * un[0]) * fmad(vx, vx, fmad(vy, vy, vz * vz));
      T pn = gm1 * (un[4] - ek);
      if (COOL) {
        const T Tn = cool_T(un[0], pn * ir, dt, a.cool);
        un[4] = fmad(un[0] * Tn, gm1inv, ek);
        pn = gm1 * (un[4] - ek);
      }
      if (inside) {
        store_lane(a.uout + (long long)z * plane, N, col_b, un);
        if (a.epilogue) {
          // CFL signal speed of the new state and the health check
          T wn[5] = {un[0], vx, vy, vz, pn};
          const T cs = sound_speed(gamma * pn, un[0]);
          const T s = fmax(fmax((fabs(wn[1]) + cs) * a.ihx, (fabs(wn[2]) + cs) * a.ihy),
                           (fabs(wn[3]) + cs) * a.ihz);
          smax = fmax(smax, s);
          const bool ok = (wn[0] > T(0)) && (wn[4] > T(0)) && isfinite(un[1]) &&
                          isfinite(un[2]) && isfinite(un[3]) && isfinite(un[4]) && isfinite(s);
          if (!ok) {
            ++nbad;
            if ((unsigned long long)q < first_bad) first_bad = (unsigned long long)q;
          }
        }
      }
    }

    // advance the z ring
    pq_slot = pq_slot == 2 ? 0 : pq_slot + 1;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      fzm[f] = fzp[f];
      dz1[f] = dz2[f];
      w[0][f] = w[1][f];
      w[1][f] = w[2][f];
      w[2][f] = w[3][f];
      u[0][f] = u[1][f];
      u[1][f] = u[2][f];
    }
  }

  if (STAGE == 2 && a.epilogue) {
    T m = wave_max(smax);
    if ((tid & 63) == 0) sRed[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      T bm = sRed[0];
      for (int i = 1; i < NTHREADS / 64; ++i) bm = fmax(bm, sRed[i]);
      atomicMax(&a.clk->smax, pos_bits(bm));
    }
    if (nbad) {
      atomicAdd(&a.clk->bad_count, nbad);
      atomicMin(&a.clk->bad_first, first_bad);
    }
  }
}

// The end of the last stage for a step that keeps its state after the
// forcing kick (`ub`, written by k_stage<2> with the cooling and the epilogue
// left out): the exact cooling and the CFL / health epilogue of k_stage<2>,
// the same arithmetic from the stored state instead of registers, so the
// result is bitwise the fused stage's.  One thread per cell.
template <typename T, bool COOL>
__global__ __launch_bounds__(256) void k_stage2_finish(const StageArgs<T> a,
                                                       const T* __restrict__ ub) {
  __shared__ T sRed[4];
  const long long N = a.ncell;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  const int tid = threadIdx.x;
  const T gamma = a.gamma, gm1 = a.gm1, gm1inv = a.gm1inv;
  const T dt = (T)a.clk->dt;
  T smax = T(0);
  unsigned nbad = 0;
  if (q < N) {
    T un[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) un[f] = ub[f * N + q];
    const T ir = dev_rcp(un[0]);
    const T vx = un[1] * ir, vy = un[2] * ir, vz = un[3] * ir;
    const T ek = (T(0.5) * un[0]) * fmad(vx, vx, fmad(vy, vy, vz * vz));
    T pn = gm1 * (un[4] - ek);
    if (COOL) {
      const T Tn = cool_T(un[0], pn * ir, dt, a.cool);
      un[4] = fmad(un[0] * Tn, gm1inv, ek);
      pn = gm1 * (un[4] - ek);
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) a.uout[f * N + q] = un[f];
    const T cs = sound_speed(gamma * pn, un[0]);
    const T sp = fmax(fmax((fabs(vx) + cs) * a.ihx, (fabs(vy) + cs) * a.ihy),
                      (fabs(vz) + cs) * a.ihz);
    smax = sp;
    const bool ok = (un[0] > T(0)) && (pn > T(0)) && isfinite(un[1]) && isfinite(un[2]) &&
                    isfinite(un[3]) && isfinite(un[4]) && isfinite(sp);
    if (!ok) nbad = 1;
  }
  const T m = wave_max(smax);
  if ((tid & 63) == 0) sRed[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    T bm = sRed[0];
    for (int i = 1; i < 4; ++i) bm = fmax(bm, sRed[i]);
    atomicMax(&a.clk->smax, pos_bits(bm));
  }
  if (nbad) {
    atomicAdd(&a.clk->bad_count, 1ull);
    atomicMin(&a.clk->bad_first, (unsigned long long)q);
  }
}

// Forcing row records, once per step.  The OU acceleration
//   a_c(x, y, z) = sum_m Re(coef_{m,c} X_{n_x}(x) Y_{n_y}(y) Z_{n_z}(z)),
// coef = 2 * scale * ahat and X_n(x) = exp(2 pi i n (x + 1/2) / n_x) (the
// complex conjugate for n < 0), separates over x: with
//   B_{n,c}(y, z) = sum over modes with n_x = n of coef_{m,c} Y(y) Z(z),
//   P_{n,c} = Re(B_{n,c} + B_{-n,c}),  Q_{n,c} = Im(B_{n,c} - B_{-n,c}),
// a_c = P_{0,c} + sum_{n >= 1} (Re X_n P_{n,c} - Im X_n Q_{n,c}).  One thread
// per (row (y, z), n) writes [n][c][P, Q] of the row's record (6 (R+1) values).
template <typename T>
__global__ __launch_bounds__(256) void k_force_rows(const T* __restrict__ coef,
                                                    const int* __restrict__ nvec, int nmodes,
                                                    const T* __restrict__ tabY,
                                                    const T* __restrict__ tabZ, int ny, int nz,
                                                    int R, T* __restrict__ rows) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)ny * nz * (R + 1)) return;
  const int n = (int)(t % (R + 1));
  const long long row = t / (R + 1);  // z * ny + y
  const int y = (int)(row % ny), z = (int)(row / ny);
  T P[3] = {T(0), T(0), T(0)}, Q[3] = {T(0), T(0), T(0)};
  for (int m = 0; m < nmodes; ++m) {
    const int nxm = nvec[3 * m];
    if (nxm != n && nxm != -n) continue;
    const int nym = nvec[3 * m + 1], nzm = nvec[3 * m + 2];
    const T* ey = tabY + 2 * ((long long)abs(nym) * ny + y);
    const T* ez = tabZ + 2 * ((long long)abs(nzm) * nz + z);
    const T yr = ey[0], yi = nym < 0 ? -ey[1] : ey[1];
    const T zr = ez[0], zi = nzm < 0 ? -ez[1] : ez[1];
    const T er = yr * zr - yi * zi, ei = yr * zi + yi * zr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T cr = coef[6 * m + 2 * c], ci = coef[6 * m + 2 * c + 1];
      const T br = cr * er - ci * ei, bi = cr * ei + ci * er;
      P[c] += br;
      Q[c] += (nxm == n) ? bi : -bi;
    }
  }
  T* out = rows + row * 6 * (R + 1) + 6 * n;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[2 * c] = P[c];
    out[2 * c + 1] = Q[c];
  }
}

template <typename T>
hipError_t launch_force_rows(const T* coef, const int* nvec, int nmodes, const T* tabY,
                             const T* tabZ, int ny, int nz, int R, T* rows, hipStream_t s) {
  const long long total = (long long)ny * nz * (R + 1);
  hipLaunchKernelGGL((k_force_rows<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     coef, nvec, nmodes, tabY, tabZ, ny, nz, R, rows);
  return hipGetLastError();
}

template hipError_t launch_force_rows<float>(const float*, const int*, int, const float*,
                                             const float*, int, int, int, float*, hipStream_t);
template hipError_t launch_force_rows<double>(const double*, const int*, int, const double*,
                                              const double*, int, int, int, double*, hipStream_t);

// CFL signal-speed max of a state (used when no stage-2 epilogue produced it,
// i.e. right after the state was set).
template <typename T>
__global__ __launch_bounds__(256) void k_smax(const T* __restrict__ U, long long N, T gm1, T gamma,
                                              T ihx, T ihy, T ihz, DevClock* clk) {
  __shared__ T sRed[4];
  T smax = T(0);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    T u[5], w[5];
    load_cell(U, N, q, u);
    to_prim(u, gm1, w);
    const T cs = dev_sqrt(gamma * w[4] * dev_rcp(w[0]));
    smax = fmax(smax, fmax(fmax((fabs(w[1]) + cs) * ihx, (fabs(w[2]) + cs) * ihy),
                           (fabs(w[3]) + cs) * ihz));
  }
  T m = wave_max(smax);
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    T bm = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
    atomicMax(&clk->smax, pos_bits(bm));
  }
}

__global__ void k_clock_reset_smax(DevClock* clk) {
  if (threadIdx.x == 0) {
    clk->smax = 0ull;
    clk->crate = 0ull;
  }
}

__global__ void k_clock_reset_health(DevClock* clk) {
  if (threadIdx.x == 0) {
    clk->bad_count = 0ull;
    clk->bad_first = ~0ull;
  }
}

__global__ void k_clock_set(DevClock* clk, double t, long long step) {
  if (threadIdx.x == 0) {
    clk->t = t;
    clk->step = step;
  }
}

// ------------------------------------------------------------------ launchers

static inline int z_chunk(const StageGeom& g) {
  // enough workgroups to fill 256 CUs several times over, long z-marches
  // otherwise (each chunk re-reads 4 planes of prologue)
  const long long tiles_xy = (long long)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  int zc = 64;
  while (zc > 4 && tiles_xy * ((g.nz + zc - 1) / zc) < 4096) zc >>= 1;
  return zc < g.nz ? zc : g.nz;
}

template <typename T>
static void fill_geom(StageArgs<T>& a, const StageGeom& g) {
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  a.bcx = g.bc[0]; a.bcy = g.bc[1]; a.bcz = g.bc[2];
  a.ncell = (long long)g.nx * g.ny * g.nz;
  a.zc = z_chunk(g);
  a.nbx = (g.nx + TX - 1) / TX;
  a.nby = (g.ny + TY - 1) / TY;
  a.nbz = (g.nz + a.zc - 1) / a.zc;
  const int nb = a.nbx * a.nby * a.nbz;
  a.nb_per_xcd = (nb + 7) / 8;
}

template <typename T, int LM>
static void launch_stage_lim(int stage, bool force, bool cool, const StageArgs<T>& a, dim3 grid,
                             dim3 block, hipStream_t s) {
#define MH_LAUNCH(ST, FO, CO) hipLaunchKernelGGL((k_stage<T, ST, LM, FO, CO>), grid, block, 0, s, a)
  if (stage == 1) MH_LAUNCH(1, false, false);
  else if (stage == 3) MH_LAUNCH(3, false, false);
  else if (force && cool) MH_LAUNCH(2, true, true);
  else if (force) MH_LAUNCH(2, true, false);
  else if (cool) MH_LAUNCH(2, false, true);
  else MH_LAUNCH(2, false, false);
#undef MH_LAUNCH
}

template <typename T>
hipError_t launch_stage(int stage, int limiter, bool force, bool cool, StageArgs<T> a,
                        const StageGeom& g, hipStream_t s) {
  // a lane's offset within a z-plane is a 32-bit byte offset
  if ((unsigned long long)g.nx * (unsigned long long)g.ny * sizeof(T) > 0xffffffffull)
    return hipErrorInvalidValue;
  fill_geom(a, g);
  dim3 block(TX, TY);
  dim3 grid(8 * a.nb_per_xcd);
  // every limiter with HLLC: the specialised kernels; another solver, or a
  // flux-correction field: the kernel that reads them at run time
  if (a.rs != RS_HLLC || a.dflux) limiter = LIM_GENERIC;
  if (limiter == LIM_NONE) launch_stage_lim<T, LIM_NONE>(stage, force, cool, a, grid, block, s);
  else if (limiter == LIM_VANLEER)
    launch_stage_lim<T, LIM_VANLEER>(stage, force, cool, a, grid, block, s);
  else if (limiter == LIM_MC) launch_stage_lim<T, LIM_MC>(stage, force, cool, a, grid, block, s);
  else if (limiter == LIM_SUPERBEE)
    launch_stage_lim<T, LIM_SUPERBEE>(stage, force, cool, a, grid, block, s);
  else if (limiter == LIM_GENERIC)
    launch_stage_lim<T, LIM_GENERIC>(stage, force, cool, a, grid, block, s);
  else launch_stage_lim<T, LIM_MINMOD>(stage, force, cool, a, grid, block, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage2_finish(bool cool, StageArgs<T> a, const T* ub, const StageGeom& g,
                                hipStream_t s) {
  fill_geom(a, g);
  const unsigned blocks = (unsigned)((a.ncell + 255) / 256);
  if (cool) hipLaunchKernelGGL((k_stage2_finish<T, true>), dim3(blocks), dim3(256), 0, s, a, ub);
  else hipLaunchKernelGGL((k_stage2_finish<T, false>), dim3(blocks), dim3(256), 0, s, a, ub);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_smax(const T* U, const StageGeom& g, T gamma, const double* ih, DevClock* clk,
                       hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  long long blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_clock_reset_smax, dim3(1), dim3(64), 0, s, clk);
  hipLaunchKernelGGL((k_smax<T>), dim3((unsigned)blocks), dim3(256), 0, s, U, N, gamma - T(1),
                     gamma, (T)ih[0], (T)ih[1], (T)ih[2], clk);
  return hipGetLastError();
}

hipError_t launch_clock_reset_health(DevClock* clk, hipStream_t s) {
  hipLaunchKernelGGL(k_clock_reset_health, dim3(1), dim3(64), 0, s, clk);
  return hipGetLastError();
}

hipError_t launch_clock_set(DevClock* clk, double t, long long step, hipStream_t s) {
  hipLaunchKernelGGL(k_clock_set, dim3(1), dim3(64), 0, s, clk, t, step);
  return hipGetLastError();
}

template hipError_t launch_stage<float>(int, int, bool, bool, StageArgs<float>, const StageGeom&,
                                        hipStream_t);
template hipError_t launch_stage<double>(int, int, bool, bool, StageArgs<double>, const StageGeom&,
                                         hipStream_t);
template hipError_t launch_stage2_finish<float>(bool, StageArgs<float>, const float*,
                                                const StageGeom&, hipStream_t);
template hipError_t launch_stage2_finish<double>(bool, StageArgs<double>, const double*,
                                                 const StageGeom&, hipStream_t);
template hipError_t launch_smax<float>(const float*, const StageGeom&, float, const double*,
                                       DevClock*, hipStream_t);
template hipError_t launch_smax<double>(const double*, const StageGeom&, double, const double*,
                                        DevClock*, hipStream_t);

}  // namespace mh
