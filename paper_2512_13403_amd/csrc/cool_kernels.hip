// cool_kernels.hip -- the paper's tabulated heating/cooling model on the
// device (arXiv 2512.13403, Sec. 4.1-4.3), the optional replacement of the
// exact two-branch cooling fused into the last stage kernel.
//
// In code units (n = rho, T = P/rho) the thermal energy density E_th =
// rho T/(gamma-1) of a cell changes at fixed rho and momentum as
//   dE_th/dt = rho Gamma(T) - rho^2 Lambda(T),
//   Lambda = L1 T^a1 + L2 T^a2, Gamma = heat          for T <  tc,
//   Lambda = 10^(log-log interpolation of the table), Gamma = 0   for T >= tc
// (the table used flat beyond its ends).  One operator-split step dt:
// trapezoid (E* = E + dt Edot(E), E' = E + dt/2 (Edot(E) + Edot(E*))),
// subcycled (N = ceil(dt |Edot| / (f E)) <= N_max substeps, each changing E
// by at most f E), or auto (trapezoid when dt |Edot| <= f E); E_th is floored
// at rho T_floor/(gamma-1) on entry and after every update.
//
// k_cool_table runs after the last stage (and after gravity, when on) as the
// final per-cell kernel of the step: cooling, then the CFL signal speed, the
// health check and, for the cooling-time step limit, max |Edot| / E_th of the
// new state, all reduced into the device clock for the next step.
#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

namespace {

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }
// grid of a grid-stride kernel that ends in one clock atomic per block
inline unsigned nblk_capped(long long n) { return nblk(n) < 4096u ? nblk(n) : 4096u; }

__device__ __forceinline__ float dpow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double dpow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float dlog10(float x) { return log10f(x); }
__device__ __forceinline__ double dlog10(double x) { return log10(x); }
__device__ __forceinline__ float dexp10(float x) { return exp10f(x); }
__device__ __forceinline__ double dexp10(double x) { return exp10(x); }

template <typename T>
__device__ T cool_lambda(const CoolTable<T>& c, T temp) {
  if (temp < c.tc) return c.L1 * dpow(temp, c.a1) + c.L2 * dpow(temp, c.a2);
  const T x = dlog10(temp);
  const int n = c.ntab;
  if (x <= c.logT[0]) return dexp10(c.logL[0]);
  if (x >= c.logT[n - 1]) return dexp10(c.logL[n - 1]);
  // logT[i] <= x < logT[i+1]; the bound (which a finite x inside the table
  // never reaches) keeps a NaN temperature from reading past the table
  int i = 0;
  while (i < n - 2 && !(x < c.logT[i + 1])) ++i;
  const T w = (x - c.logT[i]) / (c.logT[i + 1] - c.logT[i]);
  return dexp10(c.logL[i] + w * (c.logL[i + 1] - c.logL[i]));
}

template <typename T>
__device__ __forceinline__ T cool_edot(const CoolTable<T>& c, T rho, T E, T gm1) {
  const T temp = gm1 * E / rho;
  const T heat = temp < c.tc ? c.heat : T(0);
  return rho * heat - rho * rho * cool_lambda(c, temp);
}

template <typename T>
__device__ T cool_eth_step(const CoolTable<T>& c, T rho, T E, T dt, T gm1) {
  const T Ef = rho * c.tfloor / gm1;
  E = fmax(E, Ef);
  const T d0 = cool_edot(c, rho, E, gm1);
  int m = c.integ;
  if (m == COOLINT_AUTO) m = dt * fabs(d0) <= c.frac * E ? COOLINT_TRAPEZOID : COOLINT_SUBCYCLE;
  if (m == COOLINT_TRAPEZOID) {
    const T Ep = fmax(E + dt * d0, Ef);
    const T d1 = cool_edot(c, rho, Ep, gm1);
    return fmax(E + T(0.5) * dt * (d0 + d1), Ef);
  }
  const double nd = ceil((double)(dt * fabs(d0)) / (double)(c.frac * E));
  // (a NaN count, from a non-finite cell, takes one substep)
  const int N = !(nd >= 1.0) ? 1 : (nd > (double)c.nsub_max ? c.nsub_max : (int)nd);
  const T h = dt / (T)N;
  for (int k = 0; k < N; ++k) {
    T dE = (k == 0 ? d0 : cool_edot(c, rho, E, gm1)) * h;
    const T lim = c.frac * E;
    dE = fmin(fmax(dE, -lim), lim);
    E = fmax(E + dE, Ef);
  }
  return E;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cool_table(T* U, long long N, T gamma, T ihx, T ihy,
                                                    T ihz, CoolTable<T> c, DevClock* clk) {
  __shared__ T sRed[4], sRate[4];
  const T dt = (T)clk->dt;
  const T gm1 = gamma - T(1);
  T s = T(0), r = T(0);
  unsigned long long bad = 0, first_bad = ~0ull;
  // grid-stride over the cells, so that a capped grid issues few clock atomics
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < N;
       q += (long long)gridDim.x * 256) {
    T u[5];
    load_cell(U, N, q, u);
    const T ek = T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    const T E = cool_eth_step(c, u[0], u[4] - ek, dt, gm1);
    u[4] = ek + E;
    U[4 * N + q] = u[4];
    if (c.rate) r = fmax(r, fabs(cool_edot(c, u[0], E, gm1)) / E);
    T w[5];
    to_prim(u, gm1, w);
    const T cs = dev_sqrt(gamma * w[4] * dev_rcp(w[0]));
    const T sq =
        fmax(fmax((fabs(w[1]) + cs) * ihx, (fabs(w[2]) + cs) * ihy), (fabs(w[3]) + cs) * ihz);
    s = fmax(s, sq);
    const bool ok = (w[0] > T(0)) && (w[4] > T(0)) && isfinite(u[1]) && isfinite(u[2]) &&
                    isfinite(u[3]) && isfinite(u[4]) && isfinite(sq);
    if (!ok) {
      ++bad;
      if ((unsigned long long)q < first_bad) first_bad = (unsigned long long)q;
    }
  }
  const T m = wave_max(s);
  const T mr = wave_max(r);
  if ((threadIdx.x & 63) == 0) {
    sRed[threadIdx.x >> 6] = m;
    sRate[threadIdx.x >> 6] = mr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&clk->smax, pos_bits(fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]))));
    if (c.rate)
      atomicMax(&clk->crate, pos_bits(fmax(fmax(sRate[0], sRate[1]), fmax(sRate[2], sRate[3]))));
  }
  if (bad) {
    atomicAdd(&clk->bad_count, bad);
    atomicMin(&clk->bad_first, first_bad);
  }
}

// ---- reverse pass: the step's partial derivatives in forward mode ----------
// dLambda/dT on the branch taken (0 beyond the table's ends)
template <typename T>
__device__ T cool_lambda_dT(const CoolTable<T>& c, T temp) {
  if (temp < c.tc)
    return c.L1 * c.a1 * dpow(temp, c.a1 - T(1)) + c.L2 * c.a2 * dpow(temp, c.a2 - T(1));
  const T x = dlog10(temp);
  const int n = c.ntab;
  if (x <= c.logT[0] || x >= c.logT[n - 1]) return T(0);
  int i = 0;
  while (i < n - 2 && !(x < c.logT[i + 1])) ++i;  // bounded as in cool_lambda
  const T s = (c.logL[i + 1] - c.logL[i]) / (c.logT[i + 1] - c.logT[i]);
  return s * cool_lambda(c, temp) / temp;
}

// a value with its derivatives with respect to the step's inputs E_th, rho
template <typename T>
struct Dual2 {
  T v, dE, dr;
};

template <typename T>
__device__ Dual2<T> cool_edot_d(const CoolTable<T>& c, T rho, Dual2<T> E, T gm1) {
  const T temp = gm1 * E.v / rho;
  const T heat = temp < c.tc ? c.heat : T(0);
  const T L = cool_lambda(c, temp), Lp = cool_lambda_dT(c, temp);
  const T pE = -gm1 * rho * Lp;
  const T pr = heat - T(2) * rho * L + rho * temp * Lp;
  return Dual2<T>{rho * heat - rho * rho * L, pE * E.dE, pE * E.dr + pr};
}

template <typename T>
__device__ __forceinline__ Dual2<T> cool_floor_d(const CoolTable<T>& c, T rho, Dual2<T> E,
                                                 T gm1) {
  const T Ef = rho * c.tfloor / gm1;
  if (E.v > Ef) return E;
  return Dual2<T>{Ef, T(0), c.tfloor / gm1};
}

// the step's result with dE'/dE_th and dE'/drho, branches as the forward
template <typename T>
__device__ Dual2<T> cool_eth_step_d(const CoolTable<T>& c, T rho, T Eth, T dt, T gm1) {
  Dual2<T> E = cool_floor_d(c, rho, Dual2<T>{Eth, T(1), T(0)}, gm1);
  const Dual2<T> d0 = cool_edot_d(c, rho, E, gm1);
  int m = c.integ;
  if (m == COOLINT_AUTO)
    m = dt * fabs(d0.v) <= c.frac * E.v ? COOLINT_TRAPEZOID : COOLINT_SUBCYCLE;
  if (m == COOLINT_TRAPEZOID) {
    const Dual2<T> Ep = cool_floor_d(
        c, rho, Dual2<T>{E.v + dt * d0.v, E.dE + dt * d0.dE, E.dr + dt * d0.dr}, gm1);
    const Dual2<T> d1 = cool_edot_d(c, rho, Ep, gm1);
    return cool_floor_d(c, rho,
                        Dual2<T>{E.v + T(0.5) * dt * (d0.v + d1.v),
                                 E.dE + T(0.5) * dt * (d0.dE + d1.dE),
                                 E.dr + T(0.5) * dt * (d0.dr + d1.dr)},
                        gm1);
  }
  const double nd = ceil((double)(dt * fabs(d0.v)) / (double)(c.frac * E.v));
  // (a NaN count, from a non-finite cell, takes one substep)
  const int N = !(nd >= 1.0) ? 1 : (nd > (double)c.nsub_max ? c.nsub_max : (int)nd);
  const T h = dt / (T)N;
  for (int k = 0; k < N; ++k) {
    const Dual2<T> d = k == 0 ? d0 : cool_edot_d(c, rho, E, gm1);
    Dual2<T> dE{d.v * h, d.dE * h, d.dr * h};
    const Dual2<T> lim{c.frac * E.v, c.frac * E.dE, c.frac * E.dr};
    if (dE.v > lim.v) dE = lim;
    if (dE.v < -lim.v) dE = Dual2<T>{-lim.v, -lim.dE, -lim.dr};
    E = cool_floor_d(c, rho, Dual2<T>{E.v + dE.v, E.dE + dE.dE, E.dr + dE.dr}, gm1);
  }
  return E;
}

// reverse of the cooling of one cell at the state U it acted on:
// E' = ek + C(rho, E - ek), ek = |m|^2/(2 rho)
template <typename T>
__global__ __launch_bounds__(256) void k_cool_table_vjp(const T* __restrict__ U, long long N,
                                                        T gamma, T dt, CoolTable<T> c,
                                                        const T* __restrict__ lin, T* lout) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const T gm1 = gamma - T(1);
  const T rho = U[q], mx = U[N + q], my = U[2 * N + q], mz = U[3 * N + q];
  const T ek = T(0.5) * (mx * mx + my * my + mz * mz) / rho;
  const Dual2<T> r = cool_eth_step_d(c, rho, U[4 * N + q] - ek, dt, gm1);
  const T Eb = lin[4 * N + q];
  const T ekb = Eb * (T(1) - r.dE);
  lout[q] = lin[q] + Eb * r.dr - ekb * ek / rho;
  lout[N + q] = lin[N + q] + ekb * mx / rho;
  lout[2 * N + q] = lin[2 * N + q] + ekb * my / rho;
  lout[3 * N + q] = lin[3 * N + q] + ekb * mz / rho;
  lout[4 * N + q] = Eb * r.dE;
}

// max |Edot| / E_th of a state (the first step's cooling-time limit)
template <typename T>
__global__ __launch_bounds__(256) void k_cool_rate(const T* __restrict__ U, long long N, T gamma,
                                                   CoolTable<T> c, DevClock* clk) {
  __shared__ T sRate[4];
  const T gm1 = gamma - T(1);
  T r = T(0);
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < N;
       q += (long long)gridDim.x * 256) {
    T u[5];
    load_cell(U, N, q, u);
    const T E = u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    r = fmax(r, fabs(cool_edot(c, u[0], E, gm1)) / E);
  }
  const T mr = wave_max(r);
  if ((threadIdx.x & 63) == 0) sRate[threadIdx.x >> 6] = mr;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(&clk->crate, pos_bits(fmax(fmax(sRate[0], sRate[1]), fmax(sRate[2], sRate[3]))));
}

}  // namespace

template <typename T>
hipError_t launch_cool_table(T* U, const StageGeom& g, T gamma, const double* ih,
                             const CoolTable<T>& c, DevClock* clk, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL((k_cool_table<T>), dim3(nblk_capped(N)), dim3(256), 0, s, U, N, gamma, (T)ih[0],
                     (T)ih[1], (T)ih[2], c, clk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cool_rate(const T* U, const StageGeom& g, T gamma, const CoolTable<T>& c,
                            DevClock* clk, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL((k_cool_rate<T>), dim3(nblk_capped(N)), dim3(256), 0, s, U, N, gamma, c, clk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cool_table_vjp(const T* U, long long N, T gamma, T dt, const CoolTable<T>& c,
                                 const T* lin, T* lout, hipStream_t s) {
  hipLaunchKernelGGL((k_cool_table_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, U, N, gamma, dt, c,
                     lin, lout);
  return hipGetLastError();
}

template hipError_t launch_cool_table_vjp<float>(const float*, long long, float, float,
                                                 const CoolTable<float>&, const float*, float*,
                                                 hipStream_t);
template hipError_t launch_cool_table_vjp<double>(const double*, long long, double, double,
                                                  const CoolTable<double>&, const double*,
                                                  double*, hipStream_t);
template hipError_t launch_cool_table<float>(float*, const StageGeom&, float, const double*,
                                             const CoolTable<float>&, DevClock*, hipStream_t);
template hipError_t launch_cool_table<double>(double*, const StageGeom&, double, const double*,
                                              const CoolTable<double>&, DevClock*, hipStream_t);
template hipError_t launch_cool_rate<float>(const float*, const StageGeom&, float,
                                            const CoolTable<float>&, DevClock*, hipStream_t);
template hipError_t launch_cool_rate<double>(const double*, const StageGeom&, double,
                                             const CoolTable<double>&, DevClock*, hipStream_t);

}  // namespace mh
