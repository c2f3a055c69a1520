// mh_device.h -- device-side types and helpers shared by the HIP kernels of
// libmihydro (gfx950 only).  Internal: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mh {

// Tile of the fused stage kernel: one thread per (x, y) column of a 64 x 8
// tile (one wave64 per row), marching along z through a chunk of planes.
constexpr int TX = 64;
constexpr int TY = 8;
constexpr int NTHREADS = TX * TY;
constexpr int MAX_MODES = 64;   // OU modes
constexpr int MAX_R = 8;        // largest |n_a| of a forced OU mode
constexpr int MAX_ZC = 64;      // longest z-chunk of the stage kernel
constexpr int DTLOG_CAP = 4096; // per-step dt records kept on the device

// Device clock and per-step scalars, written by one thread of the prologue
// kernel and read by every stage kernel of the same step.
struct DevClock {
  double t;                 // simulated time at the start of the next step
  double dt;                // dt of the step in flight
  int64_t step;             // global index of the next step
  unsigned long long smax;  // bit pattern of max_a (|v_a|+c)/h_a (float or double)
  unsigned long long bad_count;
  unsigned long long bad_first;
  double ou_scale;
  int32_t mg_cycles;
  int32_t pad;
  double mg_fnorm2;         // ||F||^2 of the current gravity solve
  double mg_rnorm2;         // ||r||^2 of the last residual
  double mean;              // scratch: mean of a field
  unsigned long long crate; // bit pattern of max |Edot| / E_th (tabulated cooling)
  long long sched_pos;      // next entry of a device dt schedule (batched corrected steps)
};

enum : int { BC_PERIODIC = 0, BC_OUTFLOW = 1 };
enum : int { LIM_MINMOD = 0, LIM_NONE = 1, LIM_VANLEER = 2, LIM_MC = 3, LIM_SUPERBEE = 4 };
enum : int { COOLINT_TRAPEZOID = 0, COOLINT_SUBCYCLE = 1, COOLINT_AUTO = 2 };
// template tag of the stage kernel that selects limiter and solver at run time
enum : int { LIM_GENERIC = 15 };
enum : int { RS_HLLC = 0, RS_HLL = 1, RS_RUSANOV = 2 };

__device__ __forceinline__ int bc_map(int i, int n, int bc) {
  if ((unsigned)i < (unsigned)n) return i;
  if (bc == BC_PERIODIC) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : n - 1;
}

template <typename T> __device__ __forceinline__ T dev_rcp(T x);
template <> __device__ __forceinline__ float dev_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
// fp64: the hardware estimate refined by two Newton steps r <- r + r (1 - x r)
// (each squares the relative error: a few ulp at most, against the ~10
// instructions of an IEEE division sequence)
template <> __device__ __forceinline__ double dev_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// 1 / sqrt(x): fp32 hardware instruction; fp64 estimate refined by two Newton
// steps y <- y + (y/2)(1 - x y^2)
__device__ __forceinline__ float dev_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double dev_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  return __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
}

template <typename T> __device__ __forceinline__ T dev_sqrt(T x);
template <> __device__ __forceinline__ float dev_sqrt<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}
template <> __device__ __forceinline__ double dev_sqrt<double>(double x) { return sqrt(x); }

// transcendentals of the cooling source: the hardware instructions in fp32
// (about 1 ulp for sqrt, a few ulp for log/exp, far inside the fp32 parity
// tolerance), correctly rounded library calls in fp64
__device__ __forceinline__ float acc_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double acc_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float acc_log(float x) { return __logf(x); }
__device__ __forceinline__ double acc_log(double x) { return log(x); }
__device__ __forceinline__ float acc_exp(float x) { return __expf(x); }
__device__ __forceinline__ double acc_exp(double x) { return exp(x); }

// order-preserving bit pattern of a non-negative value, for atomicMax
__device__ __forceinline__ unsigned long long pos_bits(float v) {
  return (unsigned long long)__float_as_uint(v);
}
__device__ __forceinline__ unsigned long long pos_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__host__ __device__ inline double bits_to_double_f32(unsigned long long b) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)b;
  return (double)c.f;
}
__host__ __device__ inline double bits_to_double_f64(unsigned long long b) {
  union { unsigned long long u; double d; } c;
  c.u = b;
  return c.d;
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Cooling constants.  k1r = (gamma-1) L0 / (2 sqrt(tc)) and k2r = (gamma-1) L0 / ts
// are the per-unit-density rates at which sqrt(T) falls above tc and
// exp(-(T - tc)/ts) rises below tc.
template <typename T>
struct CoolParams {
  T tc, ts, its, tfloor, sqrt_tc, k1r, k2r;  // its = 1 / ts
};

// the tabulated heating/cooling model (cool_kernels.hip)
template <typename T>
struct CoolTable {
  const T* logT;  // [ntab] log10 T
  const T* logL;  // [ntab] log10 Lambda
  int ntab, integ, nsub_max, rate;  // rate: reduce max |Edot|/E_th
  T tc, tfloor, L1, a1, L2, a2, heat, frac;
};

// a * b + c in one rounding (v_fma_f32 / v_fma_f64), written out where a
// fused multiply-add is wanted, so that results do not depend on whether the
// compiler contracts the expression at a given call site
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ void to_prim(const T (&u)[5], T gm1, T (&w)[5]) {
  const T ir = dev_rcp(u[0]);
  const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  w[0] = u[0];
  w[1] = vx;
  w[2] = vy;
  w[3] = vz;
  w[4] = gm1 * fmad(-(T(0.5) * u[0]), fmad(vx, vx, fmad(vy, vy, vz * vz)), u[4]);
}

template <typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ U, long long N, long long q,
                                          T (&u)[5]) {
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f] = U[f * N + q];
}

// Exact isochoric cooling of one cell over dt (closed form on each branch of
// the two-branch curve), then the temperature floor; returns the new T.
template <typename T>
__device__ __forceinline__ T cool_T(T rho, T Tin, T dt, const CoolParams<T>& c) {
  const T k2 = c.k2r * rho;
  T Tn;
  if (Tin >= c.tc) {
    const T k1 = c.k1r * rho;
    const T st = acc_sqrt(Tin);
    const T t1 = (st - c.sqrt_tc) * dev_rcp(k1);
    if (dt <= t1) {
      const T s = fmad(-k1, dt, st);
      Tn = s * s;
    } else {
      Tn = fmad(-c.ts, acc_log(fmad(k2, dt - t1, T(1))), c.tc);
    }
  } else {
    Tn = fmad(-c.ts, acc_log(fmad(k2, dt, acc_exp((c.tc - Tin) * c.its))), c.tc);
  }
  return fmax(Tn, c.tfloor);
}

}  // namespace mh
