// step_kernels.hip -- per-step scalar work on the device: the CFL dt of the
// step, the device clock, and the Ornstein-Uhlenbeck forcing modes
// (arXiv 2512.13403, App. A.4 and Sec. 3.1.1).  One tiny workgroup per step,
// so a run of steps never synchronises with the host.
#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

// Counter-based normal draws for the OU noise.  SplitMix64 (Steele, Lea &
// Flood, OOPSLA 2014): output c of the stream seeded with s is
// mix(s + (c + 1) * 0x9E3779B97F4A7C15).  Two outputs give two uniforms
// (53-bit), the Box-Muller transform gives one complex normal with real and
// imaginary parts ~ N(0, 1/2).  Draw index: ((group + 1) * 64 + mode) * 3 + comp.
__device__ inline unsigned long long sm64(unsigned long long seed, unsigned long long c) {
  unsigned long long z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline void complex_normal(unsigned long long seed, long long group, int mode, int comp,
                                      double& re, double& im) {
  const unsigned long long d =
      ((unsigned long long)(group + 1) * MAX_MODES + (unsigned long long)mode) * 3ull +
      (unsigned long long)comp;
  const unsigned long long x1 = sm64(seed, 2ull * d), x2 = sm64(seed, 2ull * d + 1ull);
  const double u1 = (double)((x1 >> 11) + 1ull) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586 * u2;
  re = r * cos(th) * sqrt(0.5);
  im = r * sin(th) * sqrt(0.5);
}

// M eta with M = zeta P + (1 - zeta) C, P = I - n n^T/|n|^2, C = n n^T/|n|^2
__device__ inline void projected_noise(const OUArgs& a, long long group, int mode,
                                       double (&out)[3][2]) {
  const int* n = a.nvec + 3 * mode;
  double er[3], ei[3];
  for (int c = 0; c < 3; ++c) complex_normal(a.seed, group, mode, c, er[c], ei[c]);
  const double k2 = (double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int i = 0; i < 3; ++i) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < 3; ++j) {
      const double C = (double)n[i] * n[j] / k2;
      const double P = (i == j ? 1.0 : 0.0) - C;
      const double m = a.zeta * P + (1.0 - a.zeta) * C;
      sr += m * er[j];
      si += m * ei[j];
    }
    out[i][0] = sr;
    out[i][1] = si;
  }
}

__global__ void k_ou_init(const OUArgs a) {
  const int m = threadIdx.x;
  if (m < a.nmodes) {
    double pe[3][2];
    projected_noise(a, -1, m, pe);
    for (int c = 0; c < 3; ++c) {
      a.ahat[6 * m + 2 * c] = pe[c][0];
      a.ahat[6 * m + 2 * c + 1] = pe[c][1];
    }
  }
}

// dt of this step, OU update a <- e^{-dt/tau} a + sqrt(1 - e^{-2dt/tau}) M eta,
// the rms normalisation a_rms / sqrt(2 sum |ahat|^2), and the clock advance.
__global__ void k_prologue(const PrologueArgs a) {
  __shared__ double s_dt, s_scale;
  const int t = threadIdx.x;
  DevClock* clk = a.clk;
  if (t == 0) {
    double dt;
    if (a.dt_sched) {
      dt = a.dt_sched[clk->sched_pos * a.sched_stride];
      clk->sched_pos += 1;
    } else if (a.dt_fixed > 0.0) {
      dt = a.dt_fixed;
    } else {
      const double smax = a.f64 ? bits_to_double_f64(clk->smax) : bits_to_double_f32(clk->smax);
      dt = a.cfl / smax;
      if (a.ccool > 0.0) {
        // cooling-time limit of the tabulated cooling model
        const double r = a.f64 ? bits_to_double_f64(clk->crate) : bits_to_double_f32(clk->crate);
        if (r > 0.0 && a.ccool / r < dt) dt = a.ccool / r;
      }
    }
    const double cap = a.t_stop - clk->t;
    if (dt > cap) dt = cap;
    clk->dt = dt;
    a.dt_log[a.log_index] = dt;
    s_dt = dt;
  }
  __syncthreads();
  if (a.forcing) {
    const OUArgs& o = a.ou;
    const long long step = clk->step;
    if (step % o.every == 0 && t < o.nmodes) {
      const double dte = s_dt * o.every;
      const double f = exp(-dte / o.tau);
      const double g = sqrt(1.0 - exp(-2.0 * dte / o.tau));
      double pe[3][2];
      projected_noise(o, step / o.every, t, pe);
      for (int c = 0; c < 3; ++c) {
        o.ahat[6 * t + 2 * c] = f * o.ahat[6 * t + 2 * c] + g * pe[c][0];
        o.ahat[6 * t + 2 * c + 1] = f * o.ahat[6 * t + 2 * c + 1] + g * pe[c][1];
      }
    }
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int q = 0; q < 6 * o.nmodes; ++q) s += o.ahat[q] * o.ahat[q];
      s_scale = o.arms / sqrt(2.0 * s);
      clk->ou_scale = s_scale;
    }
    __syncthreads();
    if (t < o.nmodes) {
      for (int q = 0; q < 6; ++q) {
        const double v = 2.0 * s_scale * o.ahat[6 * t + q];
        if (o.f64) ((double*)o.coef)[6 * t + q] = v;
        else ((float*)o.coef)[6 * t + q] = (float)v;
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    clk->t += s_dt;
    clk->step += 1;
    clk->smax = 0ull;
    clk->crate = 0ull;
  }
}

hipError_t launch_prologue(const PrologueArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue, dim3(1), dim3(MAX_MODES), 0, s, a);
  return hipGetLastError();
}

__global__ void k_sched_reset(DevClock* clk) {
  if (threadIdx.x == 0) clk->sched_pos = 0;
}

hipError_t launch_sched_reset(DevClock* clk, hipStream_t s) {
  hipLaunchKernelGGL(k_sched_reset, dim3(1), dim3(64), 0, s, clk);
  return hipGetLastError();
}

// plain device copy in 16-byte words (the corrected step's gathers and
// scatters, as kernels so that a captured step holds no copy nodes)
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}
__global__ void k_copy1(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                        size_t n) {
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16) {
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src,
                       (uint4*)dst, n16);
  }
  if (bytes % 16)
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, s, (const unsigned char*)src + 16 * n16,
                       (unsigned char*)dst + 16 * n16, bytes % 16);
  return hipGetLastError();
}

// One ADAM update of `count` parameters in place (Kingma & Ba 2015):
// m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// theta -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^it, c2 = 1 - b2^it.
template <typename T>
__global__ __launch_bounds__(256) void k_adam_any(T* __restrict__ th, T* __restrict__ m,
                                                  T* __restrict__ v, const T* __restrict__ g,
                                                  long long count, T lr, T b1, T b2, T eps, T c1,
                                                  T c2) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (long long)gridDim.x * 256) {
    const T gi = g[i];
    const T mi = b1 * m[i] + (T(1) - b1) * gi;
    const T vi = b2 * v[i] + (T(1) - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
  }
}

template <typename T>
hipError_t launch_adam(T* th, T* m, T* v, const T* g, long long count, double lr, double b1,
                       double b2, double eps, long long it, hipStream_t s) {
  const double c1 = 1.0 - pow(b1, (double)it), c2 = 1.0 - pow(b2, (double)it);
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_adam_any<T>), dim3((unsigned)blocks), dim3(256), 0, s, th, m, v, g, count,
                     (T)lr, (T)b1, (T)b2, (T)eps, (T)c1, (T)c2);
  return hipGetLastError();
}
template hipError_t launch_adam<float>(float*, float*, float*, const float*, long long, double,
                                       double, double, double, long long, hipStream_t);
template hipError_t launch_adam<double>(double*, double*, double*, const double*, long long,
                                        double, double, double, double, long long, hipStream_t);

hipError_t launch_ou_init(const OUArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_ou_init, dim3(1), dim3(MAX_MODES), 0, s, a);
  return hipGetLastError();
}

}  // namespace mh
