// mg_kernels.hip -- geometric multigrid Poisson solver and gravity source on
// the device (arXiv 2512.13403, Sec. 6, 6.2 and App. C).
//
// The discrete problem is A phi = F on the periodic n^3 cube, A the
// seven-point Laplacian, F = 4 pi G (rho - <rho>).  One V-cycle: nu1 weighted
// Jacobi sweeps (omega = 2/3) or red-black Gauss-Seidel sweeps, residual,
// restriction by the mean of the 8 children, the coarse error equation solved
// recursively from zero, cell-centred trilinear prolongation (per axis 3/4
// parent + 1/4 neighbour on the child's side) and correction, nu2 sweeps; the
// coarsest grid is solved by many Jacobi sweeps inside one workgroup.  The
// W-cycle (the paper's default, App. C) solves each coarse error equation
// with two recursive cycles, the second from the first one's result (one
// solve where the next level is the coarsest).  Means are removed from every
// restricted right-hand side and from phi after every cycle (gauge <phi> = 0).
// All reductions are two-stage with fixed block counts, so results do not
// depend on scheduling.  Every kernel here is memory-bound (about 2 field
// reads and 1 write per cell per sweep).
#include <cmath>

#include "mg.h"
#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T nb6(const T* __restrict__ p, int n, int i, int j, int k) {
  const long long n2 = (long long)n * n;
  const int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
  const int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
  const int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
  const long long row = (long long)k * n2 + (long long)j * n;
  return p[row + im] + p[row + ip] + p[(long long)k * n2 + (long long)jm * n + i] +
         p[(long long)k * n2 + (long long)jp * n + i] + p[(long long)km * n2 + (long long)j * n + i] +
         p[(long long)kp * n2 + (long long)j * n + i];
}

// a fixed tree inside each wave: lane l adds lane l + s for s = 32, 16, ...,
// 1 (lane 0 holds the wave's sum)
__device__ __forceinline__ double wave_tree_sum(double v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_down(v, s, 64);
  return v;
}

// the sum of v over a 256-thread block, returned to every thread: the four
// wave sums added pairwise
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  const int t = threadIdx.x;
  v = wave_tree_sum(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <typename T, bool SQUARE>
__global__ __launch_bounds__(256) void k_sum_partial(const T* __restrict__ x, long long n,
                                                     double* __restrict__ partial) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long long)gridDim.x * 256) {
    const double v = (double)x[q];
    s += SQUARE ? v * v : v;
  }
  const double b = block_sum256(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// out = sum(partial[0..nb)) * scale, written to a clock field
__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int nb,
                                                   double scale, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += partial[i];
  const double b = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = b * scale;
}

// y = scale * (x - *mean)   (in place allowed)
template <typename T>
__global__ __launch_bounds__(256) void k_shift_scale(T* y, const T* x, long long n,
                                                     const double* mean, double scale) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) y[q] = (T)(scale * ((double)x[q] - *mean));
}

template <typename T>
__global__ __launch_bounds__(256) void k_sub_mean(T* y, long long n, const double* mean) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) y[q] = y[q] - (T)(*mean);
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T* y, long long n) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < n) y[q] = T(0);
}

// phi' = (1 - w) phi + (w/6)(sum of neighbours - h^2 F), w = 2/3
template <typename T>
__global__ __launch_bounds__(256) void k_jacobi(int n, T h2, const T* __restrict__ phi,
                                                const T* __restrict__ F, T* __restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;  // launched by plane_grid(n * n, n)
  if (p >= n * n) return;
  const int k = blockIdx.y, j = p / n, i = p - j * n;
  const long long q = (long long)k * n * n + p;
  const T w = T(2) / T(3);
  out[q] = (T(1) - w) * phi[q] + (w / T(6)) * (nb6(phi, n, i, j, k) - h2 * F[q]);
}

// one half of a red-black Gauss-Seidel sweep, in place: every cell of the
// colour (i + j + k) mod 2 = `colour` is set to (sum of neighbours - h^2 F)/6;
// the smoothed levels have an even n, so those cells read only the other
// colour
template <typename T>
__global__ __launch_bounds__(256) void k_rbgs(int n, T h2, T* phi, const T* __restrict__ F,
                                              int colour) {
  // one thread per cell of the colour: the n/2 cells of a row with
  // (i + j + k) mod 2 = colour, launched by plane_grid(n / 2 * n, n)
  const int nh = n >> 1;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nh * n) return;
  const int k = blockIdx.y, j = p / nh, i = 2 * (p - j * nh) + ((j + k + colour) & 1);
  const long long q = ((long long)k * n + j) * n + i;
  phi[q] = (nb6(phi, n, i, j, k) - h2 * F[q]) / T(6);
}

// the residual F - A phi at cell q = (i, j, k) of an n^3 grid
template <typename T>
__device__ __forceinline__ T residual_at(const T* __restrict__ phi, const T* __restrict__ F, int n,
                                         T ih2, int i, int j, int k, long long q) {
  return F[q] - (nb6(phi, n, i, j, k) - T(6) * phi[q]) * ih2;
}

// |F - A phi|^2 summed per block in the order of k_sum_partial<T, true>
// over the residual array (the same grid, cells and per-block tree), without
// storing the residual (cells are indexed in 32 bits: a grid holds at most
// 2^31 cells)
template <typename T>
__global__ __launch_bounds__(256) void k_residual_norm2(int n, T ih2, const T* __restrict__ phi,
                                                        const T* __restrict__ F,
                                                        double* __restrict__ partial) {
  __shared__ double sh[256];
  const unsigned n2 = (unsigned)n * (unsigned)n, N = n2 * (unsigned)n;
  double acc = 0.0;
  for (unsigned q = blockIdx.x * 256 + threadIdx.x; q < N; q += gridDim.x * 256) {
    const int k = (int)(q / n2), rem = (int)(q - (unsigned)k * n2), j = rem / n, i = rem - j * n;
    const T r = residual_at(phi, F, n, ih2, i, j, k, (long long)q);
    const double v = (double)r;
    acc += v * v;
  }
  const double b = block_sum256(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// restriction of the residual, F_c = average over the 8 children of
// F - A phi (residual_at, summed in child order): each
// coarse cell forms its children's residuals in registers, so the fine
// residual is never stored.  The coarse cells are visited in the order of
// k_sum_partial<T, false> over F_c (same grid, cells and per-block tree), and
// each block's sum of its F_c values is written to `partial`, so the mean of
// F_c needs only k_sum_final.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_restrict(int nc, T ih2, const T* __restrict__ phi,
                                                           const T* __restrict__ F,
                                                           T* __restrict__ rc,
                                                           double* __restrict__ partial) {
  __shared__ double sh[256];
  const unsigned nc2 = (unsigned)nc * (unsigned)nc, Nc = nc2 * (unsigned)nc;
  const int nf = 2 * nc;
  const long long nf2 = (long long)nf * nf;
  double acc = 0.0;
  for (unsigned q = blockIdx.x * 256 + threadIdx.x; q < Nc; q += gridDim.x * 256) {
    const int K = (int)(q / nc2), rem = (int)(q - (unsigned)K * nc2), J = rem / nc,
              I = rem - J * nc;
    T s = T(0);
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
          const long long f = (long long)k * nf2 + (long long)j * nf + i;
          s += residual_at(phi, F, nf, ih2, i, j, k, f);
        }
    const T v = T(0.125) * s;
    rc[q] = v;
    acc += (double)v;
  }
  const double b = block_sum256(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(int nc, const T* __restrict__ ec, T* __restrict__ phif) {
  const int nf = 2 * nc;
  const int p = blockIdx.x * 256 + threadIdx.x;  // launched by plane_grid(nf * nf, nf)
  if (p >= nf * nf) return;
  const int k = blockIdx.y, j = p / nf, i = p - j * nf;
  const long long q = (long long)k * nf * nf + p;
  const int I = i >> 1, J = j >> 1, K = k >> 1;
  const int I2 = wrapi(I + ((i & 1) ? 1 : -1), nc);
  const int J2 = wrapi(J + ((j & 1) ? 1 : -1), nc);
  const int K2 = wrapi(K + ((k & 1) ? 1 : -1), nc);
  const long long nc2 = (long long)nc * nc;
  auto at = [&](int a, int b, int c) { return ec[(long long)c * nc2 + (long long)b * nc + a]; };
  const T w0 = T(0.75), w1 = T(0.25);
  T e = T(0);
  e += w0 * w0 * w0 * at(I, J, K);
  e += w1 * w0 * w0 * at(I2, J, K);
  e += w0 * w1 * w0 * at(I, J2, K);
  e += w1 * w1 * w0 * at(I2, J2, K);
  e += w0 * w0 * w1 * at(I, J, K2);
  e += w1 * w0 * w1 * at(I2, J, K2);
  e += w0 * w1 * w1 * at(I, J2, K2);
  e += w1 * w1 * w1 * at(I2, J2, K2);
  phif[q] += e;
}

// coarsest grid: phi = 0, `sweeps` Jacobi sweeps, remove the mean; one
// workgroup of 256 threads, the whole grid (<= 4096 cells) in LDS
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(int n, T h2, const T* __restrict__ F,
                                                      T* __restrict__ phi, int sweeps) {
  __shared__ T a[MG_COARSE_MAX_CELLS], b[MG_COARSE_MAX_CELLS], f[MG_COARSE_MAX_CELLS];
  __shared__ double sh[256];
  const int N = n * n * n;
  for (int q = threadIdx.x; q < N; q += 256) {
    a[q] = T(0);
    f[q] = F[q];  // the right-hand side stays in LDS for all sweeps
  }
  __syncthreads();
  const T w = T(2) / T(3);
  T* src = a;
  T* dst = b;
  for (int s = 0; s < sweeps; ++s) {
    for (int q = threadIdx.x; q < N; q += 256) {
      const int i = q % n, j = (q / n) % n, k = q / (n * n);
      dst[q] = (T(1) - w) * src[q] + (w / T(6)) * (nb6(src, n, i, j, k) - h2 * f[q]);
    }
    __syncthreads();
    T* t = src;
    src = dst;
    dst = t;
  }
  double s = 0.0;
  for (int q = threadIdx.x; q < N; q += 256) s += (double)src[q];
  const double mean = block_sum256(s, sh) / (double)N;
  for (int q = threadIdx.x; q < N; q += 256) phi[q] = src[q] - (T)mean;
}

// The bottom of the cycle in one workgroup.  Every level with at most
// MG_TAIL_MAX_CELLS cells lives in LDS (the levels below a 16^3 level take
// 4096 + 512 + 64 + ... cells), so the many small launches those levels would
// cost (sweeps, residual, restriction, mean removal, coarse solve,
// prolongation) become one.  On entry F of the tail's first level is its
// restricted, mean-free right-hand side and its phi starts from zero, or from
// phi0 (`warm`: the second cycle of a W-cycle); on exit phi0 holds the result.
// Inside, the V- or W-cycle over the tail's levels runs as a loop over an
// explicit per-level count of the coarse cycles still to do.  The arithmetic
// of each step is that of the corresponding kernel above; the means are
// summed with a different fixed tree.
constexpr int MG_TAIL_MAX_CELLS = 4096;
constexpr int MG_TAIL_ALLOC = 4688;  // >= 4096 * 8 / 7: all levels of the tail
constexpr int MG_TAIL_THREADS = 1024;

template <typename T>
struct TailArgs {
  int nl;                    // levels in the tail (>= 2)
  int n[MG_MAX_LEVELS];      // cells per axis
  T h2[MG_MAX_LEVELS];       // h^2
  T ih2[MG_MAX_LEVELS];      // 1 / h^2
  int off[MG_MAX_LEVELS];    // offset of each level in the LDS arrays
  const T* F0;               // right-hand side of the first level (global)
  T* phi0;                   // its phi (global: read when warm, written)
  int pre, post, csweeps;
  int wcycle;                // 1: two coarse cycles per level (W), 0: one (V)
  int rbgs;                  // smoother: 1 red-black Gauss-Seidel, 0 Jacobi
  int warm;                  // start the first level from phi0
};

// the sum of v over the workgroup, returned to every thread: a fixed tree
// inside each wave, then the same over the 16 wave sums
__device__ __forceinline__ double block_sum1024(double v, double* sh) {
  static_assert(MG_TAIL_THREADS == 1024, "16 waves");
  const int t = threadIdx.x;
  v = wave_tree_sum(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t < 64) {
    double w = t < 16 ? sh[t] : 0.0;
    for (int s = 8; s > 0; s >>= 1) w += __shfl_down(w, s, 64);
    if (t == 0) sh[16] = w;
  }
  __syncthreads();
  const double r = sh[16];
  __syncthreads();
  return r;
}

template <typename T>
__device__ void tail_sweeps(T* pa, T* pb, const T* ff, int o, int n, T h2, int sweeps, int& cur) {
  const int N = n * n * n;
  const T w = T(2) / T(3);
  for (int it = 0; it < sweeps; ++it) {
    const T* src = (cur ? pb : pa) + o;
    T* dst = (cur ? pa : pb) + o;
    for (int q = threadIdx.x; q < N; q += MG_TAIL_THREADS) {
      const int i = q % n, j = (q / n) % n, k = q / (n * n);
      dst[q] = (T(1) - w) * src[q] + (w / T(6)) * (nb6(src, n, i, j, k) - h2 * ff[o + q]);
    }
    __syncthreads();
    cur ^= 1;
  }
}

// The same sweeps on a level of at most 64 cells (the coarsest level): one
// wave, a cell per lane, so no workgroup barrier is needed between sweeps
// (a wave's LDS accesses complete in program order; the fences only keep the
// compiler from moving them).  Same arithmetic as tail_sweeps.
template <typename T>
__device__ void tail_sweeps_wave(T* pa, T* pb, const T* ff, int o, int n, T h2, int sweeps,
                                 int& cur) {
  const int N = n * n * n;
  const T w = T(2) / T(3);
  if (threadIdx.x < 64) {
    const int q = threadIdx.x;
    const int i = q % n, j = (q / n) % n, k = q / (n * n);
    int c = cur;
    for (int it = 0; it < sweeps; ++it) {
      const T* src = (c ? pb : pa) + o;
      T* dst = (c ? pa : pb) + o;
      if (q < N) dst[q] = (T(1) - w) * src[q] + (w / T(6)) * (nb6(src, n, i, j, k) - h2 * ff[o + q]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      c ^= 1;
    }
  }
  __syncthreads();
  cur ^= sweeps & 1;
}

// red-black sweeps of a tail level (n even): per colour, a thread per cell
// of the colour, the arithmetic of k_rbgs
template <typename T>
__device__ void tail_rbgs(T* pa, T* pb, const T* ff, int o, int n, T h2, int sweeps, int cur) {
  const int nh = n >> 1, Nh = nh * n * n;
  T* phi = (cur ? pb : pa) + o;
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      for (int p = threadIdx.x; p < Nh; p += MG_TAIL_THREADS) {
        const int r = p / nh, j = r % n, k = r / n;
        const int i = 2 * (p - r * nh) + ((j + k + colour) & 1);
        const int q = (k * n + j) * n + i;
        phi[q] = (nb6(phi, n, i, j, k) - h2 * ff[o + q]) / T(6);
      }
      __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(MG_TAIL_THREADS) void k_mgcycle_tail(TailArgs<T> t) {
  __shared__ T pa[MG_TAIL_ALLOC], pb[MG_TAIL_ALLOC], ff[MG_TAIL_ALLOC];
  __shared__ double sh[MG_TAIL_THREADS];
  int cur[MG_MAX_LEVELS];
  int todo[MG_MAX_LEVELS];  // coarse cycles of level m + 1 still to run for level m
  {
    const int N0 = t.n[0] * t.n[0] * t.n[0];
    for (int q = threadIdx.x; q < N0; q += MG_TAIL_THREADS) {
      ff[t.off[0] + q] = t.F0[q];
      pa[t.off[0] + q] = t.warm ? t.phi0[q] : T(0);
    }
    cur[0] = 0;
    __syncthreads();
  }
  auto smooth = [&](int m, int sweeps) {
    if (t.rbgs) tail_rbgs(pa, pb, ff, t.off[m], t.n[m], t.h2[m], sweeps, cur[m]);
    else tail_sweeps(pa, pb, ff, t.off[m], t.n[m], t.h2[m], sweeps, cur[m]);
  };
  int m = 0;
  bool down = true;
  for (;;) {
    if (down) {
      if (m == t.nl - 1) {
        // coarsest level: phi = 0, Jacobi sweeps, remove the mean (as
        // k_coarse_solve)
        const int n = t.n[m], N = n * n * n, o = t.off[m];
        for (int q = threadIdx.x; q < N; q += MG_TAIL_THREADS) pa[o + q] = T(0);
        cur[m] = 0;
        __syncthreads();
        if (N <= 64) tail_sweeps_wave(pa, pb, ff, o, n, t.h2[m], t.csweeps, cur[m]);
        else tail_sweeps(pa, pb, ff, o, n, t.h2[m], t.csweeps, cur[m]);
        T* phi = (cur[m] ? pb : pa) + o;
        double s = 0.0;
        for (int q = threadIdx.x; q < N; q += MG_TAIL_THREADS) s += (double)phi[q];
        const double mean = block_sum1024(s, sh) / (double)N;
        for (int q = threadIdx.x; q < N; q += MG_TAIL_THREADS) phi[q] = phi[q] - (T)mean;
        __syncthreads();
        down = false;
        continue;
      }
      const int n = t.n[m], o = t.off[m];
      smooth(m, t.pre);
      // restricted residual: F_{m+1} = average over the 8 children of F - A phi
      const T* phi = (cur[m] ? pb : pa) + o;
      const int nc = t.n[m + 1], Nc = nc * nc * nc, oc = t.off[m + 1];
      for (int Q = threadIdx.x; Q < Nc; Q += MG_TAIL_THREADS) {
        const int I = Q % nc, J = (Q / nc) % nc, K = Q / (nc * nc);
        T sum = T(0);
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
              const int q = (k * n + j) * n + i;
              sum += ff[o + q] - (nb6(phi, n, i, j, k) - T(6) * phi[q]) * t.ih2[m];
            }
        ff[oc + Q] = T(0.125) * sum;
      }
      __syncthreads();
      double s = 0.0;
      for (int Q = threadIdx.x; Q < Nc; Q += MG_TAIL_THREADS) s += (double)ff[oc + Q];
      const T mean = (T)(block_sum1024(s, sh) / (double)Nc);
      for (int Q = threadIdx.x; Q < Nc; Q += MG_TAIL_THREADS) {
        ff[oc + Q] = ff[oc + Q] - mean;
        pa[oc + Q] = T(0);  // the coarse error starts from zero
      }
      cur[m + 1] = 0;
      __syncthreads();
      todo[m] = (t.wcycle && m + 1 < t.nl - 1) ? 2 : 1;
      ++m;
    } else {
      if (m == 0) break;
      const int p = m - 1;
      if (--todo[p] > 0) {
        down = true;  // the next coarse cycle starts from the current result
        continue;
      }
      // cell-centred trilinear prolongation of the coarse correction, added
      const int nc = t.n[m], nf = t.n[p], Nf = nf * nf * nf;
      const T* ec = (cur[m] ? pb : pa) + t.off[m];
      T* phif = (cur[p] ? pb : pa) + t.off[p];
      for (int q = threadIdx.x; q < Nf; q += MG_TAIL_THREADS) {
        const int i = q % nf, j = (q / nf) % nf, k = q / (nf * nf);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int I2 = wrapi(I + ((i & 1) ? 1 : -1), nc);
        const int J2 = wrapi(J + ((j & 1) ? 1 : -1), nc);
        const int K2 = wrapi(K + ((k & 1) ? 1 : -1), nc);
        auto at = [&](int a, int b, int c) { return ec[(c * nc + b) * nc + a]; };
        const T w0 = T(0.75), w1 = T(0.25);
        T e = T(0);
        e += w0 * w0 * w0 * at(I, J, K);
        e += w1 * w0 * w0 * at(I2, J, K);
        e += w0 * w1 * w0 * at(I, J2, K);
        e += w1 * w1 * w0 * at(I2, J2, K);
        e += w0 * w0 * w1 * at(I, J, K2);
        e += w1 * w0 * w1 * at(I2, J, K2);
        e += w0 * w1 * w1 * at(I, J2, K2);
        e += w1 * w1 * w1 * at(I2, J2, K2);
        phif[q] += e;
      }
      __syncthreads();
      m = p;
      smooth(m, t.post);
    }
  }
  {
    const int N0 = t.n[0] * t.n[0] * t.n[0];
    const T* phi = (cur[0] ? pb : pa) + t.off[0];
    for (int q = threadIdx.x; q < N0; q += MG_TAIL_THREADS) t.phi0[q] = phi[q];
  }
}

// gravity kick g = -(phi_{i+1} - phi_{i-1}) / (2h) with m += rho g dt,
// E += (m_old . g) dt; then cooling; then the CFL max and the health check
template <typename T, bool COOL>
__global__ __launch_bounds__(256) void k_grav_sources(T* U, const T* __restrict__ phi, int n, T i2h,
                                                      T gamma, T ihx, CoolParams<T> cool, DevClock* clk,
                                                      int cfl) {
  __shared__ T sRed[4];
  const long long N = (long long)n * n * n;
  const T dt = (T)clk->dt;
  const T gm1 = gamma - T(1);
  T s = T(0);
  unsigned long long bad = 0, first_bad = ~0ull;
  // grid-stride over the cells, so that a capped grid issues few clock atomics
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < N;
       q += (long long)gridDim.x * 256) {
    const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((long long)n * n));
    const long long n2 = (long long)n * n;
    const long long row = (long long)k * n2 + (long long)j * n;
    const T gx = -(phi[row + wrapi(i + 1, n)] - phi[row + wrapi(i - 1, n)]) * i2h;
    const T gy = -(phi[(long long)k * n2 + (long long)wrapi(j + 1, n) * n + i] -
                   phi[(long long)k * n2 + (long long)wrapi(j - 1, n) * n + i]) * i2h;
    const T gz = -(phi[(long long)wrapi(k + 1, n) * n2 + (long long)j * n + i] -
                   phi[(long long)wrapi(k - 1, n) * n2 + (long long)j * n + i]) * i2h;
    T u[5];
    load_cell(U, N, q, u);
    const T dE = u[1] * gx + u[2] * gy + u[3] * gz;
    u[1] += u[0] * gx * dt;
    u[2] += u[0] * gy * dt;
    u[3] += u[0] * gz * dt;
    u[4] += dE * dt;
    if (COOL) {
      const T ek = T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
      const T Tin = gm1 * (u[4] - ek) / u[0];
      const T Tn = cool_T(u[0], Tin, dt, cool);
      u[4] = ek + u[0] * Tn / gm1;
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) U[f * N + q] = u[f];
    if (!cfl) continue;  // a later kernel reduces the CFL speed of the final state
    T w[5];
    to_prim(u, gm1, w);
    const T cs = dev_sqrt(gamma * w[4] * dev_rcp(w[0]));
    const T sq = (fmax(fmax(fabs(w[1]), fabs(w[2])), fabs(w[3])) + cs) * ihx;
    s = fmax(s, sq);
    const bool ok = (w[0] > T(0)) && (w[4] > T(0)) && isfinite(u[1]) && isfinite(u[2]) &&
                    isfinite(u[3]) && isfinite(u[4]) && isfinite(sq);
    if (!ok) {
      ++bad;
      if ((unsigned long long)q < first_bad) first_bad = (unsigned long long)q;
    }
  }
  if (!cfl) return;  // uniform: the whole block returns
  const T m = wave_max(s);
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(&clk->smax, pos_bits(fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]))));
  if (bad) {
    atomicAdd(&clk->bad_count, bad);
    atomicMin(&clk->bad_first, first_bad);
  }
}

__global__ void k_set_cycles(DevClock* clk, int cycles) {
  if (threadIdx.x == 0) clk->mg_cycles = cycles;
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }
// a launch over `planes` z-planes of `m` cells each: blockIdx.y is the plane
inline dim3 plane_grid(long long m, int planes) { return dim3(nblk(m), (unsigned)planes); }
// grid of a grid-stride kernel that ends in one clock atomic per block
inline unsigned nblk_capped(long long n) { return nblk(n) < 4096u ? nblk(n) : 4096u; }

// blocks of a two-stage reduction over n values (k_sum_partial's grid)
inline int sum_blocks(long long n) {
  const int nb = (int)((n + 255) / 256);
  return nb < MG_PARTIALS ? nb : MG_PARTIALS;
}

template <typename T>
hipError_t sum_to(const T* x, long long n, bool square, double* partial, double scale, double* out,
                  hipStream_t s) {
  const int nb = sum_blocks(n);
  if (square) hipLaunchKernelGGL((k_sum_partial<T, true>), dim3(nb), dim3(256), 0, s, x, n, partial);
  else hipLaunchKernelGGL((k_sum_partial<T, false>), dim3(nb), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, scale, out);
  return hipGetLastError();
}

template <typename T>
hipError_t remove_mean(T* x, long long n, double* partial, double* mean_slot, hipStream_t s) {
  hipError_t e = sum_to(x, n, false, partial, 1.0 / (double)n, mean_slot, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sub_mean<T>), dim3(nblk(n)), dim3(256), 0, s, x, n, mean_slot);
  return hipGetLastError();
}

template <typename T>
T* P(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

// smoothing sweeps on host-launched level l: weighted Jacobi (ping-pong,
// flips cur) or red-black Gauss-Seidel (in place)
template <typename T>
void smooth_level(char* ws, MGLevel& lv, int sweeps, int rbgs, int& cur, hipStream_t s) {
  const long long N = (long long)lv.n * lv.n * lv.n;
  const T h2 = (T)(lv.h * lv.h);
  for (int it = 0; it < sweeps; ++it) {
    if (rbgs) {
      for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL((k_rbgs<T>), plane_grid((long long)(lv.n / 2) * lv.n, lv.n),
                           dim3(256), 0, s, lv.n, h2,
                           P<T>(ws, lv.phi[cur]), P<T>(ws, lv.F), colour);
    } else {
      hipLaunchKernelGGL((k_jacobi<T>), plane_grid((long long)lv.n * lv.n, lv.n), dim3(256), 0,
                         s, lv.n, h2,
                         P<T>(ws, lv.phi[cur]), P<T>(ws, lv.F), P<T>(ws, lv.phi[1 - cur]));
      cur = 1 - cur;
    }
  }
}

// first level handled by the single-workgroup tail: the first one after the
// fine level with at most MG_TAIL_MAX_CELLS cells that is not the coarsest
// (nlev when there is none)
inline int tail_level(const MGLayout& L) {
  for (int l = 1; l < L.nlev - 1; ++l) {
    const long long Nl = (long long)L.lev[l].n * L.lev[l].n * L.lev[l].n;
    if (Nl <= MG_TAIL_MAX_CELLS) return l;
  }
  return L.nlev;
}

// one cycle on level l < l0 from its current phi (lev[l].phi[cur[l]]): pre
// smoothing, restriction of the residual, the coarse error equation solved by
// one (V) or two (W) cycles of level l + 1 from zero -- one solve when level
// l + 1 is the coarsest -- prolongation and correction, post smoothing
template <typename T>
hipError_t level_cycle(char* ws, MGLayout& L, const mh_physics_desc& p, int l, int l0,
                       int* cur, double* partial, double* mean_slot, hipStream_t s) {
  const int nl = L.nlev;
  const int rbgs = p.mg_smoother == MH_SMOOTH_RBGS;
  MGLevel& lv = L.lev[l];
  const long long N = (long long)lv.n * lv.n * lv.n;
  smooth_level<T>(ws, lv, p.mg_pre, rbgs, cur[l], s);
  MGLevel& cv = L.lev[l + 1];
  const long long Nc = (long long)cv.n * cv.n * cv.n;
  // F_c and its block sums in one pass, then its mean removed
  const int nbc = sum_blocks(Nc);
  hipLaunchKernelGGL((k_residual_restrict<T>), dim3(nbc), dim3(256), 0, s, cv.n,
                     (T)(1.0 / (lv.h * lv.h)), P<T>(ws, lv.phi[cur[l]]), P<T>(ws, lv.F),
                     P<T>(ws, cv.F), partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nbc, 1.0 / (double)Nc,
                     mean_slot);
  hipLaunchKernelGGL((k_sub_mean<T>), dim3(nblk(Nc)), dim3(256), 0, s, P<T>(ws, cv.F), Nc,
                     mean_slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int mu = (p.mg_cycle == MH_MG_W && l + 1 < nl - 1) ? 2 : 1;
  if (l + 1 == l0) {
    TailArgs<T> t{};
    t.nl = nl - l0;
    int off = 0;
    for (int m = 0; m < t.nl; ++m) {
      const MGLevel& tv = L.lev[l0 + m];
      t.n[m] = tv.n;
      t.h2[m] = (T)(tv.h * tv.h);
      t.ih2[m] = (T)(1.0 / (tv.h * tv.h));
      t.off[m] = off;
      off += tv.n * tv.n * tv.n;
    }
    if (off > MG_TAIL_ALLOC) return hipErrorInvalidValue;
    t.F0 = P<T>(ws, cv.F);
    t.phi0 = P<T>(ws, cv.phi[0]);
    t.pre = p.mg_pre;
    t.post = p.mg_post;
    t.csweeps = p.mg_coarse_sweeps;
    t.wcycle = p.mg_cycle == MH_MG_W;
    t.rbgs = rbgs;
    cur[l + 1] = 0;
    for (int k = 0; k < mu; ++k) {
      t.warm = k > 0;
      hipLaunchKernelGGL((k_mgcycle_tail<T>), dim3(1), dim3(MG_TAIL_THREADS), 0, s, t);
    }
  } else if (l + 1 == nl - 1) {
    cur[l + 1] = 0;
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(256), 0, s, cv.n, (T)(cv.h * cv.h),
                       P<T>(ws, cv.F), P<T>(ws, cv.phi[0]), p.mg_coarse_sweeps);
  } else {
    cur[l + 1] = 0;
    hipLaunchKernelGGL((k_zero<T>), dim3(nblk(Nc)), dim3(256), 0, s, P<T>(ws, cv.phi[0]), Nc);
    for (int k = 0; k < mu; ++k) {
      e = level_cycle<T>(ws, L, p, l + 1, l0, cur, partial, mean_slot, s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL((k_prolong_add<T>), plane_grid((long long)lv.n * lv.n, lv.n), dim3(256),
                     0, s, cv.n,
                     P<T>(ws, cv.phi[cur[l + 1]]), P<T>(ws, lv.phi[cur[l]]));
  smooth_level<T>(ws, lv, p.mg_post, rbgs, cur[l], s);
  return hipGetLastError();
}

// one cycle (V or W) on level 0; phi of level 0 is lev[0].phi[L.cur0]
template <typename T>
hipError_t vcycle(char* ws, MGLayout& L, const mh_physics_desc& p, double* partial,
                  double* mean_slot, hipStream_t s) {
  const int nl = L.nlev;
  int cur[MG_MAX_LEVELS];
  cur[0] = L.cur0;
  if (nl == 1) {
    // the whole grid is the coarsest grid: plain Jacobi sweeps from the warm
    // start
    MGLevel& cv = L.lev[0];
    const long long N = (long long)cv.n * cv.n * cv.n;
    for (int it = 0; it < p.mg_coarse_sweeps; ++it) {
      hipLaunchKernelGGL((k_jacobi<T>), plane_grid((long long)cv.n * cv.n, cv.n), dim3(256), 0,
                         s, cv.n, (T)(cv.h * cv.h),
                         P<T>(ws, cv.phi[cur[0]]), P<T>(ws, cv.F), P<T>(ws, cv.phi[1 - cur[0]]));
      cur[0] = 1 - cur[0];
    }
    hipError_t e = remove_mean(P<T>(ws, cv.phi[cur[0]]), N, partial, mean_slot, s);
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = level_cycle<T>(ws, L, p, 0, tail_level(L), cur, partial, mean_slot, s);
    if (e != hipSuccess) return e;
  }
  L.cur0 = cur[0];
  return hipGetLastError();
}

}  // namespace

mh_status mg_validate(const mh_grid_desc* g, const mh_physics_desc* p, std::string& err) {
  for (int a = 0; a < 3; ++a)
    if (g->bc[a] != MH_BC_PERIODIC) {
      err = "gravity needs periodic boundaries on every axis";
      return MH_E_SHAPE;
    }
  if (g->n[0] != g->n[1] || g->n[0] != g->n[2] || g->h[0] != g->h[1] || g->h[0] != g->h[2]) {
    err = "gravity needs a cubic grid with equal spacing";
    return MH_E_SHAPE;
  }
  if (!(p->grav_G >= 0.0) || p->mg_pre < 0 || p->mg_post < 0 || p->mg_max_cycles < 0 ||
      p->mg_coarsest < 1 || !(p->mg_tol >= 0.0) || p->mg_coarse_sweeps < 0) {
    err = "bad multigrid parameters";
    return MH_E_INVALID;
  }
  if (p->mg_cycle != MH_MG_V && p->mg_cycle != MH_MG_W) {
    err = "unknown multigrid cycle";
    return MH_E_UNSUPPORTED;
  }
  if (p->mg_smoother != MH_SMOOTH_JACOBI && p->mg_smoother != MH_SMOOTH_RBGS) {
    err = "unknown multigrid smoother";
    return MH_E_UNSUPPORTED;
  }
  if (p->grav_solver == MH_GRAV_FFT) {
    if (!fft_size_ok(g->n[0])) {
      err = "the spectral gravity solver needs a power-of-two n <= 1024";
      return MH_E_SHAPE;
    }
    return MH_OK;
  }
  if (p->grav_solver != MH_GRAV_MG) {
    err = "unknown gravity solver";
    return MH_E_UNSUPPORTED;
  }
  int n = g->n[0], levels = 1;
  while (!(n <= p->mg_coarsest || (n % 2) != 0)) {
    n /= 2;
    ++levels;
  }
  if ((long long)n * n * n > MG_COARSE_MAX_CELLS && levels > 1) {
    err = "coarsest multigrid grid exceeds 2048 cells";
    return MH_E_SHAPE;
  }
  if (levels > MG_MAX_LEVELS) {
    err = "too many multigrid levels";
    return MH_E_SHAPE;
  }
  return MH_OK;
}

size_t mg_layout(const mh_grid_desc* g, const mh_physics_desc* p, size_t off, size_t es,
                 MGLayout& L) {
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  // levels halve n while n > coarsest and n is even (the rule of mg_validate)
  L = MGLayout();
  L.partial = take(MG_PARTIALS * sizeof(double));
  int n = g->n[0];
  double h = g->h[0];
  if (p->grav_solver == MH_GRAV_FFT) {
    MGLevel& lv = L.lev[L.nlev++];
    const size_t bytes = (size_t)n * n * n * es;
    lv.n = n;
    lv.h = h;
    lv.phi[0] = take(bytes);
    lv.phi[1] = take(bytes);
    lv.F = take(bytes);
    return fft_layout(n, off, es, L);
  }
  for (;;) {
    MGLevel& lv = L.lev[L.nlev++];
    const size_t bytes = (size_t)n * n * n * es;
    lv.n = n;
    lv.h = h;
    lv.phi[0] = take(bytes);
    lv.phi[1] = take(bytes);
    lv.F = take(bytes);
    if (n <= p->mg_coarsest || (n % 2) != 0 || L.nlev == MG_MAX_LEVELS) break;
    n /= 2;
    h *= 2.0;
  }
  return off;
}

hipError_t mg_init(char* ws, const MGLayout& L, const mh_grid_desc* g, hipStream_t s) {
  const bool f64 = g->dtype == MH_F64;
  for (int l = 0; l < L.nlev; ++l) {
    const MGLevel& lv = L.lev[l];
    const long long N = (long long)lv.n * lv.n * lv.n;
    const size_t offs[3] = {lv.phi[0], lv.phi[1], lv.F};
    for (size_t o : offs) {
      if (f64) hipLaunchKernelGGL((k_zero<double>), dim3(nblk(N)), dim3(256), 0, s, P<double>(ws, o), N);
      else hipLaunchKernelGGL((k_zero<float>), dim3(nblk(N)), dim3(256), 0, s, P<float>(ws, o), N);
    }
  }
  return hipGetLastError();
}

#define MG_CHECK(x)                \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// F = scale (x - <x>) on the fine level
template <typename T>
hipError_t mg_set_rhs(char* ws, MGLayout& L, const T* x, double scale, DevClock* clk,
                      hipStream_t s) {
  MGLevel& f = L.lev[0];
  const long long N = (long long)f.n * f.n * f.n;
  double* partial = P<double>(ws, L.partial);
  MG_CHECK(sum_to(x, N, false, partial, 1.0 / (double)N, &clk->mean, s));
  hipLaunchKernelGGL((k_shift_scale<T>), dim3(nblk(N)), dim3(256), 0, s, P<T>(ws, f.F), x, N,
                     &clk->mean, scale);
  return hipGetLastError();
}

// fine-level initial guess: a copy of phi0, or zero
template <typename T>
hipError_t mg_set_guess(char* ws, MGLayout& L, const T* phi0, hipStream_t s) {
  MGLevel& f = L.lev[0];
  const long long N = (long long)f.n * f.n * f.n;
  if (phi0)
    return hipMemcpyAsync(P<T>(ws, f.phi[L.cur0]), phi0, N * sizeof(T), hipMemcpyDeviceToDevice, s);
  hipLaunchKernelGGL((k_zero<T>), dim3(nblk(N)), dim3(256), 0, s, P<T>(ws, f.phi[L.cur0]), N);
  return hipGetLastError();
}

// V-cycles on A phi = F (F already mean-free on the fine level) from the
// current guess until ||F - A phi||_2 <= tol ||F||_2 or max_cycles cycles;
// the mean of phi is removed before the first and after every cycle.
void MGGraphCache::reset() {
  for (int k = 0; k < 2; ++k) {
    if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
    exec[k] = nullptr;
  }
  ws = nullptr;
}

void MGGraphCache::destroy() {
  reset();
  if (cs) (void)hipStreamDestroy(cs);
  cs = nullptr;
}

// one V-cycle: replayed from the cached graph of the current parity (captured
// on first use), or launched kernel by kernel when no cache is attached
template <typename T>
hipError_t run_vcycle(char* ws, MGLayout& L, const mh_physics_desc& p, double* partial,
                      double* mean_slot, hipStream_t s) {
  MGGraphCache* G = L.graphs;
  if (!G || !G->enabled) return vcycle<T>(ws, L, p, partial, mean_slot, s);
  if (G->ws != ws) {
    G->reset();
    G->ws = ws;
  }
  const int k = L.cur0;
  if (!G->exec[k]) {
    if (!G->cs) MG_CHECK(hipStreamCreateWithFlags(&G->cs, hipStreamNonBlocking));
    MG_CHECK(hipStreamBeginCapture(G->cs, hipStreamCaptureModeRelaxed));
    const hipError_t e = vcycle<T>(ws, L, p, partial, mean_slot, G->cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(G->cs, &graph);
    G->cur_after[k] = L.cur0;
    L.cur0 = k;  // nothing ran during the capture
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    MG_CHECK(e2);
    const hipError_t e3 = hipGraphInstantiate(&G->exec[k], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    MG_CHECK(e3);
  }
  MG_CHECK(hipGraphLaunch(G->exec[k], s));
  L.cur0 = G->cur_after[k];
  return hipSuccess;
}

template <typename T>
hipError_t mg_solve(char* ws, MGLayout& L, const mh_physics_desc& p, DevClock* clk, int* cycles_out,
                    hipStream_t s) {
  MGLevel& f = L.lev[0];
  const int n = f.n;
  const long long N = (long long)n * n * n;
  double* partial = P<double>(ws, L.partial);
  if (L.fft) {
    // the spectral solve: exact for the spectral operator, no cycles
    MG_CHECK(fft_poisson<T>(ws, L, f.h, s));
    hipLaunchKernelGGL(k_set_cycles, dim3(1), dim3(64), 0, s, clk, 0);
    if (cycles_out) *cycles_out = 0;
    return hipGetLastError();
  }
  MG_CHECK(sum_to(P<T>(ws, f.F), N, true, partial, 1.0, &clk->mg_fnorm2, s));
  MG_CHECK(remove_mean(P<T>(ws, f.phi[L.cur0]), N, partial, &clk->mean, s));
  int cycles = 0;
  double prev = INFINITY;
  for (;;) {
    // |r|^2 without storing r: the sum k_sum_partial would form over it
    const int nbr = sum_blocks(N);
    hipLaunchKernelGGL((k_residual_norm2<T>), dim3(nbr), dim3(256), 0, s, n,
                       (T)(1.0 / (f.h * f.h)), P<T>(ws, f.phi[L.cur0]), P<T>(ws, f.F), partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nbr, 1.0,
                       &clk->mg_rnorm2);
    double norms[2];
    MG_CHECK(hipMemcpyAsync(norms, &clk->mg_fnorm2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    MG_CHECK(hipStreamSynchronize(s));
    const double rn = std::sqrt(norms[1]);
    if (rn <= p.mg_tol * std::sqrt(norms[0]) || cycles >= p.mg_max_cycles) break;
    // with a tolerance, a cycle that no longer cuts the residual by MG_STALL
    // has reached the round-off floor of the precision (in fp32 it lies above
    // the usual tolerances): stop there rather than run to the cycle cap
    if (p.mg_tol > 0.0 && rn > MG_STALL * prev) break;
    prev = rn;
    MG_CHECK(run_vcycle<T>(ws, L, p, partial, &clk->mean, s));
    MG_CHECK(remove_mean(P<T>(ws, f.phi[L.cur0]), N, partial, &clk->mean, s));
    ++cycles;
  }
  hipLaunchKernelGGL(k_set_cycles, dim3(1), dim3(64), 0, s, clk, cycles);
  if (cycles_out) *cycles_out = cycles;
  return hipGetLastError();
}

template <typename T>
hipError_t mg_gravity_step(char* ws, MGLayout& L, const mh_grid_desc& g, const mh_physics_desc& p,
                           const CoolParams<T>& cp, T* U, DevClock* clk, bool last, hipStream_t s) {
  MGLevel& f = L.lev[0];
  const int n = f.n;
  const long long N = (long long)n * n * n;
  // F = 4 pi G (rho - <rho>), solve from the previous potential
  MG_CHECK(mg_set_rhs<T>(ws, L, U, 4.0 * M_PI * p.grav_G, clk, s));
  MG_CHECK(mg_solve<T>(ws, L, p, clk, nullptr, s));
  // the exact two-branch cooling is fused here when this kernel ends the step
  const bool cool = last && (p.flags & MH_SRC_COOLING) && p.cool_model == MH_COOL_EXACT2;
  if (L.fft) return fft_sources<T>(ws, L, g, cool, last, cp, U, clk, s);
  const T i2h = (T)(1.0 / (2.0 * f.h));
  if (cool)
    hipLaunchKernelGGL((k_grav_sources<T, true>), dim3(nblk_capped(N)), dim3(256), 0, s, U,
                       P<T>(ws, f.phi[L.cur0]), n, i2h, (T)g.gamma, (T)(1.0 / f.h), cp, clk,
                       (int)last);
  else
    hipLaunchKernelGGL((k_grav_sources<T, false>), dim3(nblk_capped(N)), dim3(256), 0, s, U,
                       P<T>(ws, f.phi[L.cur0]), n, i2h, (T)g.gamma, (T)(1.0 / f.h), cp, clk,
                       (int)last);
  return hipGetLastError();
}

// gravity kick alone from the fine-level potential (no cooling), for the
// forward recomputation inside the adjoint step
template <typename T>
hipError_t mg_kick(char* ws, MGLayout& L, const mh_grid_desc& g, T* U, DevClock* clk,
                   hipStream_t s) {
  MGLevel& f = L.lev[0];
  const long long N = (long long)f.n * f.n * f.n;
  CoolParams<T> none{};
  if (L.fft) return fft_sources<T>(ws, L, g, false, true, none, U, clk, s);
  hipLaunchKernelGGL((k_grav_sources<T, false>), dim3(nblk_capped(N)), dim3(256), 0, s, U,
                     P<T>(ws, f.phi[L.cur0]), f.n, (T)(1.0 / (2.0 * f.h)), (T)g.gamma,
                     (T)(1.0 / f.h), none, clk, 1);
  return hipGetLastError();
}

#undef MG_CHECK

#define MG_INSTANTIATE(T)                                                                      \
  template hipError_t mg_gravity_step<T>(char*, MGLayout&, const mh_grid_desc&,                \
                                         const mh_physics_desc&, const CoolParams<T>&, T*,     \
                                         DevClock*, bool, hipStream_t);                         \
  template hipError_t mg_set_rhs<T>(char*, MGLayout&, const T*, double, DevClock*, hipStream_t); \
  template hipError_t mg_set_guess<T>(char*, MGLayout&, const T*, hipStream_t);                 \
  template hipError_t mg_solve<T>(char*, MGLayout&, const mh_physics_desc&, DevClock*, int*,    \
                                  hipStream_t);                                                 \
  template hipError_t mg_kick<T>(char*, MGLayout&, const mh_grid_desc&, T*, DevClock*, hipStream_t);
MG_INSTANTIATE(float)
MG_INSTANTIATE(double)
#undef MG_INSTANTIATE

size_t mg_phi_offset(const MGLayout& L) { return L.lev[0].phi[L.cur0]; }

}  // namespace mh
