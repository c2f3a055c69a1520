// fft_kernels.hip -- spectral self-gravity on the device (arXiv 2512.13403,
// Sec. 6.1): the Poisson equation lap(Phi) = 4 pi G (rho - <rho>) solved in
// Fourier space, Phi_hat = -F_hat / |kappa|^2 (zero mode 0), the acceleration
// a = -grad Phi by multiplying with -i kappa, and the adjoint of rho -> a for
// the reverse pass (the potential adjoint sum_a i kappa_a g_hat_a scaled by
// -4 pi G / kappa^2).
//
// Transforms are complex-to-complex over the whole n^3 cube (n a power of
// two), one axis at a time.  A workgroup loads `lpb` whole lines along the
// axis into LDS -- for the y and z axes lines of consecutive x, so
// every load and store touches lpb consecutive elements -- and transforms
// them with the self-sorting (Stockham) formulation: radix-8 passes and one
// radix-2 or radix-4 pass for the rest of log2(n), each an in-register DFT
// of the values a thread reads, so a 512-point line takes three passes
// through LDS and no bit-reversal.  Twiddles exp(-2 pi i t / n), t < n/2,
// come from fp64 sincospi (a table read through the caches).  The inverse
// transform is conj(FFT(conj x)), unscaled; the 1/n^3 is folded into the
// spectral multipliers.
//
// Wavenumbers on a box of length L = n h: kappa = 2 pi m / L with m = q for
// index q <= n/2, q - n above.  The derivative uses kappa with the Nyquist
// index q = n/2 set to 0 (its i kappa factor has no real counterpart), while
// |kappa|^2 keeps it.
#include <cmath>
#include <mutex>

#include "mg.h"
#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

namespace {

template <typename T>
struct CplxOf;
template <>
struct CplxOf<float> {
  using type = float2;
};
template <>
struct CplxOf<double> {
  using type = double2;
};

constexpr int FFT_THREADS = 256;
// values per thread: 128 bytes (16 in fp32, 8 in fp64), so a workgroup holds
// 32 KB of whole lines in LDS
template <typename C>
constexpr int fft_elems() {
  return 128 / (int)sizeof(C);
}
static_assert(fft_elems<double2>() >= 8, "a radix-8 pass needs 8 values per thread");

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }
// grid of a grid-stride kernel that ends in one clock atomic per block
inline unsigned nblk_capped(long long n) { return nblk(n) < 4096u ? nblk(n) : 4096u; }

template <typename T>
T* P(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_twiddles(typename CplxOf<T>::type* tw, int n) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n / 2) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)n, &s, &c);
  tw[t].x = (T)c;
  tw[t].y = (T)s;
}

// element index of point j of line `line` along AXIS of the n^3 cube (n =
// 2^logn <= 1024, so every index fits 32 bits); lines are numbered with x
// fastest among the two other coordinates
template <int AXIS>
__device__ __forceinline__ unsigned line_elem(int logn, unsigned line, unsigned j) {
  if (AXIS == 0) return (line << logn) + j;
  if (AXIS == 1)
    return ((line >> logn) << (2 * logn)) + (j << logn) + (line & ((1u << logn) - 1u));
  return (j << (2 * logn)) + line;  // line = y n + x
}

// v exp(-2 pi i j / ln) for the roots of an in-register DFT (ln <= 8)
template <typename C>
__device__ __forceinline__ C mul_root(C v, int j, int ln) {
  using T = decltype(v.x);
  const T s = T(0.70710678118654752440);
  if (j == 0) return v;
  if (4 * j == ln) return C{v.y, -v.x};
  if (8 * j == ln) return C{(v.x + v.y) * s, (v.y - v.x) * s};
  return C{(v.y - v.x) * s, -(v.x + v.y) * s};  // 8 j == 3 ln
}

// R-point DFT (R = 2, 4, 8) of u in registers: radix-2 decimation in time on
// the bit-reversed values
template <typename C, int R>
__device__ __forceinline__ void dft_regs(C (&u)[R]) {
  constexpr int LB = R == 2 ? 1 : (R == 4 ? 2 : 3);
  C v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    int b = 0;
#pragma unroll
    for (int q = 0; q < LB; ++q) b |= ((i >> q) & 1) << (LB - 1 - q);
    v[b] = u[i];
  }
#pragma unroll
  for (int ln = 2; ln <= R; ln <<= 1)
#pragma unroll
    for (int i = 0; i < R; i += ln)
#pragma unroll
      for (int j = 0; j < ln / 2; ++j) {
        const C t = mul_root(v[i + j + ln / 2], j, ln);
        const C a = v[i + j];
        v[i + j] = C{a.x + t.x, a.y + t.y};
        v[i + j + ln / 2] = C{a.x - t.x, a.y - t.y};
      }
#pragma unroll
  for (int i = 0; i < R; ++i) u[i] = v[i];
}

// One radix-R pass of the self-sorting (Stockham) FFT over the E = lpb n
// values of the workgroup's lines in LDS, after passes whose radices multiply
// to p: group i (< n / R) of a line reads x[i + r n / R], multiplies by
// exp(-2 pi i r k / (R p)) with k = i mod p, transforms them, and writes
// x'[(i - k) R + k + r p].  All groups are read before any is written (one
// barrier), so the pass works in place; E / FFT_THREADS <= ELEMS, so every
// thread holds its values in registers.
template <typename C, int R, int ELEMS>
__device__ __forceinline__ void stockham_pass(C* buf, const C* __restrict__ stw, int logn, int E,
                                              int p) {
  constexpr int GMAX = ELEMS / R;
  constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : 3);
  const int n = 1 << logn, logm = logn - LR, m = n >> LR, groups = E >> LR;
  C u[GMAX][R];
#pragma unroll
  for (int gi = 0; gi < GMAX; ++gi) {
    const int g = threadIdx.x + gi * FFT_THREADS;
    if (g < groups) {
      const int li = g >> logm, i = g & (m - 1), k = i & (p - 1);
      const C* x = buf + (li << logn);
      const int step = n / (R * p);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C v = x[i + r * m];
        if (r > 0) {
          const int t = r * k * step;  // < n: table of the first half, negated above it
          C w = stw[t < n / 2 ? t : t - n / 2];
          if (t >= n / 2) w = C{-w.x, -w.y};
          v = C{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
        }
        u[gi][r] = v;
      }
      dft_regs<C, R>(u[gi]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int gi = 0; gi < GMAX; ++gi) {
    const int g = threadIdx.x + gi * FFT_THREADS;
    if (g < groups) {
      const int li = g >> logm, i = g & (m - 1), k = i & (p - 1);
      C* x = buf + (li << logn);
      const int j = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[j + r * p] = u[gi][r];
    }
  }
  __syncthreads();
}

// FFT of 2^loglpb lines per workgroup (unscaled); the inverse is
// conj(FFT(conj)).  Every thread first issues all of its (at most ELEMS)
// loads, then writes them to LDS, so that each wave has its whole share of
// the lines in flight at once; the store to the cube is batched the same way.
// IO selects the ends of a 3D transform: 0 in place on `data`; FFT_REAL_IN
// reads the real field `rin` (imaginary part 0) and writes `data`;
// FFT_REAL_OUT reads `data` and writes only the real part, to `rout`;
// FFT_SPLIT_OUT writes the real part to `rout` and the imaginary part to
// `rout2` (the inverse transform of two Hermitian spectra packed as A + i B
// gives the two real fields a + i b); FFT_PAIR_IN reads `rin` + i `rin2` (the
// transform of two real fields at once, separated by Hermitian symmetry).
enum : int { FFT_COMPLEX = 0, FFT_REAL_IN = 1, FFT_REAL_OUT = 2, FFT_SPLIT_OUT = 3,
             FFT_PAIR_IN = 4 };
template <typename T, int AXIS, int IO>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_lines(typename CplxOf<T>::type* data,
                                                           const T* __restrict__ rin,
                                                           const T* __restrict__ rin2,
                                                           T* __restrict__ rout,
                                                           T* __restrict__ rout2,
                                                           const typename CplxOf<T>::type* tw,
                                                           int logn, int loglpb, int inverse) {
  using C = typename CplxOf<T>::type;
  constexpr int ELEMS = fft_elems<C>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  // workgroups are dealt round-robin over the 8 XCDs: give each XCD a
  // contiguous range of line blocks, so that the y and z passes' neighbouring
  // blocks (the next lpb values of x) share that XCD's L2 lines
  unsigned b = blockIdx.x;
  if ((gridDim.x & 7u) == 0) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
  const unsigned line0 = b << loglpb;
  const int E = 1 << (logn + loglpb);  // <= ELEMS * FFT_THREADS (the launch sizes lpb so)
  // x axis: consecutive threads walk along a line; y, z: across lines
  auto line_of = [&](int e) { return AXIS == 0 ? e >> logn : e & ((1 << loglpb) - 1); };
  auto point_of = [&](int e) { return AXIS == 0 ? e & ((1 << logn) - 1) : e >> loglpb; };
  C v[ELEMS];
#pragma unroll
  for (int q = 0; q < ELEMS; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < E) {
      const unsigned idx = line_elem<AXIS>(logn, line0 + line_of(e), point_of(e));
      if (IO == FFT_REAL_IN) v[q] = C{rin[idx], T(0)};
      else if (IO == FFT_PAIR_IN) v[q] = C{rin[idx], rin2[idx]};
      else v[q] = data[idx];
    }
  }
#pragma unroll
  for (int q = 0; q < ELEMS; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < E) {
      C x = v[q];
      if (inverse) x.y = -x.y;
      buf[(line_of(e) << logn) + point_of(e)] = x;
    }
  }
  __syncthreads();
  int p = 1;
  for (int q = 0; q < logn / 3; ++q) {
    stockham_pass<C, 8, ELEMS>(buf, tw, logn, E, p);
    p *= 8;
  }
  if (logn % 3 == 1) stockham_pass<C, 2, ELEMS>(buf, tw, logn, E, p);
  else if (logn % 3 == 2) stockham_pass<C, 4, ELEMS>(buf, tw, logn, E, p);
#pragma unroll
  for (int q = 0; q < ELEMS; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < E) v[q] = buf[(line_of(e) << logn) + point_of(e)];
  }
#pragma unroll
  for (int q = 0; q < ELEMS; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < E) {
      C x = v[q];
      if (inverse) x.y = -x.y;
      const unsigned idx = line_elem<AXIS>(logn, line0 + line_of(e), point_of(e));
      if (IO == FFT_REAL_OUT) {
        rout[idx] = x.x;
      } else if (IO == FFT_SPLIT_OUT) {
        rout[idx] = x.x;
        rout2[idx] = x.y;
      } else {
        data[idx] = x;
      }
    }
  }
}

__device__ __forceinline__ int wavenum(int q, int n) { return q <= n / 2 ? q : q - n; }

// Phi_hat / N = -F_hat / (|kappa|^2 N), 0 at kappa = 0
template <typename T>
__global__ __launch_bounds__(256) void k_fft_phi(typename CplxOf<T>::type* c, int n, double tk) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int kx = wavenum((int)(q % n), n), ky = wavenum((int)((q / n) % n), n),
            kz = wavenum((int)(q / ((long long)n * n)), n);
  const double k2 = tk * tk * (double)(kx * kx + ky * ky + kz * kz);
  const T f = k2 > 0.0 ? (T)(-1.0 / (k2 * (double)N)) : T(0);
  c[q].x *= f;
  c[q].y *= f;
}

// derivative wavenumber of index q along an axis (Nyquist -> 0)
__device__ __forceinline__ double dkappa(int q, int n, double tk) {
  return q == n / 2 ? 0.0 : tk * (double)wavenum(q, n);
}

template <int AXIS>
__device__ __forceinline__ int axis_index(long long q, int n) {
  return AXIS == 0 ? (int)(q % n) : (AXIS == 1 ? (int)((q / n) % n) : (int)(q / ((long long)n * n)));
}

// the four real fields of the solve packed two per complex spectrum: with
// Phi_hat in c (already divided by N) and a_hat_a = -i kappa~_a Phi_hat,
// c1 = a_hat_x + i a_hat_y and c (in place) = a_hat_z + i Phi_hat; each of
// the four spectra is Hermitian (the Nyquist index has kappa~ = 0), so the
// inverse transforms give a_x + i a_y and a_z + i Phi
template <typename T>
__global__ __launch_bounds__(256) void k_fft_grad_pairs(typename CplxOf<T>::type* c,
                                                        typename CplxOf<T>::type* c1, int n,
                                                        double tk) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const T kx = (T)dkappa(axis_index<0>(q, n), n, tk), ky = (T)dkappa(axis_index<1>(q, n), n, tk),
          kz = (T)dkappa(axis_index<2>(q, n), n, tk);
  const T re = c[q].x, im = c[q].y;
  // -i k (re + i im) = (k im, -k re); i (u + i w) = (-w, u)
  c1[q].x = kx * im + ky * re;
  c1[q].y = -kx * re + ky * im;
  c[q].x = kz * im - im;
  c[q].y = -kz * re + re;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_real_add(const typename CplxOf<T>::type* __restrict__ c,
                                                      T* out, long long N) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q < N) out[q] += c[q].x;
}

// adjoint accumulation: acc (+)= conj(m_a) g_hat / N with m_a = 4 pi G i
// kappa~_a / |kappa|^2, i.e. conj(m_a) g = -4 pi G kappa~_a / k2 (-g.y, g.x)
template <typename T, int AXIS>
__global__ __launch_bounds__(256) void k_fft_adj_accum(const typename CplxOf<T>::type* __restrict__ g,
                                                       typename CplxOf<T>::type* acc, int n,
                                                       double tk, double fourpiG, int first) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int kx = wavenum((int)(q % n), n), ky = wavenum((int)((q / n) % n), n),
            kz = wavenum((int)(q / ((long long)n * n)), n);
  const double k2 = tk * tk * (double)(kx * kx + ky * ky + kz * kz);
  const T f = k2 > 0.0 ? (T)(-fourpiG * dkappa(axis_index<AXIS>(q, n), n, tk) / (k2 * (double)N))
                       : T(0);
  const T re = -f * g[q].y, im = f * g[q].x;
  if (first) {
    acc[q].x = re;
    acc[q].y = im;
  } else {
    acc[q].x += re;
    acc[q].y += im;
  }
}

// the same for the x and y components from Z = FFT(g_x + i g_y): G_x(k) =
// (Z(k) + conj Z(-k)) / 2 and G_y(k) = (Z(k) - conj Z(-k)) / 2i (the two
// spectra of real fields), acc = conj(m_x) G_x + conj(m_y) G_y
template <typename T>
__global__ __launch_bounds__(256) void k_fft_adj_accum_pair(
    const typename CplxOf<T>::type* __restrict__ z, typename CplxOf<T>::type* acc, int n,
    double tk, double fourpiG) {
  const long long N = (long long)n * n * n;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int ix = (int)(q % n), iy = (int)((q / n) % n), iz = (int)(q / ((long long)n * n));
  const long long r = ((long long)((n - iz) % n) * n + (n - iy) % n) * n + (n - ix) % n;
  const T zr = z[q].x, zi = z[q].y, wr = z[r].x, wi = z[r].y;
  const T gxr = T(0.5) * (zr + wr), gxi = T(0.5) * (zi - wi);  // (Z + conj W) / 2
  const T gyr = T(0.5) * (zi + wi), gyi = T(-0.5) * (zr - wr);  // (Z - conj W) / 2i
  const int kx = wavenum(ix, n), ky = wavenum(iy, n), kz = wavenum(iz, n);
  const double k2 = tk * tk * (double)(kx * kx + ky * ky + kz * kz);
  const double s = k2 > 0.0 ? -fourpiG / (k2 * (double)N) : 0.0;
  const T fx = (T)(s * dkappa(ix, n, tk)), fy = (T)(s * dkappa(iy, n, tk));
  acc[q].x = -fx * gxi - fy * gyi;
  acc[q].y = fx * gxr + fy * gyr;
}

// gravity kick with a given acceleration field, m += rho a dt, E += (m_old .
// a) dt; then cooling; then the CFL max and the health check (the same
// epilogue as the multigrid path's sources kernel)
template <typename T, bool COOL>
__global__ __launch_bounds__(256) void k_accel_sources(T* U, const T* __restrict__ acc,
                                                       long long N, T gamma, T ihx,
                                                       CoolParams<T> cool, DevClock* clk,
                                                       int cfl) {
  __shared__ T sRed[4];
  const T dt = (T)clk->dt;
  const T gm1 = gamma - T(1);
  T s = T(0);
  unsigned long long bad = 0, first_bad = ~0ull;
  // grid-stride over the cells, so that a capped grid issues few clock atomics
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < N;
       q += (long long)gridDim.x * 256) {
    const T gx = acc[q], gy = acc[N + q], gz = acc[2 * N + q];
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

// reverse of the kick at fixed acceleration: lout from lin, and the
// acceleration adjoint accb
template <typename T>
__global__ __launch_bounds__(256) void k_accel_kick_vjp(const T* __restrict__ U,
                                                        const T* __restrict__ acc, long long N,
                                                        T dt, const T* __restrict__ lin, T* lout,
                                                        T* __restrict__ accb) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const T rho = U[q], Eb = lin[4 * N + q];
  T rb = lin[q];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T a = acc[c * N + q];
    const T mb = lin[(1 + c) * N + q];
    rb += mb * a * dt;
    lout[(1 + c) * N + q] = mb + Eb * a * dt;
    accb[c * N + q] = mb * rho * dt + Eb * U[(1 + c) * N + q] * dt;
  }
  lout[q] = rb;
  lout[4 * N + q] = Eb;
}

// the three one-axis passes over the n^3 cube c, with the twiddles tw; with
// rin the x pass reads the real field rin instead of c, with rout the z pass
// writes only the real part of the result, to rout (c then holds no result)
// the three one-axis passes over the n^3 cube c, with the twiddles tw; with
// rin the x pass reads the real field rin (with rin2 too: rin + i rin2)
// instead of c, with rout the z pass writes only the real part of the result
// to rout (with rout2 too: the imaginary part to rout2; c then holds no
// result)
template <typename T>
hipError_t fft3_raw(typename CplxOf<T>::type* c, const typename CplxOf<T>::type* tw, int n,
                    int inverse, hipStream_t s, const T* rin = nullptr, T* rout = nullptr,
                    T* rout2 = nullptr, const T* rin2 = nullptr) {
  using C = typename CplxOf<T>::type;
  int logn = 0;
  while ((1 << logn) < n) ++logn;
  const long long lines = (long long)n * n;
  // lines per workgroup: a power of two, as many as fit in the LDS budget
  int loglpb = 0;
  while (((long long)n << (loglpb + 1)) <= (long long)FFT_THREADS * fft_elems<C>() &&
         (1ll << (loglpb + 1)) <= lines)
    ++loglpb;
  const unsigned grid = (unsigned)(lines >> loglpb);
  const size_t lds = (size_t)n * sizeof(C) << loglpb;
  T* const nul = nullptr;
  const T* const cnul = nullptr;
#define MH_LINES(AX, IO, RI, RI2, RO, RO2)                                                   \
  hipLaunchKernelGGL((k_fft_lines<T, AX, IO>), dim3(grid), dim3(FFT_THREADS), lds, s, c, RI, \
                     RI2, RO, RO2, tw, logn, loglpb, inverse)
  if (rin && rin2) MH_LINES(0, FFT_PAIR_IN, rin, rin2, nul, nul);
  else if (rin) MH_LINES(0, FFT_REAL_IN, rin, cnul, nul, nul);
  else MH_LINES(0, FFT_COMPLEX, cnul, cnul, nul, nul);
  MH_LINES(1, FFT_COMPLEX, cnul, cnul, nul, nul);
  if (rout && rout2) MH_LINES(2, FFT_SPLIT_OUT, cnul, cnul, rout, rout2);
  else if (rout) MH_LINES(2, FFT_REAL_OUT, cnul, cnul, rout, nul);
  else MH_LINES(2, FFT_COMPLEX, cnul, cnul, nul, nul);
#undef MH_LINES
  return hipGetLastError();
}

template <typename T>
hipError_t fft3(char* ws, const MGLayout& L, typename CplxOf<T>::type* c, int inverse,
                hipStream_t s, const T* rin = nullptr, T* rout = nullptr, T* rout2 = nullptr,
                const T* rin2 = nullptr) {
  using C = typename CplxOf<T>::type;
  return fft3_raw<T>(c, P<C>(ws, L.fft_tw), L.lev[0].n, inverse, s, rin, rout, rout2, rin2);
}

template <typename T>
hipError_t fft3_standalone(void* data, int n, int inverse, void* tw, hipStream_t s) {
  using C = typename CplxOf<T>::type;
  hipLaunchKernelGGL((k_fft_twiddles<T>), dim3(nblk(n / 2 > 0 ? n / 2 : 1)), dim3(256), 0, s,
                     (C*)tw, n);
  return fft3_raw<T>((C*)data, (const C*)tw, n, inverse, s);
}

}  // namespace

bool fft_size_ok(int n) { return n >= 2 && n <= 1024 && (n & (n - 1)) == 0; }

size_t fft_layout(int n, size_t off, size_t es, MGLayout& L) {
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t N = (size_t)n * n * n;
  L.fft = 1;
  L.fft_c0 = take(2 * N * es);
  L.fft_c1 = take(2 * N * es);
  L.fft_tw = take((size_t)(n / 2 > 0 ? n / 2 : 1) * 2 * es);
  L.fft_acc = take(3 * N * es);
  return off;
}

// From F = 4 pi G (rho - <rho>) on level 0: the potential into
// lev[0].phi[cur0] and the acceleration into fft_acc
template <typename T>
hipError_t fft_poisson(char* ws, MGLayout& L, double h, hipStream_t s) {
  using C = typename CplxOf<T>::type;
  const MGLevel& f = L.lev[0];
  const int n = f.n;
  const long long N = (long long)n * n * n;
  const double tk = 2.0 * M_PI / ((double)n * h);
  C* c0 = P<C>(ws, L.fft_c0);
  C* c1 = P<C>(ws, L.fft_c1);
  T* acc = P<T>(ws, L.fft_acc);
  hipLaunchKernelGGL((k_fft_twiddles<T>), dim3(nblk(n / 2 > 0 ? n / 2 : 1)), dim3(256), 0, s,
                     P<C>(ws, L.fft_tw), n);
  hipError_t e = fft3<T>(ws, L, c0, 0, s, P<T>(ws, f.F));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_phi<T>), dim3(nblk(N)), dim3(256), 0, s, c0, n, tk);
  // two inverse transforms for the four real outputs (a_x, a_y | a_z, Phi)
  hipLaunchKernelGGL((k_fft_grad_pairs<T>), dim3(nblk(N)), dim3(256), 0, s, c0, c1, n, tk);
  e = fft3<T>(ws, L, c1, 1, s, nullptr, acc, acc + N);
  if (e != hipSuccess) return e;
  e = fft3<T>(ws, L, c0, 1, s, nullptr, acc + 2 * N, P<T>(ws, f.phi[L.cur0]));
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// kick (+ cooling if `cool`), CFL and health check with the acceleration of
// the last fft_poisson
template <typename T>
hipError_t fft_sources(char* ws, const MGLayout& L, const mh_grid_desc& g, bool cool, bool cfl,
                       const CoolParams<T>& cp, T* U, DevClock* clk, hipStream_t s) {
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  const T* acc = P<T>(ws, L.fft_acc);
  if (cool)
    hipLaunchKernelGGL((k_accel_sources<T, true>), dim3(nblk_capped(N)), dim3(256), 0, s, U, acc, N,
                       (T)g.gamma, (T)(1.0 / g.h[0]), cp, clk, (int)cfl);
  else
    hipLaunchKernelGGL((k_accel_sources<T, false>), dim3(nblk_capped(N)), dim3(256), 0, s, U, acc, N,
                       (T)g.gamma, (T)(1.0 / g.h[0]), cp, clk, (int)cfl);
  return hipGetLastError();
}

// reverse of the spectral gravity kick at the state Ub the kick acted on
// (whose acceleration the last fft_poisson left in fft_acc): lout from lin,
// then lout_rho += (d a / d rho)^T accb
template <typename T>
hipError_t fft_gravity_vjp(char* ws, MGLayout& L, double h, double G, const T* Ub, T dt,
                           const T* lin, T* lout, T* accb, hipStream_t s) {
  using C = typename CplxOf<T>::type;
  const int n = L.lev[0].n;
  const long long N = (long long)n * n * n;
  const double tk = 2.0 * M_PI / ((double)n * h);
  const double fourpiG = 4.0 * M_PI * G;
  C* c0 = P<C>(ws, L.fft_c0);
  C* c1 = P<C>(ws, L.fft_c1);
  hipLaunchKernelGGL((k_accel_kick_vjp<T>), dim3(nblk(N)), dim3(256), 0, s, Ub,
                     P<T>(ws, L.fft_acc), N, dt, lin, lout, accb);
  hipLaunchKernelGGL((k_fft_twiddles<T>), dim3(nblk(n / 2 > 0 ? n / 2 : 1)), dim3(256), 0, s,
                     P<C>(ws, L.fft_tw), n);
  // x and y in one transform (two real fields as re + i im), then z
  hipError_t e = fft3<T>(ws, L, c1, 0, s, accb, nullptr, nullptr, accb + N);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_adj_accum_pair<T>), dim3(nblk(N)), dim3(256), 0, s, c1, c0, n, tk,
                     fourpiG);
  e = fft3<T>(ws, L, c1, 0, s, accb + 2 * N);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_adj_accum<T, 2>), dim3(nblk(N)), dim3(256), 0, s, c1, c0, n, tk,
                     fourpiG, 0);
  e = fft3<T>(ws, L, c0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_real_add<T>), dim3(nblk(N)), dim3(256), 0, s, c0, lout, N);
  return hipGetLastError();
}

#define FFT_INSTANTIATE(T)                                                                     \
  template hipError_t fft_poisson<T>(char*, MGLayout&, double, hipStream_t);                  \
  template hipError_t fft_sources<T>(char*, const MGLayout&, const mh_grid_desc&, bool, bool, \
                                     const CoolParams<T>&, T*, DevClock*, hipStream_t);       \
  template hipError_t fft_gravity_vjp<T>(char*, MGLayout&, double, double, const T*, T,       \
                                         const T*, T*, T*, hipStream_t);
FFT_INSTANTIATE(float)
FFT_INSTANTIATE(double)
#undef FFT_INSTANTIATE

}  // namespace mh

extern "C" mh_status mh_fft3_query_workspace(int32_t n, int32_t dtype, size_t* bytes) {
  if (!bytes) return MH_E_INVALID;
  if (!mh::fft_size_ok(n)) return MH_E_SHAPE;
  if (dtype != MH_F32 && dtype != MH_F64) return MH_E_DTYPE;
  const size_t es = dtype == MH_F64 ? 8 : 4;
  *bytes = (size_t)(n / 2 > 0 ? n / 2 : 1) * 2 * es;
  return MH_OK;
}

extern "C" mh_status mh_fft3(void* data, int32_t n, int32_t dtype, int32_t inverse,
                             void* workspace, size_t workspace_bytes, void* stream) {
  size_t need = 0;
  const mh_status st = mh_fft3_query_workspace(n, dtype, &need);
  if (st != MH_OK) return st;
  if (!data || !workspace || (inverse != 0 && inverse != 1)) return MH_E_INVALID;
  if (workspace_bytes < need) return MH_E_WORKSPACE;
  const hipError_t e =
      dtype == MH_F64
          ? mh::fft3_standalone<double>(data, n, inverse, workspace, (hipStream_t)stream)
          : mh::fft3_standalone<float>(data, n, inverse, workspace, (hipStream_t)stream);
  return e == hipSuccess ? MH_OK : MH_E_DEVICE;
}

// ------------------------------------------- the transform without allocation

// Twiddle table of mh_fft3_noalloc: n/2 complex values of the largest dtype at
// the largest n (512 x 16 B).  Each GPU the library runs on holds its own copy
// until the process ends; every call on that GPU rewrites it.
constexpr size_t FFT_SCRATCH_BYTES = 8192;
static __device__ __align__(256) char scratch[FFT_SCRATCH_BYTES];

namespace {
constexpr int FFT_SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[FFT_SCRATCH_MAX_DEVICES] = {};

// device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the host-side symbol is not a device address)
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= FFT_SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" mh_status mh_fft3_noalloc(void* data, int32_t n, int32_t dtype, int32_t inverse,
                                     void* stream) {
  size_t need = 0;
  const mh_status st = mh_fft3_query_workspace(n, dtype, &need);
  if (st != MH_OK) return st;
  if (!data || (inverse != 0 && inverse != 1)) return MH_E_INVALID;
  if (need > FFT_SCRATCH_BYTES) return MH_E_WORKSPACE;
  void* tw = nullptr;
  if (scratch_address(&tw) != hipSuccess) return MH_E_DEVICE;
  const hipError_t e =
      dtype == MH_F64 ? mh::fft3_standalone<double>(data, n, inverse, tw, (hipStream_t)stream)
                      : mh::fft3_standalone<float>(data, n, inverse, tw, (hipStream_t)stream);
  return e == hipSuccess ? MH_OK : MH_E_DEVICE;
}
