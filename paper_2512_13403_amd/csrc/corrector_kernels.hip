// corrector_kernels.hip -- the learned state corrector on gfx950 matrix cores.
//
// The corrector is a 3D convolutional network applied after a coarse step,
// trained through the solver (the solver-in-the-loop setting of arXiv
// 2512.13403 Sec. 8): x = (U - mean)/std, h1 = GELU(conv(x)), h2 =
// GELU(conv(h1)), y = conv(h2), U' = U + scale * y, with 3x3x3 periodic
// cross-correlations of 5 -> 32 -> 32 -> 5 channels.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16.  A
// workgroup stages a 16 x 4 x 4 block of cells plus its one-cell periodic halo
// in LDS (bf16, 32 channels per cell, channels contiguous); each of its four
// waves owns four rows of 16 cells along x (the MFMA rows) and all output
// channels (the MFMA columns, 16 per tile).  For each of the 27 taps a wave
// loads that tap's weight block once and multiplies it into its four rows,
// whose shifted inputs it reads from LDS, accumulating in fp32.  Activations
// are stored cell-major with 32 channels (the network input fills 10 of them:
// each of the 5 standardised fields as two bf16 parts, hi + lo, which meet
// the same first-layer weights, so the input keeps about 16 bits at no extra
// matrix-core work; the last layer's 5 outputs sit in 16).  The same kernel
// serves the input-gradient pass: there the weights are packed transposed
// with the taps mirrored, so reading at cell + off_tap applies the transpose
// of the forward map.  Weight gradients are GEMMs over cells: one workgroup
// per (tap, chunk of 4096 cells) writes a 32 x 32 partial product, and a
// second kernel adds the chunks in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "mh_corrector.h"

namespace mh {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned short)))) unsigned short u16x4;

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ bf16x8 load8(const unsigned short* p) {
  bf16x8 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// GELU(z) = z Phi(z), Phi(z) = erfc(-z / sqrt 2) / 2, and its derivative
// Phi(z) + z phi(z).  erfc is evaluated with the Chebyshev-fitted form of
// Press et al., Numerical Recipes (2nd ed., Sec. 6.2, erfcc): for x >= 0,
// erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + x/2), P a degree-9 polynomial,
// relative error below 1.2e-7 everywhere (so the negative side, where
// 1 + erf cancels, stays accurate), and erfc(-x) = 2 - erfc(x).  The same
// exponential gives phi(z) = exp(-z^2/2) / sqrt(2 pi).  About 15 VALU
// instructions instead of a library erfcf and a separate expf.
struct PhiPair {
  float Phi, phi;
};
__device__ __forceinline__ PhiPair normal_cdf_pdf(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  const float e = __expf(-x * x);           // exp(-z^2 / 2)
  const float ec = t * e * __expf(p);        // erfc(|z| / sqrt 2)
  const float Phi = z >= 0.0f ? 1.0f - 0.5f * ec : 0.5f * ec;
  return {Phi, e * 0.39894228040143268f};
}
__device__ __forceinline__ float gelu(float z) { return z * normal_cdf_pdf(z).Phi; }
__device__ __forceinline__ float gelu_grad(float z) {
  const PhiPair q = normal_cdf_pdf(z);
  return fmaf(z, q.phi, q.Phi);
}

enum : int { EPI_GELU = 0, EPI_LINEAR = 1, EPI_GELU_BWD = 2, EPI_RAW = 3, EPI_RESIDUAL = 4 };

// the last layer's epilogue in inference: out = U + scale * (y + bias) for the
// five fields of each cell (the residual update, written field-major like U)
template <typename TU>
struct ResArgs {
  const TU* U;
  TU* out;
  double scale[5];
  long long n3;  // cells per sample
};

// Halo tile of the tiled convolution: 16 cells along x (the MFMA rows) by
// CTY x CTZ rows in (y, z), with a one-cell periodic halo, staged in LDS.
constexpr int CTX = 16, CTY = 4, CTZ = 4;
constexpr int CHX = CTX + 2, CHY = CTY + 2, CHZ = CTZ + 2, CNH = CHX * CHY * CHZ;
constexpr int CROWS = CTY * CTZ / 4;  // rows per wave (4 waves)
constexpr int CPD = 4;                // weight prefetch distance, in taps
static_assert(CTX * CTY * CTZ == CORR_BLOCK_CELLS, "tile size");

typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;

// 16-byte channel chunk c of halo cell (hx, ...) sits in slot c ^ ((hx >> 2) & 3):
// the 16 lanes of a row read 16 consecutive hx and so 16 distinct bank groups.
__device__ __forceinline__ int cslot(int h, int hx, int c) { return h * 4 + (c ^ ((hx >> 2) & 3)); }

// out[cell][co] for COT output channels (16 or 32) from in[cell][32] (bf16):
// per tap, the wave's CROWS rows of 16 cells read their shifted inputs from
// the LDS tile and multiply them by the tap's 32 x COT weight block (bf16
// [NT][COT][32]), loaded once per tap and prefetched CPD taps ahead.  NT = 9
// for an input whose 32 channels already hold the three x neighbours (the
// first layer: 3 x 10 input parts): the taps then run over (dy, dz) only.
template <int COT, int EPI, int NT = 27, typename TU = float>
__global__ __launch_bounds__(256, 3) void k_conv(const unsigned short* __restrict__ in,
                                              const unsigned short* __restrict__ w,
                                              const float* __restrict__ bias, int nbias, int n,
                                              const float* __restrict__ zin,
                                              float* __restrict__ fout,
                                              unsigned short* __restrict__ hout, int ntiles,
                                              ResArgs<TU> ra) {
  __shared__ u32x4 tile[CNH * 4];
  constexpr int NLD = (CNH * 4 + 255) / 256;  // 16-byte halo chunks per thread
  const int ntx = n / CTX, nty = n / CTY, ntz = n / CTZ;
  // tile t: origin (x0, y0, z0) in sample b, whose first cell is `base`
  auto origin = [&](int t, int& x0, int& y0, int& z0, long long& base) {
    const int bx = t % ntx;
    t /= ntx;
    const int by = t % nty;
    t /= nty;
    const int bz = t % ntz;
    base = (long long)(t / ntz) * n * n * (long long)n;
    x0 = bx * CTX;
    y0 = by * CTY;
    z0 = bz * CTZ;
  };
  // a persistent workgroup walks the tiles t = blockIdx.x, + gridDim.x, ...;
  // the halo of its next tile is loaded into registers while the current
  // tile's outputs are formed and stored, then written to LDS
  // (the thread index is made opaque where the chunk coordinates are
  // derived, so that they are recomputed per tile rather than hoisted out of
  // the tile loop and held in registers)
  u32x4 pre[NLD];
  auto fetch = [&](int t) {
    int x0, y0, z0;
    long long base;
    origin(t, x0, y0, z0, base);
    unsigned tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const unsigned short* ib = in + base * 32;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      // lanes past the last chunk load the last chunk again (unused): every
      // load is unconditional
      const unsigned i = min(tid + 256u * k, (unsigned)(CNH * 4 - 1));
      const unsigned h = i >> 2, c = i & 3;
      const unsigned hx = h % CHX, hy = (h / CHX) % CHY, hz = h / (CHX * CHY);
      const unsigned zy = (unsigned)wrap(z0 - 1 + (int)hz, n) * (unsigned)n +
                          (unsigned)wrap(y0 - 1 + (int)hy, n);
      const size_t src = (size_t)zy * (unsigned)n + (unsigned)wrap(x0 - 1 + (int)hx, n);
      __builtin_memcpy(&pre[k], ib + src * 32 + c * 8, 16);
    }
  };
  fetch(blockIdx.x);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + 256 * k;
      if (i < CNH * 4) {
        const int h = i >> 2;
        tile[cslot(h, h % CHX, i & 3)] = pre[k];
      }
    }
    __syncthreads();
    int x0, y0, z0;
    long long base;
    origin(t, x0, y0, z0, base);
    const int lane = tid & 63, wave = tid >> 6;  // (tid: opaque, see above)
    const int row = lane & 15, grp = lane >> 4;
    // the wave's rows (y0 + r, z0 + wave) for r < CROWS = CTY: the halo slab
    // hz = wave + 1 + dz starts at wtile; lslot: the lane's slot offset for
    // dx = -1, 0, 1 (cslot of hx = row + 1 + dx, channel chunk grp)
    static_assert(CROWS == CTY, "a wave's rows are one z-row of the tile");
    const u32x4* wtile = tile + ((wave + 1) * CHY) * CHX * 4;
    int lslot[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lslot[d] = cslot(0, row + d, grp) + (row + d) * 4;
    f32x4 acc[CROWS][COT / 16];
#pragma unroll
    for (int r = 0; r < CROWS; ++r)
#pragma unroll
      for (int nt = 0; nt < COT / 16; ++nt) acc[r][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weights: CPD taps in flight (a register ring), so the load of a tap's
    // block is issued CPD taps before its MFMAs
    // (opaque per tile: the weight loads stay inside the tile loop instead of
    // being hoisted out of it and held, all 27 taps, in registers)
    const unsigned short* wl = w + row * 32 + 8 * grp;
    asm volatile("" : "+v"(wl));
    bf16x8 bq[CPD][COT / 16];
#pragma unroll
    for (int p = 0; p < CPD; ++p)
#pragma unroll
      for (int nt = 0; nt < COT / 16; ++nt) bq[p][nt] = load8(wl + (p * COT + nt * 16) * 32);
#pragma unroll
    for (int tap = 0; tap < NT; ++tap) {
      bf16x8 bw[COT / 16];
#pragma unroll
      for (int nt = 0; nt < COT / 16; ++nt) bw[nt] = bq[tap % CPD][nt];
      if (tap + CPD < NT) {
#pragma unroll
        for (int nt = 0; nt < COT / 16; ++nt)
          bq[tap % CPD][nt] = load8(wl + ((tap + CPD) * COT + nt * 16) * 32);
      }
      // 27 taps (dx, dy, dz); 9 taps (dy, dz) when the x shifts are packed
      // into the input channels (the first layer)
      const int dx = NT == 27 ? tap % 3 - 1 : 0;
      const int dy = NT == 27 ? (tap / 3) % 3 - 1 : tap % 3 - 1;
      const int dz = NT == 27 ? tap / 9 - 1 : tap / 3 - 1;
#pragma unroll
      for (int r = 0; r < CROWS; ++r) {
        // row r of the wave: hy = r + 1 + dy, hz = wave + 1 + dz; the lane's
        // part of the slot depends on dx only, the rest is a constant
        const u32x4 raw = wtile[lslot[dx + 1] + ((dz * CHY + r + 1 + dy) * CHX) * 4];
        bf16x8 a;
        __builtin_memcpy(&a, &raw, 16);
#pragma unroll
        for (int nt = 0; nt < COT / 16; ++nt)
          acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[nt], a, acc[r][nt], 0, 0, 0);
      }
    }
    // the next tile's loads are in flight during the epilogue
    if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);
    // the weights are the A operand (rows: output channels) and the shifted
    // inputs B (columns: the row's 16 cells), so lane (row, grp) holds output
    // channels nt * 16 + 4 grp .. + 3 of cell x0 + row: four consecutive
    // channels, written with one vector store per (row, tile)
#pragma unroll
    for (int r = 0; r < CROWS; ++r) {
      const int j = wave * CROWS + r;
      const long long cell =
          base + ((long long)(z0 + j / CTY) * n + (y0 + j % CTY)) * n + x0 + row;
#pragma unroll
      for (int nt = 0; nt < COT / 16; ++nt) {
        const int co = nt * 16 + 4 * grp;
        const long long o = cell * COT + co;
        const f32x4 v = acc[r][nt];
        if (EPI == EPI_GELU) {
          f32x4 zz;
          unsigned short hv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            zz[q] = v[q] + bias[co + q];
            hv[q] = f2bf(gelu(zz[q]));
          }
          if (fout) *(f32x4*)(fout + o) = zz;
          *(u16x4*)(hout + o) = u16x4{hv[0], hv[1], hv[2], hv[3]};
        } else if (EPI == EPI_LINEAR) {
          f32x4 y;
#pragma unroll
          for (int q = 0; q < 4; ++q) y[q] = v[q] + (co + q < nbias ? bias[co + q] : 0.f);
          *(f32x4*)(fout + o) = y;
        } else if (EPI == EPI_RESIDUAL) {
          // lanes of channel groups 0 and 1 hold fields 0-3 and 4; the
          // arithmetic of k_residual
          const long long b = cell / ra.n3, q = cell - b * ra.n3;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int c = co + k;
            if (c < 5) {
              const float y = v[k] + bias[c];
              const TU d = (TU)(ra.scale[c] * (double)y);
              const long long f = (b * 5 + c) * ra.n3 + q;
              ra.out[f] = ra.U[f] + d;
            }
          }
        } else if (EPI == EPI_GELU_BWD) {
          const f32x4 zi = *(const f32x4*)(zin + o);
          unsigned short hv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) hv[q] = f2bf(v[q] * gelu_grad(zi[q]));
          *(u16x4*)(hout + o) = u16x4{hv[0], hv[1], hv[2], hv[3]};
        } else {
          *(f32x4*)(fout + o) = v;
        }
      }
    }
    __syncthreads();  // the tile is read by every wave before the next is stored
  }
}

// Weight gradient of one layer, dW[tap][co][ci] = sum over cells of
// dz[cell][co] x[cell + off_tap][ci], on the same 16 x 4 x 4 halo tiles as
// k_conv.  A persistent workgroup takes every gridDim.x-th block of cells; per
// block it stages the layer input with its halo and the block's output
// gradients in LDS, both channel-major (each channel's x rows contiguous), so
// that every MFMA operand of a lane -- 8 consecutive cells of one channel --
// is one 16-byte LDS read; the next block's data is loaded into registers
// while the current one is reduced.  Per MFMA the reduction runs over 32
// cells (16 along x in two rows), dz^T is the A operand (rows: output
// channels) and the shifted input the B operand (columns: input channels).
// The taps are grouped by their (dy, dz) row: wave w takes the rows w and
// w + 4 with their three x shifts, and waves 0-2 one x shift each of row 8
// (seven taps per wave); a lane reads cells xs .. xs + 9 of its channel (one
// 16-byte and one 4-byte read) and forms the shifted operands in registers
// (the shift by one cell is a byte alignment of neighbouring words, the
// shift by two a choice of words).  Wave 3 forms the bias gradient (slot 27).
// Each workgroup writes its partial [28][COT][32]; k_wgrad_reduce adds them
// in a fixed order (deterministic, no atomics).
constexpr int WXS = 24;                      // x stride of a staged row (18 used), 16-byte aligned
constexpr int WCS = CHY * CHZ * WXS + 8;     // channel stride of the input tile: 109 x 16 B
constexpr int WDS = CTX * CTY * CTZ + 8;     // channel stride of the gradients: 33 x 16 B

template <int COT, bool XPACK = false>
__global__ __launch_bounds__(256, 2) void k_wgrad(const unsigned short* __restrict__ dz,
                                               const unsigned short* __restrict__ x, int n,
                                               int nblocks, float* __restrict__ partial) {
  constexpr int CB = CTX * CTY * CTZ;  // cells per block
  static_assert(CHX % 2 == 0 && CTX % 2 == 0, "cell pairs stay within an x row");
  __shared__ u32x4 tin[32 * WCS / 8];
  __shared__ u32x4 dzs[COT * WDS / 8];
  unsigned short* tin16 = reinterpret_cast<unsigned short*>(tin);
  unsigned short* dz16 = reinterpret_cast<unsigned short*>(dzs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int ntx = n / CTX, nty = n / CTY, ntz = n / CTZ;
  // acc[row][dx + 1][co tile][ci tile] for the wave's rows g = wave and
  // wave + 4; acc8: waves 0-2 the tap (dy, dz) row 8, dx = wave - 1 (the
  // taps split evenly, seven per wave), wave 3 the bias gradient
  f32x4 acc[2][3][COT / 16][2], acc8[COT / 16][2];
#pragma unroll
  for (int gg = 0; gg < 2; ++gg)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int mt = 0; mt < COT / 16; ++mt)
        acc[gg][d][mt][0] = acc[gg][d][mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < COT / 16; ++mt) acc8[mt][0] = acc8[mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  // The next block's tile and gradients are loaded into registers while the
  // current block is reduced (the loads of a block are issued before the
  // MFMA loop of the previous one), then transposed into LDS.
  constexpr int NIN = ((CNH / 2) * 4 + 255) / 256;       // input items per thread
  constexpr int NDZ = ((CB / 2) * (COT / 8) + 255) / 256;  // gradient items per thread
  u32x4 rin[NIN][2], rdz[NDZ][2];
  auto load_block = [&](int blk) {
    int t = blk;
    const int bx = t % ntx;
    t /= ntx;
    const int by = t % nty;
    t /= nty;
    const int bz = t % ntz;
    const long long b = t / ntz;
    const int x0 = bx * CTX, y0 = by * CTY, z0 = bz * CTZ;
    const long long base = b * n * n * (long long)n;
    // the halo tile: two cells of one x row and 8 channels per item
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < (CNH / 2) * 4) {
        const int hp = i % (CNH / 2), c = i / (CNH / 2);
        const int h = 2 * hp;
        const int hx = h % CHX, hr = h / CHX;  // hr = hz * CHY + hy
        const int hy = hr % CHY, hz = hr / CHY;
        const long long rowc =
            base + ((long long)wrap(z0 - 1 + hz, n) * n + wrap(y0 - 1 + hy, n)) * n;
        __builtin_memcpy(&rin[k][0], x + (rowc + wrap(x0 - 1 + hx, n)) * 32 + c * 8, 16);
        __builtin_memcpy(&rin[k][1], x + (rowc + wrap(x0 + hx, n)) * 32 + c * 8, 16);
      }
    }
    // the block's output gradients: two cells and 8 channels per item
#pragma unroll
    for (int k = 0; k < NDZ; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < (CB / 2) * (COT / 8)) {
        const int pr = i % (CB / 2), c = i / (CB / 2);
        const int cl = 2 * pr, r = cl / CTX;
        const long long cell =
            base + ((long long)(z0 + r / CTY) * n + (y0 + r % CTY)) * n + x0 + cl % CTX;
        __builtin_memcpy(&rdz[k][0], dz + cell * COT + c * 8, 16);
        __builtin_memcpy(&rdz[k][1], dz + (cell + 1) * COT + c * 8, 16);
      }
    }
  };
  // two cells' 8 channels as 8 32-bit words (cell pair per channel) at dst,
  // one word per `stride` 16-bit elements
  auto put_pair = [](unsigned int* dst, int stride, const u32x4& v0, const u32x4& v1) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned int lo = j & 1 ? v0[j >> 1] >> 16 : v0[j >> 1] & 0xffffu;
      const unsigned int hi = j & 1 ? v1[j >> 1] >> 16 : v1[j >> 1] & 0xffffu;
      dst[j * (stride / 2)] = lo | (hi << 16);
    }
  };
  if (blockIdx.x < nblocks) load_block(blockIdx.x);
  for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < (CNH / 2) * 4) {
        const int hp = i % (CNH / 2), c = i / (CNH / 2);
        const int h = 2 * hp;
        put_pair(reinterpret_cast<unsigned int*>(tin16 + (c * 8) * WCS + (h / CHX) * WXS + h % CHX),
                 WCS, rin[k][0], rin[k][1]);
      }
    }
#pragma unroll
    for (int k = 0; k < NDZ; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < (CB / 2) * (COT / 8)) {
        const int pr = i % (CB / 2), c = i / (CB / 2);
        put_pair(reinterpret_cast<unsigned int*>(dz16 + (c * 8) * WDS + 2 * pr), WDS, rdz[k][0],
                 rdz[k][1]);
      }
    }
    __syncthreads();
    if (blk + (int)gridDim.x < nblocks) load_block(blk + gridDim.x);
#pragma unroll 1
    for (int ks = 0; ks < CB / 32; ++ks) {
      // this lane's 8 cells of the 32-cell step: x = xs .. xs + 7 of row r
      const int r = 2 * ks + (grp >> 1), xs = 8 * (grp & 1);
      const int ty = r % CTY, tz = r / CTY;
      bf16x8 a[COT / 16];
#pragma unroll
      for (int mt = 0; mt < COT / 16; ++mt)
        __builtin_memcpy(&a[mt], dz16 + (mt * 16 + row) * WDS + r * CTX + xs, 16);
      // input channel ci at hx = xs .. xs + 9 of (dy, dz) row g: the strip
      // for dx = -1, 0, 1, as the operand for shift d
      auto strip = [&](int g, int ct, u32x4& lo, unsigned int& hi) {
        const int hrow = (tz + g / 3) * CHY + (ty + g % 3);
        const unsigned short* src = tin16 + (ct * 16 + row) * WCS + hrow * WXS + xs;
        __builtin_memcpy(&lo, src, 16);
        __builtin_memcpy(&hi, src + 8, 4);
      };
      auto shifted = [](int d, const u32x4& lo, unsigned int hi) {
        u32x4 w;
        if (d == 0) {
          w = lo;
        } else if (d == 1) {
          w[0] = __builtin_amdgcn_alignbyte(lo[1], lo[0], 2);
          w[1] = __builtin_amdgcn_alignbyte(lo[2], lo[1], 2);
          w[2] = __builtin_amdgcn_alignbyte(lo[3], lo[2], 2);
          w[3] = __builtin_amdgcn_alignbyte(hi, lo[3], 2);
        } else {
          w[0] = lo[1];
          w[1] = lo[2];
          w[2] = lo[3];
          w[3] = hi;
        }
        bf16x8 bv;
        __builtin_memcpy(&bv, &w, 16);
        return bv;
      };
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        const int g = wave + 4 * gg;  // (dy, dz) row: dy = g % 3 - 1, dz = g / 3 - 1
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          u32x4 lo;
          unsigned int hi;
          strip(g, ct, lo, hi);
#pragma unroll
          for (int d = XPACK ? 1 : 0; d < (XPACK ? 2 : 3); ++d) {
            const bf16x8 bv = shifted(d, lo, hi);
#pragma unroll
            for (int mt = 0; mt < COT / 16; ++mt)
              acc[gg][d][mt][ct] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bv, acc[gg][d][mt][ct], 0, 0, 0);
          }
        }
      }
      if (wave < 3 && (!XPACK || wave == 1)) {
        // row 8 at the x shift dx = wave - 1 (a packed input has only dx = 0)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          u32x4 lo;
          unsigned int hi;
          strip(8, ct, lo, hi);
          const bf16x8 bv = wave == 0 ? shifted(0, lo, hi)
                                      : (wave == 1 ? shifted(1, lo, hi) : shifted(2, lo, hi));
#pragma unroll
          for (int mt = 0; mt < COT / 16; ++mt)
            acc8[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bv, acc8[mt][ct], 0, 0, 0);
        }
      } else if (wave == 3) {
        // the bias gradient, sum over cells of dz, as one more product with a
        // B operand of ones (column 0 is kept)
        bf16x8 ones;
        const unsigned short one[8] = {0x3F80, 0x3F80, 0x3F80, 0x3F80,
                                       0x3F80, 0x3F80, 0x3F80, 0x3F80};
        __builtin_memcpy(&ones, one, 16);
#pragma unroll
        for (int mt = 0; mt < COT / 16; ++mt)
          acc8[mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], ones, acc8[mt][0], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  auto put = [&](int tap, const f32x4 (&ac)[COT / 16][2]) {
#pragma unroll
    for (int mt = 0; mt < COT / 16; ++mt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int co = mt * 16 + 4 * grp + q, ci = ct * 16 + row;
          partial[(((long long)blockIdx.x * 28 + tap) * COT + co) * 32 + ci] = ac[mt][ct][q];
        }
  };
#pragma unroll
  for (int gg = 0; gg < 2; ++gg)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (!XPACK || d == 1) put(3 * (wave + 4 * gg) + d, acc[gg][d]);  // packed: dx = 0 only
  if (wave == 3) put(27, acc8);
  else if (!XPACK || wave == 1) put(24 + wave, acc8);
}

// gtheta[off + (co * ci_real + ci) * 27 + tap] += sum of the nwg partials
// [nwg][28][cot][32]; with `fold`, input channel ci also collects channel
// ci + ci_real (the two bf16 parts of the network input share the first
// layer's weights).  The co_real entries after the weights take the bias
// gradient (slot 27, column 0) into gb.  A block takes 64 consecutive
// elements of a partial (one per lane, ci fastest, so each load of a wave is
// 256 contiguous bytes); wave v adds the partials v, v + 4, ... in order, and
// the four sums are added in a fixed order: the result is deterministic.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial, int cot,
                                                      int nwg, int co_real, int ci_real,
                                                      int fold, int xpack, float* __restrict__ g,
                                                      float* __restrict__ gb) {
  __shared__ float sp[4][64];
  const int per = 28 * cot * 32;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int ci = e % 32, co = (e / 32) % cot, tap = e / (32 * cot);
  const bool need =
      e < per && co < co_real && (tap == 27 ? ci == 0 : ci < ci_real);
  const bool two = fold && tap < 27;
  // xpack: the partial of (dy, dz) row g = tap / 3 sits at slot 3 g + 1, its
  // x shift dx = tap % 3 - 1 in input-channel block 2 ci_real (dx + 1)
  const int src = (xpack && tap < 27)
                      ? ((3 * (tap / 3) + 1) * cot + co) * 32 + 2 * ci_real * (tap % 3) + ci
                      : e;
  float acc = 0.f;
  if (need) {
#pragma unroll 8
    for (int w = wv; w < nwg; w += 4) {
      const float* pw = partial + (long long)w * per;
      acc += two ? pw[src] + pw[src + ci_real] : pw[src];
    }
  }
  sp[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && need) {
    const float tot = ((sp[0][lane] + sp[1][lane]) + sp[2][lane]) + sp[3][lane];
    if (tap < 27) g[(co * ci_real + ci) * 27 + tap] += tot;
    else gb[co] += tot;
  }
}

// network input, two bf16 parts per channel: with x32 = float((U_c - mean_c) /
// std_c), hi = bf16(x32) and lo = bf16(x32 - hi) (the difference is exact in
// fp32), stored for the three x neighbours of the cell: x[cell][10 (dx + 1) +
// c] = hi and x[cell][10 (dx + 1) + 5 + c] = lo of cell x + dx (periodic),
// channels 30, 31 zero, so the first layer's three x taps meet one 32-wide
// operand (its K dimension) instead of three mostly zero ones
template <typename T>
__global__ __launch_bounds__(256) void k_standardize(const T* __restrict__ U, int n, long long cells,
                                                     CorrStats st, unsigned short* __restrict__ x) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  const long long n3 = (long long)n * n * n;
  const long long b = cell / n3, q = cell % n3;
  const int ix = (int)(q % n);
  const long long row = q - ix;
  unsigned short v[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) v[c] = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int xs = ix + d - 1 < 0 ? n - 1 : (ix + d - 1 >= n ? 0 : ix + d - 1);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const float s = (float)(((double)U[(b * 5 + c) * n3 + row + xs] - st.mean[c]) / st.std[c]);
      v[10 * d + c] = f2bf(s);
      v[10 * d + 5 + c] = f2bf(s - bf2f(v[10 * d + c]));
    }
  }
#pragma unroll
  for (int c = 0; c < 32; c += 8) __builtin_memcpy(x + cell * 32 + c, v + c, 16);
}

// U' = U + scale * y (y: [cell][16] fp32, first 5 channels)
template <typename T>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ U, const float* __restrict__ y,
                                                  int n, long long cells, CorrStats st,
                                                  T* __restrict__ out, int add_u) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  const long long n3 = (long long)n * n * n;
  const long long b = cell / n3, q = cell % n3;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const T d = (T)(st.scale[c] * (double)y[cell * 16 + c]);
    out[(b * 5 + c) * n3 + q] = add_u ? U[(b * 5 + c) * n3 + q] + d : d;
  }
}

// per-sample sums of rho and P of the uncorrected state (two-stage, fixed order)
template <typename T>
__global__ __launch_bounds__(256) void k_rho_p_partial(const T* __restrict__ U, long long n3, double gm1,
                                                       int blocks_per_sample, double* __restrict__ part) {
  __shared__ double sr[256], sp[256];
  const int b = blockIdx.x / blocks_per_sample, blk = blockIdx.x % blocks_per_sample;
  double r = 0.0, p = 0.0;
  for (long long q = (long long)blk * 256 + threadIdx.x; q < n3; q += (long long)blocks_per_sample * 256) {
    const double rho = (double)U[(b * 5) * n3 + q];
    const double mx = (double)U[(b * 5 + 1) * n3 + q], my = (double)U[(b * 5 + 2) * n3 + q],
                 mz = (double)U[(b * 5 + 3) * n3 + q], E = (double)U[(b * 5 + 4) * n3 + q];
    r += rho;
    p += gm1 * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho);
  }
  sr[threadIdx.x] = r;
  sp[threadIdx.x] = p;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      sp[threadIdx.x] += sp[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = sp[0];
  }
}

// positivity floor: rho >= f <rho>, then P >= f <P> by raising E at fixed m;
// counts floored and non-finite cells
// the floor values of each sample, frel times the mean density and pressure,
// from the k_rho_p_partial sums (one thread per sample, partials added in
// block order): ref[2 b] = rho floor, ref[2 b + 1] = pressure floor
__global__ __launch_bounds__(64) void k_floor_ref(const double* __restrict__ part,
                                                  int blocks_per_sample, int batch, long long n3,
                                                  double frel, double* __restrict__ ref) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= batch) return;
  double sr = 0.0, sp = 0.0;
  for (int k = 0; k < blocks_per_sample; ++k) {
    sr += part[2 * (b * blocks_per_sample + k)];
    sp += part[2 * (b * blocks_per_sample + k) + 1];
  }
  ref[2 * b] = frel * sr / (double)n3;
  ref[2 * b + 1] = frel * sp / (double)n3;
}

template <typename T>
__global__ __launch_bounds__(256) void k_floor(T* __restrict__ U, long long n3, long long cells, double gm1,
                                               const double* __restrict__ ref,
                                               unsigned long long* __restrict__ cpart) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  bool fl = false, bad = false;
  if (cell < cells) {
    const long long b = cell / n3, q = cell % n3;
    const double rf = ref[2 * b], pf = ref[2 * b + 1];
    T* u = U + b * 5 * n3 + q;
    double rho = (double)u[0];
    if (rho < rf) {
      rho = rf;
      u[0] = (T)rf;
      fl = true;
    }
    const double mx = (double)u[n3], my = (double)u[2 * n3], mz = (double)u[3 * n3];
    const double ek = 0.5 * (mx * mx + my * my + mz * mz) / rho;
    const double p = gm1 * ((double)u[4 * n3] - ek);
    if (p < pf) {
      u[4 * n3] = (T)(ek + pf / gm1);
      fl = true;
    }
    bad = !(isfinite(rho) && isfinite(mx) && isfinite(my) && isfinite(mz) &&
            isfinite((double)u[4 * n3]));
  }
  // the block's counts, without atomics (a mostly floored state would
  // serialise them on two addresses); k_count_sum adds the blocks
  __shared__ unsigned long long sc[2][4];
  const unsigned long long nf = __popcll(__ballot(fl)), nb = __popcll(__ballot(bad));
  if ((threadIdx.x & 63) == 0) {
    sc[0][threadIdx.x >> 6] = nf;
    sc[1][threadIdx.x >> 6] = nb;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    cpart[2 * blockIdx.x + threadIdx.x] =
        sc[threadIdx.x][0] + sc[threadIdx.x][1] + sc[threadIdx.x][2] + sc[threadIdx.x][3];
}

// counters[k] = sum over blocks of cpart[2 b + k] (fixed order)
__global__ __launch_bounds__(256) void k_count_sum(const unsigned long long* __restrict__ cpart,
                                                   int nblocks,
                                                   unsigned long long* __restrict__ counters) {
  __shared__ unsigned long long s[2][256];
  unsigned long long a = 0, b = 0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    a += cpart[2 * i];
    b += cpart[2 * i + 1];
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s[0][threadIdx.x] += s[0][threadIdx.x + st];
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) counters[threadIdx.x] = s[threadIdx.x][0];
}



// fallback on the device: when any value was non-finite or more than `limit`
// cells were floored, out = U (the plain state); counters as k_floor left them
template <typename T>
__global__ __launch_bounds__(256) void k_fallback(const T* __restrict__ U, T* __restrict__ out,
                                                  long long count, double limit,
                                                  const unsigned long long* __restrict__ counters) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  if (counters[1] > 0 || (double)counters[0] > limit) out[i] = U[i];
}

__global__ __launch_bounds__(256) void k_fill_f32(float* p, int count, float v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = v;
}

// upstream gradient of the network output: with a target T, the loss
// L = sum_c w_c mean((U'_c - T_c)^2) / sigma_c^2 (per-block partials) and its
// gradient 2 w_c (U'_c - T_c) / (sigma_c^2 cells); plus gUc = dL/dU' from the
// caller when given; dY[cell][c] = bf16(scale_c * (sum of both)); the sum
// itself goes to gfull when given (the residual path of dL/dU)
template <typename T>
__global__ __launch_bounds__(256) void k_loss(const T* __restrict__ U, const float* __restrict__ y,
                                              const T* __restrict__ tgt,
                                              const T* __restrict__ gup, int n, long long cells,
                                              CorrStats st, double* __restrict__ part,
                                              unsigned short* __restrict__ dy,
                                              T* __restrict__ gfull, int ident) {
  __shared__ double sl[256];
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (cell < cells) {
    const long long n3 = (long long)n * n * n;
    const long long b = cell / n3, q = cell % n3;
    unsigned short v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double g = 0.0;
      if (tgt) {
        const double uc = (double)U[(b * 5 + c) * n3 + q] + st.scale[c] * (double)y[cell * 16 + c];
        const double d = uc - (double)tgt[(b * 5 + c) * n3 + q];
        const double s2 = st.std[c] * st.std[c];
        l += st.lw[c] * d * d / s2;
        g = 2.0 * st.lw[c] * d / s2 / (double)cells;
      }
      if (gup) g += (double)gup[(b * 5 + c) * n3 + q];
      if (gfull) gfull[(b * 5 + c) * n3 + q] = ident ? (T)g : T(0);
      v[c] = f2bf((float)(st.scale[c] * g));
    }
    __builtin_memcpy(dy + cell * 16, v, 16);
    __builtin_memcpy(dy + cell * 16 + 8, v + 8, 16);
  }
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sl[threadIdx.x] += sl[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sl[0];
}

// the cell's own two parts (channels 10..19 of the x-packed input) in the
// unpacked layout [cell][32]: hi at c, lo at 5 + c, zeros after
__global__ __launch_bounds__(256) void k_unpack_input(const unsigned short* __restrict__ xp,
                                                      long long cells,
                                                      unsigned short* __restrict__ x0) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  unsigned short v[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) v[c] = c < 10 ? xp[cell * 32 + 10 + c] : 0;
#pragma unroll
  for (int c = 0; c < 32; c += 8) __builtin_memcpy(x0 + cell * 32 + c, v + c, 16);
}

// dL/dU += gx_c / std_c (gU holds the upstream gradient of U', the residual
// path; gx: [cell][16] fp32, the first layer's transposed convolution of dZ1;
// the two-part input split and the positivity floor pass the gradient
// through unchanged)
template <typename T>
__global__ __launch_bounds__(256) void k_input_grad(const float* __restrict__ gx, int n,
                                                    long long cells, CorrStats st,
                                                    T* __restrict__ gU) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  const long long n3 = (long long)n * n * n;
  const long long b = cell / n3, q = cell % n3;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const long long o = (b * 5 + c) * n3 + q;
    gU[o] = (T)((double)gU[o] + (double)gx[cell * 16 + c] / st.std[c]);
  }
}

// dY of 16 channels -> 32-channel operand layout for the next MFMA pass
__global__ __launch_bounds__(256) void k_pad16to32(const unsigned short* __restrict__ a, long long cells,
                                                   unsigned short* __restrict__ b) {
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  unsigned short v[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) v[c] = c < 16 ? a[cell * 16 + c] : 0;
#pragma unroll
  for (int c = 0; c < 32; c += 8) __builtin_memcpy(b + cell * 32 + c, v + c, 16);
}

__global__ __launch_bounds__(256) void k_dsum(const double* __restrict__ part, int n, double* out) {
  // fixed-order block reduction: strided per-thread sums, then a tree in LDS
  __shared__ double sd[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  sd[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sd[threadIdx.x] += sd[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sd[0];
}

// ADAM on the fp32 master parameters, then the bf16 operand layouts:
// forward weights [27][COT][32] and mirrored-transposed input-gradient weights
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int count, float lr, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.f - b1) * g[i];
  const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// first layer with the x taps packed into K: w1p[g][co][k], g = 3 (dz + 1) +
// (dy + 1), k = 10 (dx + 1) + j: W1[co][j mod 5][tap(dx, dy, dz)] for j < 10
// (both input parts share the weights), zero for k >= 30
__global__ __launch_bounds__(256) void k_pack_w1(const float* __restrict__ th, int off,
                                                 unsigned short* __restrict__ wf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 9 * 32 * 32) return;
  const int g = i / 1024, co = (i / 32) % 32, k = i % 32;
  float val = 0.f;
  if (k < 30) val = th[off + (co * 5 + (k % 10) % 5) * 27 + 3 * g + k / 10];
  wf[i] = f2bf(val);
}

__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ th, int off, int co_real,
                                              int ci_real, int dup, int cot,
                                              unsigned short* __restrict__ wf, int cit_t,
                                              unsigned short* __restrict__ wt) {
  // forward: wf[tap][co][ci] (co < cot, ci < 32), with `dup` the input
  // channels ci_real..2 ci_real-1 repeating 0..ci_real-1; transposed-mirrored
  // (when wt is given): wt[26 - tap][ci][co] (ci < cit_t rows, co < 32)
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 27 * cot * 32) return;
  const int tap = i / (cot * 32), co = (i / 32) % cot, ci = i % 32;
  const int cs = (dup && ci >= ci_real) ? ci - ci_real : ci;
  float val = 0.f;
  if (co < co_real && cs < ci_real) val = th[off + (co * ci_real + cs) * 27 + tap];
  const unsigned short h = f2bf(val);
  if (wf) wf[i] = h;
  if (wt && ci < cit_t) wt[((long long)(26 - tap) * cit_t + ci) * 32 + co] = h;
}

// conservative block average of a fine state [5][nf^3] onto [5][(nf/r)^3]
template <typename T>
__global__ __launch_bounds__(256) void k_block_average(const T* __restrict__ fine, int nf, int r,
                                                       T* __restrict__ coarse) {
  const int nc = nf / r;
  const long long Nc = (long long)nc * nc * nc, Nf = (long long)nf * nf * nf;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= 5 * Nc) return;
  const int f = (int)(t / Nc);
  const long long q = t % Nc;
  const int I = (int)(q % nc), J = (int)((q / nc) % nc), K = (int)(q / ((long long)nc * nc));
  double s = 0.0;
  for (int c = 0; c < r; ++c)
    for (int b = 0; b < r; ++b)
      for (int a = 0; a < r; ++a)
        s += (double)fine[f * Nf + ((long long)(K * r + c) * nf + (J * r + b)) * nf + (I * r + a)];
  coarse[t] = (T)(s / (double)(r * r * r));
}

inline unsigned blocks(long long n, int per) { return (unsigned)((n + per - 1) / per); }

inline unsigned conv_grid(int n, int batch) {
  return (unsigned)((long long)(n / CTX) * (n / CTY) * (n / CTZ) * batch);
}

// persistent convolution workgroups: three per CU of a 256-CU MI355X (the
// LDS tile allows three), never more than there are tiles
inline unsigned conv_wgs(unsigned ntiles) { return ntiles < 768u ? ntiles : 768u; }

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t corr_pack_weights(const CorrBuffers& B, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(blocks(27 * 32 * 32, 256)), dim3(256), 0, s, B.theta,
                     CORR_OFF_W1, 32, 5, 1, 32, (unsigned short*)nullptr, 16, B.w1t);
  hipLaunchKernelGGL(k_pack_w1, dim3(blocks(9 * 32 * 32, 256)), dim3(256), 0, s, B.theta,
                     CORR_OFF_W1, B.w1);
  hipLaunchKernelGGL(k_pack, dim3(blocks(27 * 32 * 32, 256)), dim3(256), 0, s, B.theta,
                     CORR_OFF_W2, 32, 32, 0, 32, B.w2, 32, B.w2t);
  hipLaunchKernelGGL(k_pack, dim3(blocks(27 * 16 * 32, 256)), dim3(256), 0, s, B.theta,
                     CORR_OFF_W3, 5, 32, 0, 16, B.w3, 32, B.w3t);
  return hipGetLastError();
}

template <typename T>
hipError_t corr_forward(const CorrBuffers& B, const CorrStats& st, int n, int batch, const T* U,
                        T* out, bool store_z, bool add_u, hipStream_t s) {
  const long long cells = (long long)batch * n * n * n;
  const unsigned conv_blocks = conv_grid(n, batch);
  hipLaunchKernelGGL((k_standardize<T>), dim3(blocks(cells, 256)), dim3(256), 0, s, U, n, cells, st,
                     B.x0);
  hipLaunchKernelGGL((k_conv<32, EPI_GELU, 9>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.x0, B.w1,
                     B.theta + CORR_OFF_B1, 32, n, (const float*)nullptr,
                     store_z ? B.z1 : (float*)nullptr, B.h1, (int)conv_blocks, ResArgs<float>{});
  hipLaunchKernelGGL((k_conv<32, EPI_GELU>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.h1, B.w2,
                     B.theta + CORR_OFF_B2, 32, n, (const float*)nullptr,
                     store_z ? B.z2 : (float*)nullptr, B.h2, (int)conv_blocks, ResArgs<float>{});
  if (out && add_u && !store_z) {
    // inference: the residual update in the last layer's epilogue (y is
    // not stored)
    ResArgs<T> ra{U, out, {}, (long long)n * n * n};
    for (int c = 0; c < 5; ++c) ra.scale[c] = st.scale[c];
    hipLaunchKernelGGL((k_conv<16, EPI_RESIDUAL, 27, T>), dim3(conv_wgs(conv_blocks)), dim3(256), 0,
                       s, B.h2, B.w3, B.theta + CORR_OFF_B3, 5, n, (const float*)nullptr,
                       (float*)nullptr, (unsigned short*)nullptr, (int)conv_blocks, ra);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_conv<16, EPI_LINEAR>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.h2, B.w3,
                     B.theta + CORR_OFF_B3, 5, n, (const float*)nullptr, B.y,
                     (unsigned short*)nullptr, (int)conv_blocks, ResArgs<float>{});
  if (out)
    hipLaunchKernelGGL((k_residual<T>), dim3(blocks(cells, 256)), dim3(256), 0, s, U, B.y, n, cells,
                       st, out, (int)add_u);
  return hipGetLastError();
}

template <typename T>
hipError_t corr_floor(const CorrBuffers& B, const T* U, T* out, int n, int batch, double gamma,
                      double frel, double fallback_frac, hipStream_t s) {
  const long long n3 = (long long)n * n * n, cells = batch * n3;
  const int bps = 64;
  hipLaunchKernelGGL((k_rho_p_partial<T>), dim3(batch * bps), dim3(256), 0, s, U, n3, gamma - 1.0,
                     bps, B.dpart);
  double* ref = B.dpart + 2 * batch * bps;
  hipLaunchKernelGGL(k_floor_ref, dim3(blocks(batch, 64)), dim3(64), 0, s, B.dpart, bps, batch, n3, frel, ref);
  hipLaunchKernelGGL((k_floor<T>), dim3(blocks(cells, 256)), dim3(256), 0, s, out, n3, cells,
                     gamma - 1.0, ref, B.cpart);
  hipLaunchKernelGGL(k_count_sum, dim3(1), dim3(256), 0, s, B.cpart, (int)blocks(cells, 256),
                     B.counters);
  hipLaunchKernelGGL((k_fallback<T>), dim3(blocks(5 * cells, 256)), dim3(256), 0, s, U, out,
                     5 * cells, fallback_frac * (double)cells, B.counters);
  return hipGetLastError();
}

template <typename T>
hipError_t corr_backward(const CorrBuffers& B, const CorrStats& st, int n, int batch, const T* U,
                         const T* tgt, const T* gup, T* gU, bool ident, hipStream_t s) {
  const long long cells = (long long)batch * n * n * n;
  const unsigned conv_blocks = conv_grid(n, batch);
  const unsigned lb = blocks(cells, 256);
  hipLaunchKernelGGL((k_loss<T>), dim3(lb), dim3(256), 0, s, U, B.y, tgt, gup, n, cells, st,
                     B.dpart, B.dy16, gU, (int)ident);
  hipLaunchKernelGGL(k_dsum, dim3(1), dim3(256), 0, s, B.dpart, (int)lb, B.loss);
  hipLaunchKernelGGL(k_pad16to32, dim3(lb), dim3(256), 0, s, B.dy16, cells, B.dy32);
  const int nblk = (int)(cells / (CTX * CTY * CTZ));
  const int nwg = corr_wgrad_groups(cells);
  // layer 3: dW3, db3; dH2 -> dZ2 = dH2 * GELU'(Z2)
  hipLaunchKernelGGL((k_wgrad<16>), dim3(nwg), dim3(256), 0, s, B.dy16, B.h2, n, nblk, B.wpart);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(28 * 16 * 32, 64)), dim3(256), 0, s, B.wpart,
                     16, nwg, 5, 32, 0, 0, B.grad + CORR_OFF_W3, B.grad + CORR_OFF_B3);
  hipLaunchKernelGGL((k_conv<32, EPI_GELU_BWD>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.dy32, B.w3t,
                     (const float*)nullptr, 0, n, B.z2, (float*)nullptr, B.dz2, (int)conv_blocks, ResArgs<float>{});
  // layer 2
  hipLaunchKernelGGL((k_wgrad<32>), dim3(nwg), dim3(256), 0, s, B.dz2, B.h1, n, nblk, B.wpart);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(28 * 32 * 32, 64)), dim3(256), 0, s,
                     B.wpart, 32, nwg, 32, 32, 0, 0, B.grad + CORR_OFF_W2, B.grad + CORR_OFF_B2);
  hipLaunchKernelGGL((k_conv<32, EPI_GELU_BWD>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.dz2, B.w2t,
                     (const float*)nullptr, 0, n, B.z1, (float*)nullptr, B.dz1, (int)conv_blocks, ResArgs<float>{});
  // layer 1
  hipLaunchKernelGGL((k_wgrad<32, true>), dim3(nwg), dim3(256), 0, s, B.dz1, B.x0, n, nblk,
                     B.wpart);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(28 * 32 * 32, 64)), dim3(256), 0, s,
                     B.wpart, 32, nwg, 32, 5, 1, 1, B.grad + CORR_OFF_W1, B.grad + CORR_OFF_B1);
  if (gU) {
    hipLaunchKernelGGL((k_conv<16, EPI_RAW>), dim3(conv_wgs(conv_blocks)), dim3(256), 0, s, B.dz1, B.w1t,
                       (const float*)nullptr, 0, n, (const float*)nullptr, B.gx,
                       (unsigned short*)nullptr, (int)conv_blocks, ResArgs<float>{});
    hipLaunchKernelGGL((k_input_grad<T>), dim3(lb), dim3(256), 0, s, B.gx, n, cells, st, gU);
  }
  return hipGetLastError();
}

hipError_t corr_unpack_input(const CorrBuffers& B, long long cells, unsigned short* x0,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_input, dim3(blocks(cells, 256)), dim3(256), 0, s, B.x0, cells, x0);
  return hipGetLastError();
}

hipError_t corr_zero_grad(const CorrBuffers& B, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks(CORR_NPARAM, 256)), dim3(256), 0, s, B.grad,
                     CORR_NPARAM, 0.0f);
  return hipGetLastError();
}

hipError_t corr_adam(const CorrBuffers& B, int it, float lr, hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, (float)it), c2 = 1.0f - powf(0.999f, (float)it);
  hipLaunchKernelGGL(k_adam, dim3(blocks(CORR_NPARAM, 256)), dim3(256), 0, s, B.theta, B.m, B.v,
                     B.grad, CORR_NPARAM, lr, c1, c2);
  return corr_pack_weights(B, s);
}

template <typename T>
hipError_t launch_block_average(const T* fine, int nf, int r, T* coarse, hipStream_t s) {
  const long long nc = nf / r;
  hipLaunchKernelGGL((k_block_average<T>), dim3(blocks(5 * nc * nc * nc, 256)), dim3(256), 0, s,
                     fine, nf, r, coarse);
  return hipGetLastError();
}

#define CORR_INSTANTIATE(T)                                                                       \
  template hipError_t corr_forward<T>(const CorrBuffers&, const CorrStats&, int, int, const T*, T*, \
                                      bool, bool, hipStream_t);                                   \
  template hipError_t corr_floor<T>(const CorrBuffers&, const T*, T*, int, int, double, double,    \
                                    double, hipStream_t);                                         \
  template hipError_t corr_backward<T>(const CorrBuffers&, const CorrStats&, int, int, const T*,  \
                                       const T*, const T*, T*, bool, hipStream_t);                \
  template hipError_t launch_block_average<T>(const T*, int, int, T*, hipStream_t);
CORR_INSTANTIATE(float)
CORR_INSTANTIATE(double)
#undef CORR_INSTANTIATE

}  // namespace mh
