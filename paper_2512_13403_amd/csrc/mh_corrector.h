// mh_corrector.h -- corrector buffers and launchers (internal to libmihydro).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mh {

// canonical parameter order: W1[32][5][27], b1[32], W2[32][32][27], b2[32],
// W3[5][32][27], b3[5]
constexpr int CORR_OFF_W1 = 0;
constexpr int CORR_OFF_B1 = 4320;
constexpr int CORR_OFF_W2 = 4352;
constexpr int CORR_OFF_B2 = 32000;
constexpr int CORR_OFF_W3 = 32032;
constexpr int CORR_OFF_B3 = 36352;
constexpr int CORR_NPARAM = 36357;
constexpr int CORR_BLOCK_CELLS = 256;  // cells per convolution tile (16 x 4 x 4)
constexpr int CORR_WG_MAX = 512;       // persistent weight-gradient workgroups (two per CU)

// workgroups of the weight-gradient kernel (each writes a [27][32][32] partial)
inline int corr_wgrad_groups(long long cells) {
  const long long nb = cells / CORR_BLOCK_CELLS;
  return (int)(nb < CORR_WG_MAX ? nb : CORR_WG_MAX);
}

struct CorrStats {
  double mean[5], std[5], scale[5], lw[5];
};

struct CorrBuffers {
  float *theta, *m, *v, *grad;
  unsigned short *w1, *w2, *w3, *w1t, *w2t, *w3t;
  unsigned short *x0, *h1, *h2, *dy16, *dy32, *dz2, *dz1;
  float *z1, *z2, *y, *gx, *wpart;
  double *dpart, *loss;
  unsigned long long* counters;  // [floored cells, non-finite cells] of the last floor
  unsigned long long* cpart;     // their per-block parts
};

hipError_t corr_pack_weights(const CorrBuffers& B, hipStream_t s);
template <typename T>
hipError_t corr_forward(const CorrBuffers& B, const CorrStats& st, int n, int batch, const T* U,
                        T* out, bool store_z, bool add_u, hipStream_t s);
template <typename T>
hipError_t corr_floor(const CorrBuffers& B, const T* U, T* out, int n, int batch, double gamma,
                      double frel, double fallback_frac, hipStream_t s);
template <typename T>
hipError_t corr_backward(const CorrBuffers& B, const CorrStats& st, int n, int batch, const T* U,
                         const T* tgt, const T* gup, T* gU, bool ident, hipStream_t s);
hipError_t corr_zero_grad(const CorrBuffers& B, hipStream_t s);
// the network input in the unpacked layout [cells][32] (hi parts at 0..4, lo
// parts at 5..9) from the x-packed one the first layer reads
hipError_t corr_unpack_input(const CorrBuffers& B, long long cells, unsigned short* x0,
                             hipStream_t s);
hipError_t corr_adam(const CorrBuffers& B, int it, float lr, hipStream_t s);
template <typename T>
hipError_t launch_block_average(const T* fine, int nf, int r, T* coarse, hipStream_t s);

}  // namespace mh

// the batched corrected step of api.hip drives a corrector through these
typedef struct mh_corr mh_corr;
namespace mh {
hipStream_t corr_stream(const mh_corr* c);
// a state-mode corrector of this cube size, batch and dtype
bool corr_matches(const mh_corr* c, int n, int batch, int dtype);
// mh_corr_apply's correction of the batch U into out (forward, residual,
// floor, fallback), enqueued on stream s only; counts a fallback on the device
hipError_t corr_apply_enqueue(mh_corr* c, const void* U, void* out, hipStream_t s);
hipError_t corr_fallbacks_reset(mh_corr* c);
hipError_t corr_fallbacks_read(mh_corr* c, int64_t* count);

}  // namespace mh
