// corrector_api.hip -- C ABI of the learned state corrector (include/mihydro.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mihydro.h"
#include "mh_corrector.h"

using namespace mh;

namespace {

constexpr size_t CALIGN = 256;
inline size_t calign(size_t x) { return (x + CALIGN - 1) & ~(CALIGN - 1); }

struct CorrLayout {
  size_t theta, m, v, grad, w1, w2, w3, w1t, w2t, w3t, x0, z1, h1, z2, h2, y, gx, dy16, dy32, dz2,
      dz1;
  size_t wpart, dpart, loss, counters, cpart, total;
};

CorrLayout corr_layout(const mh_corr_desc* d) {
  CorrLayout L{};
  const size_t cells = (size_t)d->batch * d->n * d->n * d->n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = calign(off + bytes);
    return o;
  };
  const size_t P = CORR_NPARAM * sizeof(float);
  L.theta = take(P);
  L.m = take(P);
  L.v = take(P);
  L.grad = take(P);
  L.w1 = take(27 * 32 * 32 * 2);
  L.w2 = take(27 * 32 * 32 * 2);
  L.w3 = take(27 * 16 * 32 * 2);
  L.w1t = take(27 * 16 * 32 * 2);
  L.w2t = take(27 * 32 * 32 * 2);
  L.w3t = take(27 * 32 * 32 * 2);
  L.x0 = take(cells * 32 * 2);
  L.z1 = take(cells * 32 * 4);
  L.h1 = take(cells * 32 * 2);
  L.z2 = take(cells * 32 * 4);
  L.h2 = take(cells * 32 * 2);
  L.y = take(cells * 16 * 4);
  L.gx = take(cells * 16 * 4);
  L.dy16 = take(cells * 16 * 2);
  L.dy32 = take(cells * 32 * 2);
  L.dz2 = take(cells * 32 * 2);
  L.dz1 = take(cells * 32 * 2);
  L.wpart = take((size_t)28 * corr_wgrad_groups((long long)cells) * 32 * 32 * 4);
  // per-block partial sums, or the floor partials (64 blocks per sample) and
  // the two floor values of each sample after them
  const size_t nd = std::max((cells + 255) / 256, (size_t)d->batch * (64 * 2 + 2));
  L.dpart = take(nd * sizeof(double));
  L.loss = take(sizeof(double));
  // [floored cells, non-finite cells] of the last floor, then the number of
  // fallbacks counted by the batched corrected step
  L.counters = take(3 * sizeof(unsigned long long));
  // per-block floored / non-finite counts of the positivity floor
  L.cpart = take(2 * ((cells + 255) / 256) * sizeof(unsigned long long));
  L.total = off;
  return L;
}

mh_status corr_validate(const mh_corr_desc* d) {
  if (!d) return MH_E_INVALID;
  if (d->n < 16 || d->n % 16 != 0 || d->batch < 1) return MH_E_SHAPE;
  if (d->dtype != MH_F32 && d->dtype != MH_F64) return MH_E_DTYPE;
  if (!(d->gamma > 1.0)) return MH_E_INVALID;
  for (int c = 0; c < 5; ++c)
    if (!(d->std[c] > 0.0) || !std::isfinite(d->mean[c]) || !std::isfinite(d->scale[c]))
      return MH_E_INVALID;
  if (!(d->floor_rel >= 0.0) || !(d->fallback_frac >= 0.0)) return MH_E_INVALID;
  if (d->mode != MH_CORR_STATE && d->mode != MH_CORR_FLUX) return MH_E_UNSUPPORTED;
  return MH_OK;
}

__global__ void k_zero_bytes(unsigned char* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

struct mh_corr {
  mh_corr_desc d;
  hipStream_t stream;
  char* ws;
  CorrLayout L;
  CorrBuffers B;
  CorrStats st;
  int it = 0;
  long long cells() const { return (long long)d.batch * d.n * d.n * d.n; }
};

#define MH_CHK(call)                           \
  do {                                         \
    if ((call) != hipSuccess) return MH_E_DEVICE; \
  } while (0)

extern "C" mh_status mh_corr_query_workspace(const mh_corr_desc* d, size_t* bytes) {
  if (!bytes) return MH_E_INVALID;
  mh_status s = corr_validate(d);
  if (s != MH_OK) return s;
  *bytes = corr_layout(d).total;
  return MH_OK;
}

extern "C" mh_status mh_corr_init(const mh_corr_desc* d, void* workspace, size_t bytes,
                                  void* stream, mh_corr** out) {
  if (!out) return MH_E_INVALID;
  *out = nullptr;
  mh_status s = corr_validate(d);
  if (s != MH_OK) return s;
  CorrLayout L = corr_layout(d);
  if (!workspace || bytes < L.total || ((uintptr_t)workspace % CALIGN) != 0) return MH_E_WORKSPACE;
  mh_corr* c = new mh_corr();
  c->d = *d;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->L = L;
  char* w = c->ws;
  auto F = [&](size_t o) { return reinterpret_cast<float*>(w + o); };
  auto H = [&](size_t o) { return reinterpret_cast<unsigned short*>(w + o); };
  c->B = CorrBuffers{F(L.theta), F(L.m), F(L.v), F(L.grad), H(L.w1), H(L.w2), H(L.w3), H(L.w1t),
                     H(L.w2t), H(L.w3t), H(L.x0), H(L.h1), H(L.h2), H(L.dy16), H(L.dy32),
                     H(L.dz2), H(L.dz1), F(L.z1), F(L.z2), F(L.y), F(L.gx), F(L.wpart),
                     reinterpret_cast<double*>(w + L.dpart), reinterpret_cast<double*>(w + L.loss),
                     reinterpret_cast<unsigned long long*>(w + L.counters),
                     reinterpret_cast<unsigned long long*>(w + L.cpart)};
  for (int k = 0; k < 5; ++k) {
    c->st.mean[k] = d->mean[k];
    c->st.std[k] = d->std[k];
    c->st.scale[k] = d->scale[k];
    c->st.lw[k] = d->loss_w[k];
  }
  // parameters, moments and weight operands start at zero (padded weight
  // rows must be zero: they meet zero activations in the products)
  const size_t zero_span = L.x0;  // theta .. w3t are laid out first
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((zero_span + 255) / 256)), dim3(256), 0,
                     c->stream, (unsigned char*)w, zero_span);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return MH_E_DEVICE;
  }
  *out = c;
  return MH_OK;
}

extern "C" mh_status mh_corr_set_params(mh_corr* c, const float* theta, int where) {
  if (!c || !theta || (where != MH_HOST && where != MH_DEVICE)) return MH_E_INVALID;
  MH_CHK(hipMemcpyAsync(c->B.theta, theta, CORR_NPARAM * sizeof(float),
                        where == MH_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                        c->stream));
  const size_t mom = c->L.grad - c->L.m;  // m and v
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((mom + 255) / 256)), dim3(256), 0, c->stream,
                     (unsigned char*)c->B.m, mom);
  MH_CHK(hipGetLastError());
  MH_CHK(corr_pack_weights(c->B, c->stream));
  if (where == MH_HOST) MH_CHK(hipStreamSynchronize(c->stream));
  c->it = 0;
  return MH_OK;
}

extern "C" mh_status mh_corr_get_params(mh_corr* c, float* theta, int where) {
  if (!c || !theta || (where != MH_HOST && where != MH_DEVICE)) return MH_E_INVALID;
  MH_CHK(hipMemcpyAsync(theta, c->B.theta, CORR_NPARAM * sizeof(float),
                        where == MH_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        c->stream));
  if (where == MH_HOST) MH_CHK(hipStreamSynchronize(c->stream));
  return MH_OK;
}

template <typename T>
static mh_status apply_impl(mh_corr* c, const T* U, T* out, int64_t* floored, int32_t* fell) {
  if (c->d.mode == MH_CORR_FLUX) {
    MH_CHK(corr_forward<T>(c->B, c->st, c->d.n, c->d.batch, U, out, false, false, c->stream));
    if (floored) *floored = 0;
    if (fell) *fell = 0;
    return MH_OK;
  }
  MH_CHK(corr_forward<T>(c->B, c->st, c->d.n, c->d.batch, U, out, false, true, c->stream));
  MH_CHK(corr_floor<T>(c->B, U, out, c->d.n, c->d.batch, c->d.gamma, c->d.floor_rel,
                       c->d.fallback_frac, c->stream));
  if (floored || fell) {
    unsigned long long cnt[2];
    MH_CHK(hipMemcpyAsync(cnt, c->B.counters, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    MH_CHK(hipStreamSynchronize(c->stream));
    if (floored) *floored = (int64_t)cnt[0];
    if (fell)
      *fell = (cnt[1] > 0 || (double)cnt[0] > c->d.fallback_frac * (double)c->cells()) ? 1 : 0;
  }
  return MH_OK;
}

namespace {
// counters[2] += 1 when the floor just run made the batch fall back
__global__ void k_fallback_count(unsigned long long* counters, double limit) {
  if (threadIdx.x == 0 && (counters[1] > 0 || (double)counters[0] > limit)) counters[2] += 1;
}

__global__ void k_fallback_reset(unsigned long long* counters) {
  if (threadIdx.x == 0) counters[2] = 0;
}
}  // namespace

namespace mh {

hipStream_t corr_stream(const mh_corr* c) { return c->stream; }

bool corr_matches(const mh_corr* c, int n, int batch, int dtype) {
  return c->d.mode == MH_CORR_STATE && c->d.n == n && c->d.batch == batch && c->d.dtype == dtype;
}

hipError_t corr_apply_enqueue(mh_corr* c, const void* U, void* out, hipStream_t s) {
  hipError_t e;
  if (c->d.dtype == MH_F64) {
    e = corr_forward<double>(c->B, c->st, c->d.n, c->d.batch, (const double*)U, (double*)out,
                             false, true, s);
    if (e == hipSuccess)
      e = corr_floor<double>(c->B, (const double*)U, (double*)out, c->d.n, c->d.batch,
                             c->d.gamma, c->d.floor_rel, c->d.fallback_frac, s);
  } else {
    e = corr_forward<float>(c->B, c->st, c->d.n, c->d.batch, (const float*)U, (float*)out,
                            false, true, s);
    if (e == hipSuccess)
      e = corr_floor<float>(c->B, (const float*)U, (float*)out, c->d.n, c->d.batch, c->d.gamma,
                            c->d.floor_rel, c->d.fallback_frac, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fallback_count, dim3(1), dim3(64), 0, s, c->B.counters,
                     c->d.fallback_frac * (double)c->cells());
  return hipGetLastError();
}

hipError_t corr_fallbacks_reset(mh_corr* c) {
  hipLaunchKernelGGL(k_fallback_reset, dim3(1), dim3(64), 0, c->stream, c->B.counters);
  return hipGetLastError();
}

hipError_t corr_fallbacks_read(mh_corr* c, int64_t* count) {
  unsigned long long v = 0;
  hipError_t e = hipMemcpyAsync(&v, c->B.counters + 2, sizeof v, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  *count = (int64_t)v;
  return e;
}

}  // namespace mh

extern "C" mh_status mh_corr_apply(mh_corr* c, const void* U, void* U_out, int64_t* floored,
                                   int32_t* fell_back) {
  if (!c || !U || !U_out || U == U_out) return MH_E_INVALID;
  if (c->d.dtype == MH_F64)
    return apply_impl<double>(c, (const double*)U, (double*)U_out, floored, fell_back);
  return apply_impl<float>(c, (const float*)U, (float*)U_out, floored, fell_back);
}

template <typename T>
static mh_status backward_impl(mh_corr* c, const T* U, const T* tgt, const T* gup, double* loss,
                               T* gU) {
  MH_CHK(corr_forward<T>(c->B, c->st, c->d.n, c->d.batch, U, (T*)nullptr, true, true, c->stream));
  MH_CHK(corr_backward<T>(c->B, c->st, c->d.n, c->d.batch, U, tgt, gup, gU,
                          c->d.mode == MH_CORR_STATE, c->stream));
  if (loss && tgt) {
    double l;
    MH_CHK(hipMemcpyAsync(&l, c->B.loss, sizeof l, hipMemcpyDeviceToHost, c->stream));
    MH_CHK(hipStreamSynchronize(c->stream));
    *loss = l / (double)c->cells();
  }
  return MH_OK;
}

static mh_status backward_any(mh_corr* c, const void* U, const void* tgt, const void* gup,
                              double* loss, void* gU) {
  if (c->d.dtype == MH_F64)
    return backward_impl<double>(c, (const double*)U, (const double*)tgt, (const double*)gup, loss,
                                 (double*)gU);
  return backward_impl<float>(c, (const float*)U, (const float*)tgt, (const float*)gup, loss,
                              (float*)gU);
}

extern "C" mh_status mh_corr_zero_grad(mh_corr* c) {
  if (!c) return MH_E_INVALID;
  MH_CHK(corr_zero_grad(c->B, c->stream));
  return MH_OK;
}

extern "C" mh_status mh_corr_backward(mh_corr* c, const void* U, const void* target,
                                      const void* gUc, double* loss, void* gU) {
  if (!c || !U || (!target && !gUc) || (gU && (gU == U || gU == gUc))) return MH_E_INVALID;
  if (c->d.mode == MH_CORR_FLUX && target) return MH_E_INVALID;
  return backward_any(c, U, target, gUc, loss, gU);
}

extern "C" mh_status mh_corr_adam_step(mh_corr* c, float lr) {
  if (!c || !(lr >= 0.0f)) return MH_E_INVALID;
  c->it += 1;
  MH_CHK(corr_adam(c->B, c->it, lr, c->stream));
  return MH_OK;
}

extern "C" mh_status mh_corr_get_grad(mh_corr* c, float* grad, int where) {
  if (!c || !grad || (where != MH_HOST && where != MH_DEVICE)) return MH_E_INVALID;
  MH_CHK(hipMemcpyAsync(grad, c->B.grad, CORR_NPARAM * sizeof(float),
                        where == MH_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        c->stream));
  if (where == MH_HOST) MH_CHK(hipStreamSynchronize(c->stream));
  return MH_OK;
}

extern "C" mh_status mh_corr_loss_grad(mh_corr* c, const void* U, const void* target, double* loss,
                                       float* grad, int where) {
  if (!c || !U || !target || (grad && where != MH_HOST && where != MH_DEVICE)) return MH_E_INVALID;
  if (c->d.mode == MH_CORR_FLUX) return MH_E_INVALID;
  MH_CHK(corr_zero_grad(c->B, c->stream));
  mh_status s = backward_any(c, U, target, nullptr, loss, nullptr);
  if (s != MH_OK) return s;
  if (grad) return mh_corr_get_grad(c, grad, where);
  return MH_OK;
}

extern "C" mh_status mh_corr_train_step(mh_corr* c, const void* U, const void* target, float lr,
                                        double* loss) {
  if (!c || !U || !target || !(lr >= 0.0f)) return MH_E_INVALID;
  mh_status s = mh_corr_loss_grad(c, U, target, loss, nullptr, MH_DEVICE);
  if (s != MH_OK) return s;
  return mh_corr_adam_step(c, lr);
}

extern "C" mh_status mh_corr_get_activation(mh_corr* c, int which, void* dst, int where) {
  if (!c || !dst || which < 0 || which > 9 || (where != MH_HOST && where != MH_DEVICE))
    return MH_E_INVALID;
  const size_t cells = (size_t)c->cells();
  if (which == 0) {
    // the stored input holds the three x neighbours of each cell: extract the
    // cell's own two parts
    if (where == MH_DEVICE) {
      MH_CHK(corr_unpack_input(c->B, (long long)cells, (unsigned short*)dst, c->stream));
      return MH_OK;
    }
    std::vector<unsigned short> xp(cells * 32);
    MH_CHK(hipMemcpyAsync(xp.data(), c->B.x0, cells * 32 * 2, hipMemcpyDeviceToHost, c->stream));
    MH_CHK(hipStreamSynchronize(c->stream));
    unsigned short* out = (unsigned short*)dst;
    for (size_t q = 0; q < cells; ++q)
      for (int k = 0; k < 32; ++k) out[q * 32 + k] = k < 10 ? xp[q * 32 + 10 + k] : 0;
    return MH_OK;
  }
  const void* src = nullptr;
  size_t bytes = 0;
  switch (which) {
    case 1: src = c->B.z1; bytes = cells * 32 * 4; break;
    case 2: src = c->B.h1; bytes = cells * 32 * 2; break;
    case 3: src = c->B.z2; bytes = cells * 32 * 4; break;
    case 4: src = c->B.h2; bytes = cells * 32 * 2; break;
    case 5: src = c->B.y; bytes = cells * 16 * 4; break;
    case 6: src = c->B.dy16; bytes = cells * 16 * 2; break;
    case 7: src = c->B.dz2; bytes = cells * 32 * 2; break;
    case 8: src = c->B.dz1; bytes = cells * 32 * 2; break;
    default: src = c->B.gx; bytes = cells * 16 * 4; break;
  }
  MH_CHK(hipMemcpyAsync(dst, src, bytes,
                        where == MH_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        c->stream));
  if (where == MH_HOST) MH_CHK(hipStreamSynchronize(c->stream));
  return MH_OK;
}

extern "C" void mh_corr_destroy(mh_corr* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

extern "C" mh_status mh_block_average(const void* fine, int32_t nf, int32_t r, void* coarse,
                                      int32_t dtype, void* stream) {
  if (!fine || !coarse || r < 1 || nf < r || nf % r != 0) return MH_E_INVALID;
  if (dtype == MH_F64)
    MH_CHK(launch_block_average<double>((const double*)fine, nf, r, (double*)coarse,
                                        (hipStream_t)stream));
  else if (dtype == MH_F32)
    MH_CHK(launch_block_average<float>((const float*)fine, nf, r, (float*)coarse,
                                       (hipStream_t)stream));
  else
    return MH_E_DTYPE;
  return MH_OK;
}
