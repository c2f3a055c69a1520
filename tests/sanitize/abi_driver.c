/*
 * abi_driver.c -- drives the host-side argument validation of the C ABI
 * (include/mihydro.h) under the address and undefined-behaviour sanitizers,
 * without a GPU: workspace queries for valid and invalid descriptors, and
 * every entry point with null handles or pointers, which must come back with
 * the documented status before touching a device.  Exit status 0 when every
 * status is the expected one and no sanitizer reported.  Test infrastructure
 * only.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/mihydro.h"

static int fails = 0;
#define EXPECT(call, status)                                                        \
  do {                                                                              \
    mh_status s_ = (call);                                                          \
    if (s_ != (status)) {                                                           \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, #call, \
              (int)s_, (int)(status));                                              \
      ++fails;                                                                      \
    }                                                                               \
  } while (0)

static mh_grid_desc grid(int nx, int ny, int nz, int dtype) {
  mh_grid_desc g;
  memset(&g, 0, sizeof g);
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
  g.h[0] = 1.0 / nx; g.h[1] = 1.0 / ny; g.h[2] = 1.0 / nz;
  g.dtype = dtype; g.gamma = 5.0 / 3.0; g.cfl = 0.4;
  return g;
}

static mh_physics_desc physics(unsigned flags) {
  mh_physics_desc p;
  memset(&p, 0, sizeof p);
  p.flags = flags;
  p.ou_every = 1; p.ou_tau = 0.5; p.ou_arms = 1.0; p.ou_zeta = 1.0; p.ou_kmin = 1.0;
  p.ou_kmax = 2.0;
  p.cool_lambda0 = 0.3; p.cool_tc = 1e-2; p.cool_ts = 1e-3; p.cool_tfloor = 1e-4;
  p.grav_G = 1.0; p.mg_pre = 2; p.mg_post = 2; p.mg_max_cycles = 20; p.mg_coarsest = 4;
  p.mg_tol = 1e-10; p.mg_coarse_sweeps = 200;
  p.cool_nsub_max = 100; p.cool_frac = 0.1;
  return p;
}

int main(void) {
  size_t b = 0;
  /* workspace queries */
  mh_grid_desc g = grid(64, 32, 16, MH_F32);
  mh_physics_desc p = physics(MH_SRC_FORCING | MH_SRC_COOLING);
  EXPECT(mh_query_workspace(&g, &p, &b), MH_OK);
  if (b < (size_t)2 * 5 * 64 * 32 * 16 * 4) ++fails;
  mh_grid_desc g64 = grid(32, 32, 32, MH_F64);
  mh_physics_desc pg = physics(MH_SRC_GRAVITY);
  EXPECT(mh_query_workspace(&g64, &pg, &b), MH_OK);
  pg.grav_solver = MH_GRAV_FFT;
  EXPECT(mh_query_workspace(&g64, &pg, &b), MH_OK);
  EXPECT(mh_query_workspace(NULL, &p, &b), MH_E_INVALID);
  EXPECT(mh_query_workspace(&g, NULL, &b), MH_E_INVALID);
  EXPECT(mh_query_workspace(&g, &p, NULL), MH_E_INVALID);
  {
    mh_grid_desc x = g; x.dtype = 7;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_DTYPE);
    x = g; x.n[0] = 0;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_INVALID);
    x = g; x.h[1] = -1.0;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_INVALID);
    x = g; x.gamma = NAN;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_INVALID);
    x = g; x.limiter = 9;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_UNSUPPORTED);
    x = g; x.integrator = -1;
    EXPECT(mh_query_workspace(&x, &p, &b), MH_E_UNSUPPORTED);
    mh_physics_desc y = p; y.flags = 64;
    EXPECT(mh_query_workspace(&g, &y, &b), MH_E_INVALID);
    y = physics(MH_SRC_COOLING); y.cool_model = MH_COOL_TABLE; y.cool_ntab = 1000;
    mh_status s = mh_query_workspace(&g, &y, &b);
    if (s == MH_OK) ++fails;
    y = physics(MH_SRC_GRAVITY); y.mg_smoother = 5;
    s = mh_query_workspace(&g64, &y, &b);
    if (s == MH_OK) ++fails;
  }
  /* corrector and transform queries */
  mh_corr_desc cd;
  memset(&cd, 0, sizeof cd);
  cd.n = 32; cd.batch = 2; cd.dtype = MH_F32; cd.gamma = 5.0 / 3.0;
  for (int c = 0; c < 5; ++c) { cd.std[c] = 1.0; cd.scale[c] = 1e-2; cd.loss_w[c] = 1.0; }
  cd.floor_rel = 1e-6; cd.fallback_frac = 1e-3;
  EXPECT(mh_corr_query_workspace(&cd, &b), MH_OK);
  EXPECT(mh_corr_query_workspace(NULL, &b), MH_E_INVALID);
  {
    mh_corr_desc x = cd; x.n = 20;
    EXPECT(mh_corr_query_workspace(&x, &b), MH_E_SHAPE);
    x = cd; x.std[2] = 0.0;
    EXPECT(mh_corr_query_workspace(&x, &b), MH_E_INVALID);
  }
  EXPECT(mh_fft3_query_workspace(64, MH_F64, &b), MH_OK);
  EXPECT(mh_fft3_query_workspace(48, MH_F32, &b), MH_E_SHAPE);
  EXPECT(mh_fft3_query_workspace(64, 3, &b), MH_E_DTYPE);
  EXPECT(mh_fft3_query_workspace(64, MH_F32, NULL), MH_E_INVALID);
  /* null handles and pointers */
  double d = 0.0;
  int64_t i64 = 0;
  int32_t i32 = 0;
  float f = 0.0f;
  EXPECT(mh_init(&g, &p, NULL, 0, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_set_state(NULL, &d, MH_HOST), MH_E_INVALID);
  EXPECT(mh_get_state(NULL, &d, MH_HOST), MH_E_INVALID);
  EXPECT(mh_step(NULL, 1, 0.0, INFINITY, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_get_clock(NULL, &d, &i64), MH_E_INVALID);
  EXPECT(mh_set_clock(NULL, 0.0, 0), MH_E_INVALID);
  EXPECT(mh_get_ou_state(NULL, &i32, &d), MH_E_INVALID);
  EXPECT(mh_set_ou_state(NULL, &d), MH_E_INVALID);
  EXPECT(mh_check(NULL, &i64, &i64), MH_E_INVALID);
  EXPECT(mh_last_mg_cycles(NULL, &i32), MH_E_INVALID);
  EXPECT(mh_get_potential(NULL, &d, MH_HOST), MH_E_INVALID);
  EXPECT(mh_set_potential(NULL, &d, MH_HOST), MH_E_INVALID);
  EXPECT(mh_query_adjoint_workspace(NULL, &b), MH_E_INVALID);
  EXPECT(mh_adjoint_step(NULL, NULL, 0, NULL, 0.1, 0, NULL, NULL, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_set_timing(NULL, 1), MH_E_INVALID);
  EXPECT(mh_get_timing(NULL, &d, &i64), MH_E_INVALID);
  EXPECT(mh_set_flux_correction(NULL, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_set_graphs(NULL, 1), MH_E_INVALID);
  EXPECT(mh_corr_init(&cd, NULL, 0, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_corr_set_params(NULL, &f, MH_HOST), MH_E_INVALID);
  EXPECT(mh_corr_get_params(NULL, &f, MH_HOST), MH_E_INVALID);
  EXPECT(mh_corr_apply(NULL, &d, &d, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_corr_loss_grad(NULL, &d, &d, &d, &f, MH_HOST), MH_E_INVALID);
  EXPECT(mh_corr_train_step(NULL, &d, &d, 1e-3f, &d), MH_E_INVALID);
  EXPECT(mh_corr_zero_grad(NULL), MH_E_INVALID);
  EXPECT(mh_corr_backward(NULL, &d, &d, NULL, NULL, NULL), MH_E_INVALID);
  EXPECT(mh_corr_adam_step(NULL, 1e-3f), MH_E_INVALID);
  EXPECT(mh_corr_get_grad(NULL, &f, MH_HOST), MH_E_INVALID);
  EXPECT(mh_corr_get_activation(NULL, 0, &f, MH_HOST), MH_E_INVALID);
  EXPECT(mh_step_corrected(NULL, 1, NULL, NULL, 1, NULL, 0, NULL), MH_E_INVALID);
  EXPECT(mh_block_average(NULL, 8, 2, NULL, MH_F32, NULL), MH_E_INVALID);
  EXPECT(mh_fft3(NULL, 8, MH_F32, 0, NULL, 0, NULL), MH_E_INVALID);
  EXPECT(mh_fft3_noalloc(NULL, 8, MH_F32, 0, NULL), MH_E_INVALID);
  EXPECT(mh_fft3_noalloc(&d, 12, MH_F32, 0, NULL), MH_E_SHAPE);
  if (mh_last_error(NULL) == NULL) ++fails;
  mh_destroy(NULL);
  mh_corr_destroy(NULL);
  if (fails) {
    fprintf(stderr, "abi driver: %d failures\n", fails);
    return 1;
  }
  puts("abi driver: ok");
  return 0;
}
