// mh_launch.h -- kernel argument structs and launcher declarations used by the
// C-ABI layer (api.hip).  Internal to libmihydro.
#pragma once

#include <hip/hip_runtime.h>

#include "mh_device.h"

namespace mh {

struct StageGeom {
  int nx, ny, nz;
  int bc[3];
};

template <typename T>
struct StageArgs {
  const T* __restrict__ uin;  // stage input (read with halo)
  const T* un;                // U^n at the cell itself (stages 2 and 3; may alias uout)
  T* uout;                    // stage output
  DevClock* clk;
  const T* __restrict__ ou_rows;  // [nz][ny][R+1][3][P, Q] forcing row records
  const T* ou_tab[3];             // per axis [R+1][n_a][cos, sin] of 2 pi n (i + 1/2) / n_a
  int ou_modes;
  int ou_R;  // largest |n_a| among the modes (floor of kmax)
  int nx, ny, nz, bcx, bcy, bcz;
  long long ncell;
  T gamma, gm1, gm1inv, ihx, ihy, ihz;
  CoolParams<T> cool;
  int zc, nbx, nby, nbz, nb_per_xcd;
  int lim, rs;  // limiter and Riemann solver (read by the run-time-scheme kernel)
  T ca, cb;     // stages 2 and 3: out = ca U^n + cb (uin + dt L(uin))
  int epilogue; // stage 2: reduce the CFL speed and check health (0 when a
                // sources kernel follows and does both on the final state)
  const T* dflux;  // learned flux correction [5][N] (the +x, +y, +z faces of
                   // each cell), or null; run-time-scheme kernel only
};

struct OUArgs {
  DevClock* clk;
  double* ahat;    // [M][3][re, im]
  const int* nvec; // [M][3]
  void* coef;      // [M][3][re, im] in the state precision
  int f64;         // coef is double (1) or float (0)
  int nmodes;
  int every;
  unsigned long long seed;
  double tau, arms, zeta;
};

struct PrologueArgs {
  DevClock* clk;
  double* dt_log;
  int log_index;
  int f64;
  double dt_fixed;  // > 0: fixed dt
  double cfl;
  double ccool;     // > 0: CFL steps also <= ccool / max |Edot|/E_th
  double t_stop;
  int forcing;
  OUArgs ou;
  const double* dt_sched;  // device dt schedule, entry clk->sched_pos * sched_stride (or null)
  long long sched_stride;
};

template <typename T>
hipError_t launch_stage(int stage, int limiter, bool force, bool cool, StageArgs<T> a,
                        const StageGeom& g, hipStream_t s);
template <typename T>
hipError_t launch_force_rows(const T* coef, const int* nvec, int nmodes, const T* tabY,
                             const T* tabZ, int ny, int nz, int R, T* rows, hipStream_t s);
// cooling and the CFL / health epilogue of the last stage from its stored
// state after the forcing kick (a step that keeps that state)
template <typename T>
hipError_t launch_stage2_finish(bool cool, StageArgs<T> a, const T* ub, const StageGeom& g,
                                hipStream_t s);
template <typename T>
hipError_t launch_smax(const T* U, const StageGeom& g, T gamma, const double* ih, DevClock* clk,
                       hipStream_t s);
template <typename T>
hipError_t launch_cool_table(T* U, const StageGeom& g, T gamma, const double* ih,
                             const CoolTable<T>& c, DevClock* clk, hipStream_t s);
template <typename T>
hipError_t launch_cool_table_vjp(const T* U, long long N, T gamma, T dt, const CoolTable<T>& c,
                                 const T* lin, T* lout, hipStream_t s);
template <typename T>
hipError_t launch_cool_rate(const T* U, const StageGeom& g, T gamma, const CoolTable<T>& c,
                            DevClock* clk, hipStream_t s);
hipError_t launch_clock_reset_health(DevClock* clk, hipStream_t s);
hipError_t launch_clock_set(DevClock* clk, double t, long long step, hipStream_t s);
hipError_t launch_prologue(const PrologueArgs& a, hipStream_t s);
hipError_t launch_sched_reset(DevClock* clk, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
template <typename T>
hipError_t launch_adam(T* th, T* m, T* v, const T* g, long long count, double lr, double b1,
                       double b2, double eps, long long it, hipStream_t s);
hipError_t launch_ou_init(const OUArgs& a, hipStream_t s);

}  // namespace mh
