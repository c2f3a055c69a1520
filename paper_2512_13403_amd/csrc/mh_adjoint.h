// mh_adjoint.h -- launchers of the adjoint kernels (internal to libmihydro).
#pragma once

#include <hip/hip_runtime.h>

#include "mg.h"
#include "mh_device.h"
#include "mh_launch.h"

namespace mh {

// scratch arrays of one adjoint step, carved from the adjoint workspace
template <typename T>
struct AdjointBuffers {
  T* Wacc;     // [5][N] primitive-variable adjoint accumulator
  T* wbar;     // [10][faces] face-state adjoints W^L_b, W^R_b of one axis, or
               // [20][faces] stencil contributions (run-time scheme)
  int* flags;  // [faces] minmod selections of the two slopes of each face
  T* accb;     // [3][N] adjoint of the gravitational acceleration
  T* phib;     // [N] adjoint of the potential
};

// limiters other than minmod / none, or a solver other than HLLC, take the
// run-time-scheme face kernel, whose face records are 20 values (wbar holds
// 20 x faces then, 10 x faces otherwise)
inline bool adj_runtime_scheme(int limiter, int riemann) {
  return riemann != RS_HLLC || (limiter != LIM_MINMOD && limiter != LIM_NONE);
}

template <typename T>
hipError_t adj_jtv(const AdjointBuffers<T>& B, const StageGeom& geom, int limiter, int riemann,
                   T gamma,
                   const double* h, const T* U, const T* v, T beta, T c0, const T* x0, T c1,
                   const T* x1, T c2, const T* x2, T* out, hipStream_t s);
template <typename T>
hipError_t adj_flux_corr_vjp(const T* v, const StageGeom& g, const double* h, double weight,
                             T* grad, hipStream_t s);
template <typename T>
hipError_t adj_force_kick_vjp(const T* rows, const T* tabx, int R, const StageGeom& g, T dt,
                              const T* lin, T* lout, hipStream_t s);
template <typename T>
hipError_t adj_cool_vjp(const T* U, long long N, T gm1, T dt, const CoolParams<T>& c, const T* lin,
                        T* lout, hipStream_t s);
// exact-cooling reverse followed by the forcing-kick reverse, one pass
template <typename T>
hipError_t adj_cool_force_vjp(const T* U, T gm1, T dt, const CoolParams<T>& c, const T* rows,
                              const T* tabx, int R, const StageGeom& g, const T* lin, T* lout,
                              hipStream_t s);
template <typename T>
hipError_t adj_gravity_vjp(const AdjointBuffers<T>& B, MGLayout& mgL, char* mgws,
                           const mh_physics_desc& p, const T* Ub, const T* phi, int n, double h,
                           T dt, const T* lin, T* lout, DevClock* clk, hipStream_t s);

}  // namespace mh
