// mg.h -- multigrid self-gravity on the device (internal to libmihydro).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mihydro.h"
#include "mh_device.h"

namespace mh {

constexpr int MG_MAX_LEVELS = 16;
constexpr int MG_PARTIALS = 1024;       // blocks of the two-stage reductions
constexpr int MG_COARSE_MAX_CELLS = 2048;
// a cycle that leaves more than this fraction of the residual has stalled at
// the round-off floor (the V- and W-cycles cut it by 0.07-0.3 otherwise)
constexpr double MG_STALL = 0.9;

struct MGLevel {
  int n;
  double h;
  size_t phi[2];  // ping-pong buffers of the Jacobi sweeps
  size_t F;       // right-hand side
};

// V-cycles replayed from captured HIP graphs: one V-cycle is ~60 small
// launches, so on a mid-size grid it is launch-bound when issued one kernel
// at a time.  A cache holds one executable graph per parity of the fine-level
// ping-pong buffer, valid for one workspace base address (the nodes hold raw
// pointers); it is captured on a private stream and launched on the caller's.
struct MGGraphCache {
  bool enabled = true;
  hipStream_t cs = nullptr;
  char* ws = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int cur_after[2] = {0, 0};
  void reset();     // drops the executable graphs (keeps the stream)
  void destroy();   // drops everything
};

struct MGLayout {
  int nlev = 0;
  MGLevel lev[MG_MAX_LEVELS];
  size_t partial = 0;  // MG_PARTIALS doubles
  int cur0 = 0;        // which fine-level phi buffer holds the solution
  MGGraphCache* graphs = nullptr;  // not owned; null: launch kernel by kernel
  // spectral solver (grav_solver = MH_GRAV_FFT): level 0 only, plus two
  // complex n^3 work arrays, the twiddles and the acceleration [3][n^3]
  int fft = 0;
  size_t fft_c0 = 0, fft_c1 = 0, fft_tw = 0, fft_acc = 0;
};

mh_status mg_validate(const mh_grid_desc* g, const mh_physics_desc* p, std::string& err);
size_t mg_layout(const mh_grid_desc* g, const mh_physics_desc* p, size_t off, size_t es,
                 MGLayout& L);
hipError_t mg_init(char* ws, const MGLayout& L, const mh_grid_desc* g, hipStream_t s);
size_t mg_phi_offset(const MGLayout& L);

// spectral gravity (fft_kernels.hip)
bool fft_size_ok(int n);
size_t fft_layout(int n, size_t off, size_t es, MGLayout& L);
template <typename T>
hipError_t fft_poisson(char* ws, MGLayout& L, double h, hipStream_t s);
template <typename T>
hipError_t fft_sources(char* ws, const MGLayout& L, const mh_grid_desc& g, bool cool, bool cfl,
                       const CoolParams<T>& cp, T* U, DevClock* clk, hipStream_t s);
template <typename T>
hipError_t fft_gravity_vjp(char* ws, MGLayout& L, double h, double G, const T* Ub, T dt,
                           const T* lin, T* lout, T* accb, hipStream_t s);

// Solves lap(phi) = 4 pi G (rho - <rho>) for the density of U (warm start from
// the previous solution), then applies the gravity kick and, when `last` (no
// later kernel in the step), the exact two-branch cooling (if on), the CFL
// reduction and the health check to U.  Synchronises once per V-cycle to test
// convergence.
template <typename T>
hipError_t mg_gravity_step(char* ws, MGLayout& L, const mh_grid_desc& g, const mh_physics_desc& p,
                           const CoolParams<T>& cool, T* U, DevClock* clk, bool last,
                           hipStream_t s);

// Pieces of the solve for the adjoint step: F = scale (x - <x>) on the fine
// level; the initial guess (a copy of phi0, or zero when phi0 is NULL); the
// V-cycle loop on the loaded F (cycles run returned in *cycles_out); and the
// gravity kick alone from the current fine-level potential.
template <typename T>
hipError_t mg_set_rhs(char* ws, MGLayout& L, const T* x, double scale, DevClock* clk,
                      hipStream_t s);
template <typename T>
hipError_t mg_set_guess(char* ws, MGLayout& L, const T* phi0, hipStream_t s);
template <typename T>
hipError_t mg_solve(char* ws, MGLayout& L, const mh_physics_desc& p, DevClock* clk, int* cycles_out,
                    hipStream_t s);
template <typename T>
hipError_t mg_kick(char* ws, MGLayout& L, const mh_grid_desc& g, T* U, DevClock* clk,
                   hipStream_t s);

}  // namespace mh
