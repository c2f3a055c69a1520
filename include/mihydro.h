/*
 * mihydro.h -- C ABI of libmihydro.so, an MI355X (gfx950) implementation of
 * the finite-volume step of "diffhydro" (Horowitz, Lukic, Nagamine & Oku,
 * arXiv 2512.13403): MUSCL/PLM reconstruction on primitive variables with a
 * minmod limiter (App. A.1), HLLC fluxes with Davis wave speeds (App. A.2),
 * unsplit conservative differencing and two-stage RK2 (App. A.3), the CFL
 * step (App. A.4), and operator-split sources after each step: OU turbulent
 * forcing (Sec. 3.1.1), multigrid self-gravity (Sec. 6, 6.2) and optically
 * thin cooling integrated exactly per cell (Sec. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout: U is a dense array [5][nz][ny][nx] (x fastest) of the
 *   conserved fields (rho, m_x, m_y, m_z, E), the state vector of the paper's
 *   Sec. 2.1 listing, in the precision chosen by mh_grid_desc.dtype (float or
 *   double).
 * Memory: the caller owns all device memory.  The library only owns its host
 *   context.  The workspace passed to mh_init must stay valid (and untouched
 *   by the caller) until mh_destroy; it holds the state, the stage buffer, the
 *   device clock, the OU mode state and the multigrid hierarchy.
 * Streams: every call enqueues its work on the HIP stream given to mh_init
 *   and returns without waiting, except where stated ("synchronises").
 * Errors: every call returns an mh_status; nothing throws across the ABI.  On
 *   an error the context keeps its previous state unless stated otherwise, and
 *   mh_last_error() returns a message (valid until the next call on ctx).
 * Threads: a context must not be used from two host threads at once.
 */
#ifndef MIHYDRO_H
#define MIHYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mh_status {
  MH_OK = 0,
  MH_E_INVALID = 1,     /* null pointer, bad enum, non-positive size/spacing */
  MH_E_SHAPE = 2,       /* grid shape not supported by the requested physics */
  MH_E_DTYPE = 3,       /* unknown precision */
  MH_E_DEVICE = 4,      /* a HIP call failed; mh_last_error has its text */
  MH_E_NONFINITE = 5,   /* non-finite value or rho <= 0 or P <= 0 detected */
  MH_E_UNSUPPORTED = 6, /* valid option that this build does not implement */
  MH_E_WORKSPACE = 7    /* workspace too small or misaligned */
} mh_status;

enum { MH_BC_PERIODIC = 0, MH_BC_OUTFLOW = 1 };
enum { MH_F32 = 0, MH_F64 = 1 };
enum { MH_LIM_MINMOD = 0, MH_LIM_NONE = 1, MH_LIM_VANLEER = 2, MH_LIM_MC = 3, MH_LIM_SUPERBEE = 4 };
enum { MH_RS_HLLC = 0, MH_RS_HLL = 1, MH_RS_RUSANOV = 2 };
enum { MH_RK_SSP2 = 0, MH_RK_SSP3 = 1, MH_RK_EULER = 2 };
enum { MH_MG_V = 0, MH_MG_W = 1 };
enum { MH_SMOOTH_JACOBI = 0, MH_SMOOTH_RBGS = 1 };
enum { MH_GRAV_MG = 0, MH_GRAV_FFT = 1 };
enum { MH_COOL_EXACT2 = 0, MH_COOL_TABLE = 1 };
enum { MH_COOLINT_TRAPEZOID = 0, MH_COOLINT_SUBCYCLE = 1, MH_COOLINT_AUTO = 2 };
#define MH_COOL_TABMAX 64
enum { MH_SRC_COOLING = 1u, MH_SRC_FORCING = 2u, MH_SRC_GRAVITY = 4u };
enum { MH_HOST = 0, MH_DEVICE = 1 };

/* Grid and scheme.
 * n[3]    cells along x, y, z (each >= 1; at most 2^31 cells in all, and one
 *         x-y plane of a field below 4 GiB, else MH_E_SHAPE).
 * bc[3]   MH_BC_PERIODIC (wrap) or MH_BC_OUTFLOW (zero-gradient copy of the
 *         edge cell) per axis.
 * h[3]    cell spacing per axis (> 0).
 * dtype   MH_F32 or MH_F64: storage and arithmetic precision of the state.
 * limiter MH_LIM_MINMOD (App. A.1; a tie |a| = |b| takes the forward
 *         difference), MH_LIM_NONE (piecewise constant), MH_LIM_VANLEER
 *         (2ab/(a+b)), MH_LIM_MC (monotonised central) or MH_LIM_SUPERBEE,
 *         each 0 when the two differences disagree in sign (App. A.1 lists
 *         the family).
 * riemann MH_RS_HLLC (App. A.2), MH_RS_HLL or MH_RS_RUSANOV, all with the
 *         Davis wave-speed estimates.  minmod or none with HLLC run the
 *         specialised kernels; the other combinations a kernel that selects
 *         limiter and solver at run time (also in the adjoint step).
 * integrator  the explicit Runge-Kutta update (App. A.3): MH_RK_SSP2 (the
 *         two-stage Heun / SSP-RK2, the default), MH_RK_SSP3 (three-stage
 *         SSPRK3; the workspace holds one more state) or MH_RK_EULER
 *         (first order, for testing; one extra state copy per step).  The
 *         sources follow the full update in every case.
 * gamma   adiabatic index (> 1).
 * cfl     Courant number C of dt = C min_a dx_a / (|v_a| + c_s) (App. A.4). */
typedef struct mh_grid_desc {
  int32_t n[3];
  int32_t bc[3];
  double h[3];
  int32_t dtype;
  int32_t limiter;
  int32_t riemann;
  int32_t integrator;
  double gamma;
  double cfl;
} mh_grid_desc;

/* Source terms, applied after each Runge-Kutta update in the order forcing ->
 * gravity -> cooling, each on the state left by the previous one.
 * flags           OR of MH_SRC_*.
 * cool_*          cooling in code units with T = P/rho.  cool_model
 *                 MH_COOL_EXACT2 (the default): the synthetic two-branch curve
 *                 Lambda = lambda0 (T/tc)^(1/2) for T >= tc,
 *                 Lambda = lambda0 exp((T - tc)/ts) for T < tc;
 *                 dT/dt = -(gamma-1) rho Lambda(T) is integrated exactly over
 *                 dt, then T is floored at tfloor (Sec. 4 and 4.3).
 *                 MH_COOL_TABLE: the paper's model (Sec. 4.1-4.3) with
 *                 dE_th/dt = rho Gamma - rho^2 Lambda, Lambda = L1 T^a1 +
 *                 L2 T^a2 and Gamma = heat below tc, Lambda from log-log
 *                 interpolation of the cool_ntab (2..64) points (log10 T,
 *                 log10 Lambda) at and above tc (flat beyond the ends), no
 *                 heating; integrated by cool_integrator (trapezoid, subcycled
 *                 with N = ceil(dt |Edot| / (frac E_th)) <= nsub_max
 *                 substeps each changing E_th by at most frac, or auto:
 *                 trapezoid when dt |Edot| <= frac E_th), E_th floored at
 *                 rho tfloor/(gamma-1).  cool_ccool > 0 (tabulated model
 *                 only) limits CFL steps to ccool min E_th/|Edot|.
 * ou_*            OU forcing (Sec. 3.1.1): seed of the counter-based noise,
 *                 correlation time tau, target rms acceleration arms,
 *                 solenoidal fraction zeta, forced band kmin <= |n| <= kmax
 *                 (integer mode numbers), and update period every (the mode
 *                 amplitudes advance once every `every` steps by every*dt).
 * grav_G          gravitational constant of lap(phi) = 4 pi G (rho - <rho>).
 * mg_*            multigrid (Sec. 6.2, App. C): pre/post smoothing sweeps,
 *                 maximum cycles per step, coarsest grid size, relative
 *                 residual tolerance (0 runs exactly max_cycles cycles; with
 *                 a tolerance the solve also stops when a cycle cuts the
 *                 residual by less than 10 %, its round-off floor, which in
 *                 fp32 lies near 1e-4 of ||F|| at 128^3),
 *                 Jacobi sweeps used to solve the coarsest grid, the cycle
 *                 (MH_MG_V, or MH_MG_W: two coarse cycles per level, the
 *                 paper's default) and the smoother (MH_SMOOTH_JACOBI,
 *                 weighted with omega = 2/3, or MH_SMOOTH_RBGS, red-black
 *                 Gauss-Seidel).
 * grav_solver     MH_GRAV_MG (the multigrid solve, central-difference
 *                 gradient) or MH_GRAV_FFT (the spectral solve and gradient
 *                 of Sec. 6.1; power-of-two n). */
typedef struct mh_physics_desc {
  uint32_t flags;
  int32_t ou_every;
  double cool_lambda0, cool_tc, cool_ts, cool_tfloor;
  uint64_t ou_seed;
  double ou_tau, ou_arms, ou_zeta, ou_kmin, ou_kmax;
  double grav_G;
  int32_t mg_pre, mg_post, mg_max_cycles, mg_coarsest;
  double mg_tol;
  int32_t mg_coarse_sweeps;
  int32_t mg_cycle;
  int32_t mg_smoother;
  int32_t grav_solver;
  int32_t cool_model;
  int32_t cool_integrator;
  int32_t cool_nsub_max;
  int32_t cool_ntab;
  double cool_frac, cool_ccool;
  double cool_L1, cool_a1, cool_L2, cool_a2, cool_heat;
  double cool_logT[MH_COOL_TABMAX], cool_logL[MH_COOL_TABMAX];
} mh_physics_desc;

typedef struct mh_ctx mh_ctx;

/* Bytes of device workspace that mh_init needs for this grid and physics.
 * Returns MH_E_INVALID / MH_E_SHAPE / MH_E_DTYPE / MH_E_UNSUPPORTED for
 * descriptors that mh_init would reject. */
mh_status mh_query_workspace(const mh_grid_desc *grid, const mh_physics_desc *phys,
                             size_t *bytes);

/* Creates a context on the current HIP device.  `workspace` is device memory
 * of at least mh_query_workspace bytes, 256-byte aligned, owned by the caller.
 * `stream` is a hipStream_t (NULL = the default stream).  The clock starts at
 * t = 0, step 0; the OU modes start from their stationary draw (Sec. 3.1.1).
 * Uploads the grid-only tables; synchronises. */
mh_status mh_init(const mh_grid_desc *grid, const mh_physics_desc *phys, void *workspace,
                  size_t workspace_bytes, void *stream, mh_ctx **out);

/* Copies a state [5][nz][ny][nx] of the context's dtype into the context.
 * where = MH_HOST (synchronises) or MH_DEVICE (device pointer, asynchronous;
 * the source must stay valid until the stream reaches this copy). */
mh_status mh_set_state(mh_ctx *ctx, const void *U, int where);

/* Copies the current state out; MH_HOST synchronises. */
mh_status mh_get_state(mh_ctx *ctx, void *U, int where);

/* Advances nsteps steps.  dt > 0: fixed step; dt <= 0: CFL step computed on
 * the device from the current state.  Each step's dt is capped so that the
 * clock does not pass t_stop (pass +INFINITY for no cap; a step that starts
 * at t_stop has dt = 0).  dt_out (nsteps doubles) and t_out (one double) are
 * optional host pointers; when either is non-NULL the call synchronises. */
mh_status mh_step(mh_ctx *ctx, int32_t nsteps, double dt, double t_stop, double *dt_out,
                  double *t_out);

/* Reads the device clock (t, global step index); synchronises. */
mh_status mh_get_clock(mh_ctx *ctx, double *t, int64_t *step);

/* Sets the device clock, e.g. to resume from a checkpoint. */
mh_status mh_set_clock(mh_ctx *ctx, double t, int64_t step);

/* Number of OU modes and copy of their amplitudes ahat[m][comp][re,im]
 * (6 doubles per mode) to or from host memory (checkpoint / resume);
 * synchronise. */
mh_status mh_get_ou_state(mh_ctx *ctx, int32_t *nmodes, double *ahat);
mh_status mh_set_ou_state(mh_ctx *ctx, const double *ahat);

/* Health of the last mh_step call: number of cells flagged (non-finite, or
 * rho <= 0, or P <= 0) after any step, and the flat index q = (k ny + j) nx + i
 * of the lowest flagged cell (-1 if none).  Synchronises.  Returns
 * MH_E_NONFINITE when any cell was flagged. */
mh_status mh_check(mh_ctx *ctx, int64_t *bad_cells, int64_t *first_bad);

/* Multigrid cycles run by the last step with gravity (0 without gravity);
 * synchronises. */
mh_status mh_last_mg_cycles(mh_ctx *ctx, int32_t *cycles);

/* Copies the gravitational potential [nz][ny][nx] (dtype of the context)
 * solved by the last step with gravity; where = MH_HOST (synchronises) or
 * MH_DEVICE. */
mh_status mh_get_potential(mh_ctx *ctx, void *phi, int where);

/* Reverse-mode derivative of one step (paper Sec. 2.3; the adjoint of the
 * Poisson solve is a second solve with the same symmetric operator,
 * Sec. 6.2.4), with dt held fixed (the gradient stop of App. A.4):
 *   lam_n = (dU^{n+1}/dU^n)^T lam_np1
 * for the step taken from the state U_n with time step dt, at global step
 * index `step` (it keys the OU noise).  At every non-smooth point the
 * derivative of the branch the forward took is used: minmod the argument it
 * returned (0 when it returned 0), the wave-speed min/max the selected
 * argument (the first on ties), HLLC the side and fan the face fell in, the
 * cooling branch and floor those taken.  Van Leer's slope 2ab/(a+b) is
 * differentiated where ab > 0; MC takes the smallest of |a+b|/2, 2|a|, 2|b|
 * (ties in that order), superbee the larger of min(2|a|, |b|) and min(|a|,
 * 2|b|) (the first on ties, each min its first argument on ties); HLL the
 * region selected; Rusanov the larger signal speed (the left one on ties)
 * with d|v|/dv = -1 for v < 0, else +1.
 * U_n, lam_np1, lam_n: device arrays [5][nz][ny][nx] of the context dtype;
 *   lam_n may alias lam_np1.
 * ou_ahat: host array of the OU amplitudes before the step (6 doubles per mode,
 *   as from mh_get_ou_state); required when forcing is on, else ignored.
 * phi_n: device array [nz][ny][nx], the potential before the step (the warm
 *   start of the forward solve), or NULL for a zero start; used with gravity.
 * adj_workspace: device memory of at least mh_query_adjoint_workspace bytes,
 *   256-byte aligned, owned by the caller; it holds the recomputed forward
 *   intermediates and the scratch of the reverse sweep.  The context's own
 *   state, clock, OU amplitudes and potential are not touched.
 * Enqueued on the context stream; with gravity it synchronises once per
 * multigrid cycle.  Every grid, scheme, integrator and source the context
 * accepts is supported; the tabulated cooling model is differentiated through
 * its integrator's branches (floor, limiter, substep count and integrator
 * choice held as taken).  Errors: MH_E_INVALID (null pointer, or ou_ahat
 * missing with forcing on), MH_E_WORKSPACE, MH_E_DEVICE. */
mh_status mh_query_adjoint_workspace(mh_ctx *ctx, size_t *bytes);
mh_status mh_adjoint_step(mh_ctx *ctx, void *adj_workspace, size_t adj_workspace_bytes,
                          const void *U_n, double dt, int64_t step, const double *ou_ahat,
                          const void *phi_n, const void *lam_np1, void *lam_n);

/* Store instead of recompute (paper Sec. 2.3: a checkpointed rollout trades
 * memory for recomputation).  mh_step_keep advances ONE SSP-RK2 step like
 * mh_step(ctx, 1, dt, +INFINITY, dt_out, NULL) and also keeps, in device
 * memory the caller owns ([5][nz][ny][nx] each, the state's dtype, distinct),
 *   U1_out  the first stage U^n + dt L(U^n),
 *   Ub_out  the state after the last stage and its forcing kick, before
 *           gravity and cooling;
 * the state it leaves is bitwise the one mh_step leaves (the cooling and the
 * CFL/health epilogue run from Ub in a second kernel with the fused stage's
 * arithmetic; with gravity or tabulated cooling Ub is copied to the state
 * and those kernels follow as usual).  Enqueued on the context stream;
 * dt_out (one double, optional) synchronises.
 * mh_adjoint_step_kept is mh_adjoint_step for that step given U1 and Ub: it
 * skips recomputing the two stages.  With multigrid gravity, phi_np1 (device,
 * [nz][ny][nx], or NULL) may give the potential the step solved for -- the
 * context's potential right after the step (mh_get_potential) -- and the
 * forward Poisson solve from phi_n is skipped too (it would return those
 * bits); the adjoint potential is still solved.  phi_np1 is ignored without
 * gravity and with the spectral solver.  The result is bitwise
 * mh_adjoint_step's.
 * Errors: MH_E_INVALID (null or equal buffers, an integrator other than
 * MH_RK_SSP2, ou_ahat missing with forcing on, bad dt or step),
 * MH_E_WORKSPACE, MH_E_DEVICE. */
mh_status mh_step_keep(mh_ctx *ctx, double dt, void *U1_out, void *Ub_out, double *dt_out);
mh_status mh_adjoint_step_kept(mh_ctx *ctx, void *adj_workspace, size_t adj_workspace_bytes,
                               const void *U_n, const void *U1, const void *Ub, double dt,
                               int64_t step, const double *ou_ahat, const void *phi_n,
                               const void *phi_np1, const void *lam_np1, void *lam_n);

/* ------------------------------------------------------------------------ */
/* Learned state corrector (solver in the loop, paper Sec. 8)               */
/* ------------------------------------------------------------------------ */
/* A 3D convolutional network applied to a batch of coarse states after a
 * step:  x = (U - mean)/std;  h1 = GELU(conv(x; W1) + b1) (5 -> 32);
 * h2 = GELU(conv(h1; W2) + b2) (32 -> 32);  y = conv(h2; W3) + b3 (32 -> 5);
 * U' = U + scale * y.  conv is a 3x3x3 cross-correlation with periodic
 * padding (the paper pads its network periodically), GELU the erf form.
 * The standardised input enters as two bf16 parts per field (hi + lo, about
 * 16 significant bits) that share the first layer's weights.
 * Operands are bf16 with fp32 accumulation on the matrix cores; the fp32
 * master parameters are trained with ADAM (Sec. 7) on the loss
 * L = sum_c w_c mean((U'_c - T_c)^2) / std_c^2 (density weighted up).
 * Parameters, flat fp32 in this order: W1[32][5][27], b1[32],
 * W2[32][32][27], b2[32], W3[5][32][27], b3[5] (36 357 values); tap
 * t = 9(dz+1) + 3(dy+1) + (dx+1) reads the input at (x+dx, y+dy, z+dz).
 * States are device arrays [batch][5][n][n][n] of dtype MH_F32 or MH_F64.
 * n must be a multiple of 16. */
enum { MH_CORR_STATE = 0, MH_CORR_FLUX = 1 };

typedef struct mh_corr_desc {
  int32_t n;          /* cells per axis of each (cubic, periodic) state */
  int32_t batch;      /* states per call */
  int32_t dtype;      /* MH_F32 or MH_F64 */
  int32_t mode;       /* MH_CORR_STATE: the corrected state U + scale Net(U);
                         MH_CORR_FLUX: the correction scale Net(U) alone, a
                         learned flux field for mh_set_flux_correction
                         (Sec. 8), without floor or fallback */
  double gamma;       /* adiabatic index (for the positivity floor) */
  double mean[5];     /* per-channel standardisation of the network input */
  double std[5];
  double scale[5];    /* per-channel scale of the network output */
  double loss_w[5];   /* per-channel loss weights */
  double floor_rel;   /* floor: rho >= floor_rel <rho>, P >= floor_rel <P> */
  double fallback_frac; /* fall back to the uncorrected state above this
                           fraction of floored cells */
} mh_corr_desc;

typedef struct mh_corr mh_corr;

mh_status mh_corr_query_workspace(const mh_corr_desc *desc, size_t *bytes);
/* Creates a corrector on the current device in caller-owned workspace (256-
 * byte aligned), enqueuing on `stream`; parameters start at zero. */
mh_status mh_corr_init(const mh_corr_desc *desc, void *workspace, size_t bytes, void *stream,
                       mh_corr **out);
/* Sets the fp32 parameters (host or device, MH_HOST synchronises) and clears
 * the ADAM moments and iteration count. */
mh_status mh_corr_set_params(mh_corr *c, const float *theta, int where);
mh_status mh_corr_get_params(mh_corr *c, float *theta, int where);
/* State mode: U_out = floor(U + scale * Net(U)); when any value is non-finite or more
 * than fallback_frac of the cells needed the floor, U_out = U instead
 * (the plain coarse state; the choice is made on the device).  U_out must
 * not alias U.  floored / fell_back are optional host outputs: when either
 * is non-null the call synchronises, otherwise it only enqueues.  Inference
 * does not store z1 and z2 (activations 1 and 3 keep the last training
 * pass's values). */
mh_status mh_corr_apply(mh_corr *c, const void *U, void *U_out, int64_t *floored,
                        int32_t *fell_back);
/* (Flux mode: U_out = scale * Net(U); floored and fell_back report 0.) */
/* Loss against the target batch and its gradient in the parameters (to host
 * or device memory): zero_grad + backward(U, target) + get_grad;
 * synchronises.  State mode only (MH_E_INVALID in flux mode, whose output
 * is trained through the solver with mh_corr_backward and an upstream
 * gradient). */
mh_status mh_corr_loss_grad(mh_corr *c, const void *U, const void *target, double *loss,
                            float *grad, int where);
/* One ADAM iteration (learning rate lr) on the loss against target; returns
 * the loss before the update when loss is non-null (then synchronises). */
mh_status mh_corr_train_step(mh_corr *c, const void *U, const void *target, float lr,
                             double *loss);
/* Sets the accumulated parameter gradient to zero. */
mh_status mh_corr_zero_grad(mh_corr *c);
/* Reverse pass at U (the forward pass is recomputed first).  The upstream
 * gradient dL/dU' is the loss gradient against `target` (when non-NULL; the
 * loss value goes to *loss when loss is non-NULL, and then the call
 * synchronises) plus gUc (when non-NULL, a device array like U); at least one
 * must be given.  The parameter gradient is added to the accumulated one.
 * When gU is non-NULL it receives dL/dU (device array like U, aliasing
 * neither U nor gUc): the upstream gradient (residual path) plus the network
 * path; the positivity floor and the two-part input split pass the gradient
 * through unchanged.  In flux mode target must be NULL and gU receives the
 * network path alone (the output has no residual term).  Used to unroll
 * training through several solver steps together with mh_adjoint_step. */
mh_status mh_corr_backward(mh_corr *c, const void *U, const void *target, const void *gUc,
                           double *loss, void *gU);
/* One ADAM iteration with the accumulated gradient (learning rate lr). */
mh_status mh_corr_adam_step(mh_corr *c, float lr);
/* Copies the accumulated parameter gradient (canonical order). */
mh_status mh_corr_get_grad(mh_corr *c, float *grad, int where);
/* Copies an activation of the last forward pass: 0 x (bf16, [cells][32]:
 * channel c < 5 holds hi = bf16(x_c), channel 5 + c holds bf16(x_c - hi)),
 * 1 z1 (fp32, [cells][32]), 2 h1 (bf16), 3 z2 (fp32), 4 h2 (bf16),
 * 5 y (fp32, [cells][16]; stored by the training forward only: mh_corr_apply
 * and mh_step_corrected write the residual update from the last layer's
 * epilogue and leave y as it was); or a gradient of the last reverse pass
 * (mh_corr_backward, mh_corr_loss_grad): 6 dY = bf16(scale dL/dU')
 * (bf16, [cells][16], channels >= 5 zero), 7 dZ2 (bf16, [cells][32]),
 * 8 dZ1 (bf16, [cells][32]), 9 the first layer's transposed convolution of
 * dZ1 (fp32, [cells][16]; channel c < 5 the gradient of input part hi,
 * 5 + c of part lo; written only when dL/dU was requested); cells =
 * batch n^3.  MH_HOST synchronises.  Errors: MH_E_INVALID (null handle or
 * destination, which outside 0..9, bad where). */
mh_status mh_corr_get_activation(mh_corr *c, int which, void *dst, int where);
void mh_corr_destroy(mh_corr *c);

/* The corrector inside the step (Sec. 8, the solver-in-the-loop update
 * U^{n+1} = U* + s Net(U*), U* = H(U^n) the plain coarse step): advances B
 * contexts together by nsteps corrected steps.  Each step enqueues every
 * context's plain step, gathers the B states into stage[0 .. B 5 n^3),
 * applies the corrector to the batch into stage[B 5 n^3 .. 2 B 5 n^3) with
 * mh_corr_apply's semantics (residual update, positivity floor, fallback to
 * the plain states when a value is non-finite or too many cells needed the
 * floor) and scatters the result back into the contexts.  No step waits for
 * the host.
 *   ctxs      B distinct contexts with the same cubic grid n^3 and dtype,
 *             created on one stream; corr: a state-mode corrector of batch B,
 *             cube n and that dtype, on the same stream.
 *   stage     caller device buffer of 2 B 5 n^3 values of the dtype.
 *   dts       device array of nsteps * B doubles: step s of context b takes
 *             dts[s B + b]; NULL = CFL steps (each context's dt from its own
 *             corrected state).  The clock, OU forcing and the other sources
 *             advance as in mh_step.
 *   use_graph 1: one corrected step is captured into a HIP graph and
 *             replayed nsteps times (synchronises at the end); contexts with
 *             gravity are rejected in this mode (MH_E_UNSUPPORTED: the
 *             multigrid convergence test reads the host).  0: launched
 *             kernel by kernel.  Both give bitwise the same states.
 *   fallbacks optional host pointer: the number of steps whose correction
 *             fell back to the plain states (synchronises).
 * Errors (message in mh_last_error(ctxs[0])): MH_E_INVALID (null pointers,
 * repeated contexts, nsteps < 0, different streams), MH_E_SHAPE (non-cubic
 * grid, grids or dtypes that differ, a corrector that does not match),
 * MH_E_UNSUPPORTED, MH_E_DEVICE. */
mh_status mh_step_corrected(mh_ctx *const *ctxs, int32_t B, mh_corr *corr, void *stage,
                            int32_t nsteps, const double *dts, int32_t use_graph,
                            int64_t *fallbacks);

/* One ADAM update (Kingma & Ba 2015; the optimiser of the paper's
 * reconstructions, Sec. 7) of `count` parameters in place, on device arrays
 * of dtype: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * theta -= lr (m / (1 - b1^it)) / (sqrt(v / (1 - b2^it)) + eps), with it >= 1
 * the iteration number.  The caller owns theta, m, v (zero before the first
 * iteration) and grad.  Enqueued on `stream`.  Errors: MH_E_INVALID (null
 * pointer, count < 0, it < 1, lr < 0, betas outside [0, 1), eps <= 0),
 * MH_E_DTYPE, MH_E_DEVICE. */
mh_status mh_adam(void *theta, void *m, void *v, const void *grad, int64_t count, int32_t dtype,
                  int64_t it, double lr, double beta1, double beta2, double eps, void *stream);

/* Conservative r^3 block average of a fine state [5][nf^3] onto
 * [5][(nf/r)^3] (targets of the corrector from a fine run); device arrays of
 * dtype, enqueued on `stream`. */
mh_status mh_block_average(const void *fine, int32_t nf, int32_t r, void *coarse, int32_t dtype,
                           void *stream);

/* In-place 3D discrete Fourier transform of an n^3 complex array on the
 * device (the transform of the spectral gravity solver, Sec. 6.1, offered on
 * its own for spectral initial conditions): data holds interleaved (re, im)
 * values of dtype, x fastest; forward X_k = sum_j x_j exp(-2 pi i j.k/n),
 * inverse unnormalised (sum with exp(+...)).  n is a power of two, 2..1024.
 * workspace: device memory of at least mh_fft3_query_workspace bytes (the
 * twiddle table, rewritten by every call).  Enqueued on `stream`.  Errors:
 * MH_E_INVALID (null pointer, inverse not 0/1), MH_E_SHAPE (n), MH_E_DTYPE,
 * MH_E_WORKSPACE, MH_E_DEVICE. */
mh_status mh_fft3_query_workspace(int32_t n, int32_t dtype, size_t *bytes);
mh_status mh_fft3(void *data, int32_t n, int32_t dtype, int32_t inverse, void *workspace,
                  size_t workspace_bytes, void *stream);

/* mh_fft3 without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The twiddle table
 * lives in a library-owned device array of 8 KiB per GPU (enough for every n
 * and dtype mh_fft3 accepts), whose device address is looked up once per GPU
 * on the first call with that GPU current; `data` and `stream` must belong to
 * the current device.  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  Every call on a GPU rewrites that GPU's table,
 * so calls that overlap on one GPU (two streams, or two host threads) race:
 * serialise them.  Arguments, layout and result are those of mh_fft3.
 * Errors: MH_E_INVALID (null data, inverse not 0/1), MH_E_SHAPE (n not a
 * power of two in 2..1024), MH_E_DTYPE, MH_E_WORKSPACE (a table larger than
 * the array; not reachable with the sizes above), MH_E_DEVICE (HIP error, or
 * a device index of 64 or more). */
mh_status mh_fft3_noalloc(void *data, int32_t n, int32_t dtype, int32_t inverse, void *stream);

/* Kernel timing with HIP events.  While enabled, mh_step records an event pair
 * on the context stream around every kernel launch it makes, by kind:
 *   MH_TIME_STAGE1, MH_TIME_STAGE2 (the fused stage kernels),
 *   MH_TIME_PROLOGUE (per-step dt / OU kernel), MH_TIME_OTHER (CFL reduction
 *   after set_state, multigrid and gravity kernels, bookkeeping).
 * mh_get_timing synchronises, returns per kind the summed milliseconds and
 * the number of timed launches (arrays of MH_TIME_KINDS), and clears the
 * records.  At most 65536 launches are timed between two reads; later ones
 * are counted in MH_TIME_OTHER's count only.  Timing adds the event records'
 * small cost to every launch; it is off by default. */
enum { MH_TIME_STAGE1 = 0, MH_TIME_STAGE2 = 1, MH_TIME_PROLOGUE = 2, MH_TIME_OTHER = 3,
       MH_TIME_KINDS = 4 };
mh_status mh_set_timing(mh_ctx *ctx, int enable);
mh_status mh_get_timing(mh_ctx *ctx, double *ms, int64_t *launches);

/* Sets the gravitational potential [nz][ny][nx] (dtype of the context) that
 * the next step's multigrid solve starts from (resume from a checkpoint);
 * where = MH_HOST (synchronises) or MH_DEVICE.  MH_E_INVALID without gravity. */
mh_status mh_set_potential(mh_ctx *ctx, const void *phi, int where);

/* Learned flux correction (Sec. 8: the solver-in-the-loop flux term added to
 * the base convective fluxes).  field: device array [5][nz][ny][nx] of the
 * context dtype, in the conserved-field order, or NULL to switch it off; its
 * value at a cell is added to the flux through the cell's upper face on each
 * axis (x+1/2, y+1/2, z+1/2; with outflow the lowest face of an axis takes
 * the value of the first cell), in every RK stage of every later mh_step,
 * until changed.  Steps with a field run the kernel that takes the scheme at
 * run time.  grad: device array of the same shape, or NULL; when given, every
 * later mh_adjoint_step adds (dU^{n+1}/d field)^T lam^{n+1} to it (the
 * caller zeroes it).  Both stay owned by the caller and must stay valid while
 * attached.  Enqueues nothing. */
mh_status mh_set_flux_correction(mh_ctx *ctx, const void *field, void *grad);

/* Multigrid V-cycles are replayed from HIP graphs captured on first use
 * (one V-cycle is ~60 small launches); enable = 0 launches them kernel by
 * kernel instead.  Default on; results are identical either way.
 * Synchronises. */
mh_status mh_set_graphs(mh_ctx *ctx, int enable);

/* Message of the last failed call on ctx (empty string if none). */
const char *mh_last_error(const mh_ctx *ctx);

/* Waits for the context's stream, then frees the host context (not the
 * workspace, which the caller owns). */
void mh_destroy(mh_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
