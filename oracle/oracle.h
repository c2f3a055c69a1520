/*
 * oracle.h -- declarations of the FP64 CPU oracle (test infrastructure only;
 * never included by the product library).
 */
#ifndef MIHYDRO_ORACLE_H
#define MIHYDRO_ORACLE_H

#include <stdint.h>

enum { OR_BC_PERIODIC = 0, OR_BC_OUTFLOW = 1 };
enum { OR_LIM_MINMOD = 0, OR_LIM_NONE = 1, OR_LIM_VANLEER = 2, OR_LIM_MC = 3,
       OR_LIM_SUPERBEE = 4 };
enum { OR_RS_HLLC = 0, OR_RS_HLL = 1, OR_RS_RUSANOV = 2 };
enum { OR_RK_SSP2 = 0, OR_RK_SSP3 = 1, OR_RK_EULER = 2 };
enum { OR_MG_V = 0, OR_MG_W = 1 };
enum { OR_SMOOTH_JACOBI = 0, OR_SMOOTH_RBGS = 1 };
enum { OR_GRAV_MG = 0, OR_GRAV_FFT = 1 };
enum { OR_COOL_EXACT2 = 0, OR_COOL_TABLE = 1 };
enum { OR_COOLINT_TRAPEZOID = 0, OR_COOLINT_SUBCYCLE = 1, OR_COOLINT_AUTO = 2 };
#define OR_COOL_TABMAX 64
enum { OR_SRC_COOLING = 1u, OR_SRC_FORCING = 2u, OR_SRC_GRAVITY = 4u };
#define OR_OU_MAXMODES 64

/* Everything one step needs.  Mirrored field for field by a ctypes Structure
 * in oracle/__init__.py. */
typedef struct {
  int32_t n[3];
  int32_t bc[3];
  double h[3];
  double gamma;
  double cfl;
  int32_t limiter;
  int32_t riemann;
  uint32_t flags;
  int32_t ou_every;
  double cool_lambda0, cool_tc, cool_ts, cool_tfloor;
  uint64_t ou_seed;
  double ou_tau, ou_arms, ou_zeta, ou_kmin, ou_kmax;
  double grav_G;
  int32_t mg_pre, mg_post, mg_max_cycles, mg_coarsest;
  double mg_tol;
  int32_t mg_coarse_sweeps;
  int32_t integrator; /* OR_RK_* */
  int32_t mg_cycle;    /* OR_MG_V or OR_MG_W */
  int32_t mg_smoother; /* OR_SMOOTH_* */
  int32_t grav_solver; /* OR_GRAV_MG or OR_GRAV_FFT */
  int32_t cool_model;  /* OR_COOL_EXACT2 or OR_COOL_TABLE */
  int32_t cool_integrator; /* OR_COOLINT_* (tabulated model) */
  int32_t cool_nsub_max;   /* most substeps of the subcycled update */
  int32_t cool_ntab;       /* points of the CIE table */
  int32_t pad2_;
  double cool_frac;  /* largest fractional change of E_th per substep */
  double cool_ccool; /* c_cool of the cooling-time step limit (0: off) */
  double cool_L1, cool_a1, cool_L2, cool_a2; /* low-T branch L1 T^a1 + L2 T^a2 */
  double cool_heat;  /* heating rate Gamma_0 below cool_tc */
  double cool_logT[OR_COOL_TABMAX], cool_logL[OR_COOL_TABMAX]; /* log10 T, log10 Lambda */
  /* learned flux correction (Sec. 8, the solver-in-the-loop flux term): a
   * per-cell field [5][N] added to the flux of the cell's +x, +y and +z
   * faces in every stage, or NULL */
  const double *flux_corr;
} or_config;

void or_primitives(const or_config *c, const double *U, double *W);
double or_cfl_dt(const or_config *c, const double *U);
void or_rhs(const or_config *c, const double *U, double *L);
void or_rk2(const or_config *c, double *U, double dt);
void or_euler(const or_config *c, double *U, double dt);
void or_ssprk3(const or_config *c, double *U, double dt);
void or_integrate(const or_config *c, double *U, double dt);

double or_cool_temperature(double rho, double T, double dt, double gamma,
                           double L0, double Tc, double Ts, double Tfloor);
void or_cool(const or_config *c, double *U, double dt);

/* the tabulated heating/cooling model (oracle_cool.c) */
double or_cool_lambda(const or_config *c, double T);
double or_cool_edot(const or_config *c, double rho, double Eth);
double or_cool_eth_step(const or_config *c, double rho, double Eth, double dt);
double or_cool_dt_limit(const or_config *c, const double *U);
double or_cool_eth_step_d(const or_config *c, double rho, double Eth, double dt, double *dE,
                          double *dr);

void or_ou_gauss(uint64_t seed, int64_t group, int mode, int comp, double out[2]);
int or_ou_modes(double kmin, double kmax, int32_t *nvec);
void or_ou_init(const or_config *c, int nmodes, const int32_t *nvec, double *ahat);
void or_ou_advance(const or_config *c, int nmodes, const int32_t *nvec,
                   double *ahat, int64_t group, double dt);
double or_ou_scale(const or_config *c, int nmodes, const double *ahat);
void or_ou_accel_at(const or_config *c, int nmodes, const int32_t *nvec,
                    const double *ahat, long i, long j, long k, double out[3]);
void or_ou_accel(const or_config *c, int nmodes, const int32_t *nvec,
                 const double *ahat, double *acc);
void or_kick(const or_config *c, double *U, const double *acc, double dt);

/* multigrid self-gravity (oracle_mg.c) */
void or_laplacian(int n, double h, const double *phi, double *out);
void or_mg_vcycle(const or_config *c, int n, double h, double *phi, const double *F);
int or_mg_solve(const or_config *c, int n, double h, double *phi, const double *F);
int or_gravity_accel(const or_config *c, const double *U, double *phi, double *acc);
void or_mg_smooth(const or_config *c, int n, double h, double *phi, const double *F);

/* spectral self-gravity (oracle_fft.c) */
void or_dft3(int n, int inverse, double *re, double *im);
void or_fft_gravity(const or_config *c, const double *rho, double *phi, double *acc);
void or_fft_gravity_vjp(const or_config *c, const double *accb, double *rhob);

int or_num_threads(void);
void or_set_num_threads(int n);

/* reverse-mode derivatives (oracle_adjoint.c) */
void or_hllc_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                 double wlb[5], double wrb[5]);
void or_hll_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                double wlb[5], double wrb[5]);
void or_rusanov_vjp(const double wl[5], const double wr[5], double g, const double Fb[5],
                    double wlb[5], double wrb[5]);
void or_rhs_vjp(const or_config *c, const double *U, const double *v, double *out);
void or_euler_vjp(const or_config *c, const double *U, double dt, const double *lam1,
                  double *lam);
void or_ssprk3_vjp(const or_config *c, const double *U, double dt, const double *lam3,
                   double *lam);
void or_integrate_vjp(const or_config *c, const double *U, double dt, const double *lamp,
                      double *lam);
void or_flux_corr_vjp(const or_config *c, const double *v, double weight, double *g);
void or_integrate_vjp_flux(const or_config *c, const double *U, double dt, const double *lamp,
                           double *lam, double *gflux);
void or_step_vjp_flux(const or_config *c, const double *Un, double dt, int64_t step, int nmodes,
                      const int32_t *nvec, const double *ou_ahat, double *phi,
                      const double *lam_np1, double *lam_n, double *gflux);
void or_rk2_vjp(const or_config *c, const double *U, double dt, const double *lam2,
                double *lam);
void or_kick_vjp(const or_config *c, const double *U, const double *acc, double dt,
                 const double *lamp, double *lam, double *accb);
void or_cool_vjp(const or_config *c, const double *U, double dt, const double *lamp,
                 double *lam);
int or_gravity_vjp(const or_config *c, const double *U, double dt, double *phi,
                   const double *lamp, double *lam);
void or_step_vjp(const or_config *c, const double *Un, double dt, int64_t step, int nmodes,
                 const int32_t *nvec, const double *ou_ahat, double *phi,
                 const double *lam_np1, double *lam_n);

double or_step(const or_config *c, double *U, double dt_fixed, double dt_cap,
               int64_t step, int nmodes, const int32_t *nvec, double *ou_ahat,
               double *phi, int *mg_cycles);

#endif
