// api.hip -- the C ABI of libmihydro (declared in include/mihydro.h): argument
// checking, the device-workspace layout, and the per-step launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mihydro.h"
#include "mg.h"
#include "mh_corrector.h"
#include "mh_adjoint.h"
#include "mh_device.h"
#include "mh_launch.h"

using namespace mh;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Layout {
  size_t U = 0, U1 = 0, U2 = 0, cool_tab = 0, clk = 0, dtlog = 0, ou_n = 0, ou_ahat = 0, ou_coef = 0, ou_rows = 0;
  size_t tab[3] = {0, 0, 0};
  MGLayout mg;
  size_t total = 0;
};

int ou_enumerate(double kmin, double kmax, std::vector<int>& nv) {
  // integer n with kmin <= |n| <= kmax, one of each +-n pair (first non-zero
  // component positive), lexicographic in (nx, ny, nz); same rule as the
  // reference order of the noise stream
  nv.clear();
  const int r = (int)std::ceil(kmax);
  for (int a = -r; a <= r; ++a)
    for (int b = -r; b <= r; ++b)
      for (int d = -r; d <= r; ++d) {
        const double k = std::sqrt((double)(a * a + b * b + d * d));
        if (k < kmin || k > kmax || k == 0.0) continue;
        const int first = a != 0 ? a : (b != 0 ? b : d);
        if (first <= 0) continue;
        nv.push_back(a);
        nv.push_back(b);
        nv.push_back(d);
      }
  return (int)(nv.size() / 3);
}

mh_status validate(const mh_grid_desc* g, const mh_physics_desc* p, std::string& err,
                   int* nmodes_out) {
  auto fail = [&](mh_status s, const char* m) {
    err = m;
    return s;
  };
  if (!g || !p) return fail(MH_E_INVALID, "null descriptor");
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1) return fail(MH_E_INVALID, "grid size must be >= 1 along every axis");
    if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a]))
      return fail(MH_E_INVALID, "cell spacing must be positive and finite");
    if (g->bc[a] != MH_BC_PERIODIC && g->bc[a] != MH_BC_OUTFLOW)
      return fail(MH_E_INVALID, "unknown boundary kind");
  }
  const long long N = (long long)g->n[0] * g->n[1] * g->n[2];
  if (N > (1ll << 31)) return fail(MH_E_SHAPE, "more than 2^31 cells");
  if (g->dtype != MH_F32 && g->dtype != MH_F64) return fail(MH_E_DTYPE, "dtype must be F32 or F64");
  if ((long long)g->n[0] * g->n[1] * (g->dtype == MH_F64 ? 8 : 4) > 0xffffffffll)
    return fail(MH_E_SHAPE, "one x-y plane of a field must stay below 4 GiB");
  if (g->limiter < MH_LIM_MINMOD || g->limiter > MH_LIM_SUPERBEE)
    return fail(MH_E_UNSUPPORTED, "unknown limiter");
  if (g->riemann < MH_RS_HLLC || g->riemann > MH_RS_RUSANOV)
    return fail(MH_E_UNSUPPORTED, "unknown Riemann solver");
  if (g->integrator < MH_RK_SSP2 || g->integrator > MH_RK_EULER)
    return fail(MH_E_UNSUPPORTED, "unknown time integrator");
  if (!(g->gamma > 1.0)) return fail(MH_E_INVALID, "gamma must exceed 1");
  if (!(g->cfl > 0.0)) return fail(MH_E_INVALID, "CFL number must be positive");
  const uint32_t known = MH_SRC_COOLING | MH_SRC_FORCING | MH_SRC_GRAVITY;
  if (p->flags & ~known) return fail(MH_E_INVALID, "unknown source flag");
  if (p->flags & MH_SRC_COOLING) {
    if (!(p->cool_lambda0 >= 0.0) || !(p->cool_tc > 0.0) || !(p->cool_ts > 0.0) ||
        !(p->cool_tfloor >= 0.0))
      return fail(MH_E_INVALID, "cooling constants must be positive");
    if (p->cool_model != MH_COOL_EXACT2 && p->cool_model != MH_COOL_TABLE)
      return fail(MH_E_UNSUPPORTED, "unknown cooling model");
    if (!(p->cool_ccool >= 0.0)) return fail(MH_E_INVALID, "cool_ccool must be >= 0");
    if (p->cool_model == MH_COOL_EXACT2 && p->cool_ccool > 0.0)
      return fail(MH_E_UNSUPPORTED, "the cooling-time step limit needs the tabulated model");
    if (p->cool_model == MH_COOL_TABLE) {
      if (p->cool_integrator < MH_COOLINT_TRAPEZOID || p->cool_integrator > MH_COOLINT_AUTO)
        return fail(MH_E_UNSUPPORTED, "unknown cooling integrator");
      if (p->cool_ntab < 2 || p->cool_ntab > MH_COOL_TABMAX)
        return fail(MH_E_INVALID, "the cooling table needs 2..64 points");
      for (int i = 0; i < p->cool_ntab; ++i)
        if (!std::isfinite(p->cool_logT[i]) || !std::isfinite(p->cool_logL[i]) ||
            (i > 0 && !(p->cool_logT[i] > p->cool_logT[i - 1])))
          return fail(MH_E_INVALID, "cooling table: finite values, increasing log10 T");
      if (!(p->cool_tfloor > 0.0) || !(p->cool_frac > 0.0 && p->cool_frac <= 1.0) ||
          p->cool_nsub_max < 1 || p->cool_nsub_max > 1000000 || !(p->cool_heat >= 0.0) ||
          !std::isfinite(p->cool_L1) || !std::isfinite(p->cool_a1) ||
          !std::isfinite(p->cool_L2) || !std::isfinite(p->cool_a2))
        return fail(MH_E_INVALID,
                    "tabulated cooling: tfloor > 0, 0 < frac <= 1, 1 <= nsub_max <= 1e6, "
                    "heat >= 0, finite L1, a1, L2, a2");
    }
  }
  int nm = 0;
  if (p->flags & MH_SRC_FORCING) {
    if (!(p->ou_tau > 0.0) || !(p->ou_arms >= 0.0) || !(p->ou_zeta >= 0.0 && p->ou_zeta <= 1.0))
      return fail(MH_E_INVALID, "OU tau > 0, arms >= 0, 0 <= zeta <= 1 required");
    if (!(p->ou_kmin > 0.0) || !(p->ou_kmax >= p->ou_kmin) || p->ou_kmax > 8.0)
      return fail(MH_E_INVALID, "OU band needs 0 < kmin <= kmax <= 8");
    if (p->ou_every < 0) return fail(MH_E_INVALID, "OU update period must be >= 0");
    std::vector<int> nv;
    nm = ou_enumerate(p->ou_kmin, p->ou_kmax, nv);
    if (nm < 1) return fail(MH_E_INVALID, "OU band holds no integer mode");
    if (nm > MAX_MODES) return fail(MH_E_UNSUPPORTED, "more than 64 OU modes");
  }
  if (p->flags & MH_SRC_GRAVITY) {
    mh_status s = mg_validate(g, p, err);
    if (s != MH_OK) return s;
  }
  if (nmodes_out) *nmodes_out = nm;
  return MH_OK;
}

Layout make_layout(const mh_grid_desc* g, const mh_physics_desc* p, int nmodes) {
  Layout L;
  const size_t es = g->dtype == MH_F64 ? 8 : 4;
  const size_t N = (size_t)g->n[0] * g->n[1] * g->n[2];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.U = take(5 * N * es);
  L.U1 = take(5 * N * es);
  if (g->integrator == MH_RK_SSP3) L.U2 = take(5 * N * es);
  if ((p->flags & MH_SRC_COOLING) && p->cool_model == MH_COOL_TABLE)
    L.cool_tab = take(2 * MH_COOL_TABMAX * es);
  L.clk = take(sizeof(DevClock));
  L.dtlog = take(DTLOG_CAP * sizeof(double));
  if (p->flags & MH_SRC_FORCING) {
    const int R = (int)std::floor(p->ou_kmax);
    L.ou_n = take(3 * MAX_MODES * sizeof(int));
    L.ou_ahat = take(6 * MAX_MODES * sizeof(double));
    L.ou_coef = take(6 * MAX_MODES * es);
    for (int a = 0; a < 3; ++a) L.tab[a] = take((size_t)(R + 1) * g->n[a] * 2 * es);
    L.ou_rows = take((size_t)g->n[1] * g->n[2] * (R + 1) * 6 * es);
  }
  if (p->flags & MH_SRC_GRAVITY) off = mg_layout(g, p, off, es, L.mg);
  L.total = off;
  (void)nmodes;
  return L;
}

}  // namespace

struct mh_ctx {
  mh_grid_desc g;
  mh_physics_desc p;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout L;
  int nmodes = 0;
  bool smax_valid = false;
  std::string err;
  // kernel timing (mh_set_timing): event pairs and the kind of each pair
  bool timing = false;
  // V-cycle graphs of the step's solver and of the adjoint's second solve
  MGGraphCache mg_graphs, adj_graphs;
  // learned flux correction and the buffer its adjoint accumulates into
  const void* dflux = nullptr;
  void* dflux_grad = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> kinds;
  int64_t untimed = 0;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  long long cells() const { return (long long)g.n[0] * g.n[1] * g.n[2]; }
  size_t esize() const { return g.dtype == MH_F64 ? 8 : 4; }
  DevClock* clk() const { return at<DevClock>(L.clk); }
  // the tabulated cooling model runs as its own kernel at the end of a step
  bool cool_table() const {
    return (p.flags & MH_SRC_COOLING) && p.cool_model == MH_COOL_TABLE;
  }
  template <typename T>
  CoolTable<T> cool_table_args() const {
    CoolTable<T> t{};
    t.logT = at<T>(L.cool_tab);
    t.logL = at<T>(L.cool_tab) + MH_COOL_TABMAX;
    t.ntab = p.cool_ntab;
    t.integ = p.cool_integrator;
    t.nsub_max = p.cool_nsub_max;
    t.rate = p.cool_ccool > 0.0;
    t.tc = (T)p.cool_tc;
    t.tfloor = (T)p.cool_tfloor;
    t.L1 = (T)p.cool_L1;
    t.a1 = (T)p.cool_a1;
    t.L2 = (T)p.cool_L2;
    t.a2 = (T)p.cool_a2;
    t.heat = (T)p.cool_heat;
    t.frac = (T)p.cool_frac;
    return t;
  }
};

static constexpr size_t MAX_TIMED = 65536;

// begins a timed launch of the given kind; returns the pair index or -1
static long time_begin(mh_ctx* c, int kind) {
  if (!c->timing) return -1;
  if (c->kinds.size() >= MAX_TIMED) {
    ++c->untimed;
    return -1;
  }
  const size_t i = c->kinds.size();
  while (c->ev.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    c->ev.push_back(e);
  }
  if (hipEventRecord(c->ev[2 * i], c->stream) != hipSuccess) return -1;
  c->kinds.push_back(kind);
  return (long)i;
}

static void time_end(mh_ctx* c, long i) {
  if (i >= 0) (void)hipEventRecord(c->ev[2 * i + 1], c->stream);
}

static mh_status set_err(mh_ctx* c, mh_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define MH_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(ctx, MH_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

extern "C" mh_status mh_query_workspace(const mh_grid_desc* grid, const mh_physics_desc* phys,
                                        size_t* bytes) {
  std::string err;
  int nm = 0;
  if (!bytes) return MH_E_INVALID;
  mh_status s = validate(grid, phys, err, &nm);
  if (s != MH_OK) return s;
  *bytes = make_layout(grid, phys, nm).total;
  return MH_OK;
}

template <typename T>
static mh_status upload_tables(mh_ctx* c) {
  const mh_physics_desc& p = c->p;
  if (c->cool_table()) {
    std::vector<T> tab(2 * MH_COOL_TABMAX, T(0));
    for (int i = 0; i < p.cool_ntab; ++i) {
      tab[i] = (T)p.cool_logT[i];
      tab[MH_COOL_TABMAX + i] = (T)p.cool_logL[i];
    }
    MH_HIP(c, hipMemcpyAsync(c->ws + c->L.cool_tab, tab.data(), tab.size() * sizeof(T),
                             hipMemcpyHostToDevice, c->stream));
    MH_HIP(c, hipStreamSynchronize(c->stream));
  }
  if (!(p.flags & MH_SRC_FORCING)) return MH_OK;
  std::vector<int> nv;
  ou_enumerate(p.ou_kmin, p.ou_kmax, nv);
  MH_HIP(c, hipMemcpyAsync(c->ws + c->L.ou_n, nv.data(), nv.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  const int R = (int)std::floor(p.ou_kmax);
  for (int a = 0; a < 3; ++a) {
    const int n = c->g.n[a];
    std::vector<T> tab((size_t)(R + 1) * n * 2);
    for (int k = 0; k <= R; ++k)
      for (int i = 0; i < n; ++i) {
        const double th = 2.0 * M_PI * k * (i + 0.5) / n;
        tab[2 * ((size_t)k * n + i)] = (T)std::cos(th);
        tab[2 * ((size_t)k * n + i) + 1] = (T)std::sin(th);
      }
    MH_HIP(c, hipMemcpyAsync(c->ws + c->L.tab[a], tab.data(), tab.size() * sizeof(T),
                             hipMemcpyHostToDevice, c->stream));
    MH_HIP(c, hipStreamSynchronize(c->stream));
  }
  return MH_OK;
}

static mh::OUArgs ou_args(const mh_ctx* c) {
  mh::OUArgs o{};
  o.clk = c->clk();
  o.ahat = c->at<double>(c->L.ou_ahat);
  o.nvec = c->at<int>(c->L.ou_n);
  o.coef = c->ws + c->L.ou_coef;
  o.f64 = c->g.dtype == MH_F64;
  o.nmodes = c->nmodes;
  o.every = c->p.ou_every > 0 ? c->p.ou_every : 1;
  o.seed = c->p.ou_seed;
  o.tau = c->p.ou_tau;
  o.arms = c->p.ou_arms;
  o.zeta = c->p.ou_zeta;
  return o;
}

extern "C" mh_status mh_init(const mh_grid_desc* grid, const mh_physics_desc* phys,
                             void* workspace, size_t workspace_bytes, void* stream,
                             mh_ctx** out) {
  if (!out) return MH_E_INVALID;
  *out = nullptr;
  std::string err;
  int nm = 0;
  mh_status s = validate(grid, phys, err, &nm);
  if (s != MH_OK) return s;
  Layout L = make_layout(grid, phys, nm);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0)
    return MH_E_WORKSPACE;
  mh_ctx* c = new mh_ctx();
  c->g = *grid;
  c->p = *phys;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->ws_bytes = workspace_bytes;
  c->L = L;
  c->L.mg.graphs = &c->mg_graphs;
  c->nmodes = nm;
  DevClock hc{};
  hc.bad_first = ~0ull;
  auto fail = [&](mh_status st) {
    delete c;
    return st;
  };
  if (hipMemcpyAsync(c->clk(), &hc, sizeof hc, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return fail(MH_E_DEVICE);
  s = grid->dtype == MH_F64 ? upload_tables<double>(c) : upload_tables<float>(c);
  if (s != MH_OK) return fail(s);
  if (phys->flags & MH_SRC_FORCING) {
    if (launch_ou_init(ou_args(c), c->stream) != hipSuccess) return fail(MH_E_DEVICE);
  }
  if (phys->flags & MH_SRC_GRAVITY) {
    if (mg_init(c->ws, L.mg, grid, c->stream) != hipSuccess) return fail(MH_E_DEVICE);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(MH_E_DEVICE);
  *out = c;
  return MH_OK;
}

extern "C" mh_status mh_set_state(mh_ctx* c, const void* U, int where) {
  if (!c) return MH_E_INVALID;
  if (!U || (where != MH_HOST && where != MH_DEVICE))
    return set_err(c, MH_E_INVALID, "mh_set_state: null pointer or bad location");
  const size_t bytes = 5 * (size_t)c->cells() * c->esize();
  MH_HIP(c, hipMemcpyAsync(c->ws + c->L.U, U, bytes,
                           where == MH_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->stream));
  if (where == MH_HOST) MH_HIP(c, hipStreamSynchronize(c->stream));
  c->smax_valid = false;
  return MH_OK;
}

extern "C" mh_status mh_get_state(mh_ctx* c, void* U, int where) {
  if (!c) return MH_E_INVALID;
  if (!U || (where != MH_HOST && where != MH_DEVICE))
    return set_err(c, MH_E_INVALID, "mh_get_state: null pointer or bad location");
  const size_t bytes = 5 * (size_t)c->cells() * c->esize();
  MH_HIP(c, hipMemcpyAsync(U, c->ws + c->L.U, bytes,
                           where == MH_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           c->stream));
  if (where == MH_HOST) MH_HIP(c, hipStreamSynchronize(c->stream));
  return MH_OK;
}

template <typename T>
static CoolParams<T> cool_params(const mh_grid_desc& g, const mh_physics_desc& p) {
  CoolParams<T> c;
  c.tc = (T)p.cool_tc;
  c.ts = (T)p.cool_ts;
  c.its = (T)(1.0 / p.cool_ts);
  c.tfloor = (T)p.cool_tfloor;
  c.sqrt_tc = (T)std::sqrt(p.cool_tc);
  c.k1r = (T)((g.gamma - 1.0) * p.cool_lambda0 / (2.0 * std::sqrt(p.cool_tc)));
  c.k2r = (T)((g.gamma - 1.0) * p.cool_lambda0 / p.cool_ts);
  return c;
}

// stage-kernel arguments shared by mh_step and mh_adjoint_step (everything
// but the state pointers)
template <typename T>
static StageArgs<T> base_stage_args(const mh_ctx* c, DevClock* clk, T* ou_rows) {
  const mh_grid_desc& g = c->g;
  const mh_physics_desc& p = c->p;
  StageArgs<T> a{};
  a.clk = clk;
  a.gamma = (T)g.gamma;
  a.gm1 = (T)(g.gamma - 1.0);
  a.gm1inv = (T)(1.0 / (g.gamma - 1.0));
  a.ihx = (T)(1.0 / g.h[0]);
  a.ihy = (T)(1.0 / g.h[1]);
  a.ihz = (T)(1.0 / g.h[2]);
  a.cool = cool_params<T>(g, p);
  a.lim = g.limiter;
  a.rs = g.riemann;
  a.ca = T(0.5);
  a.cb = T(0.5);
  a.epilogue = ((p.flags & MH_SRC_GRAVITY) || c->cool_table()) ? 0 : 1;
  a.dflux = static_cast<const T*>(c->dflux);
  if (p.flags & MH_SRC_FORCING) {
    a.ou_rows = ou_rows;
    for (int k = 0; k < 3; ++k) a.ou_tab[k] = c->at<T>(c->L.tab[k]);
    a.ou_modes = c->nmodes;
    a.ou_R = (int)std::floor(p.ou_kmax);
  }
  return a;
}

// dt_sched (device, or null): the steps take their dt from this schedule,
// entry clk->sched_pos * sched_stride, instead of `dt`
// keep_u1, keep_ub (device, or null; SSP-RK2 only): the first stage writes
// its result to keep_u1 instead of the workspace, and the last stage writes
// its state after the forcing kick to keep_ub, from which the cooling and the
// CFL / health epilogue (or the gravity and tabulated-cooling kernels) finish
// the step; the state left behind is bitwise the plain step's
template <typename T>
static mh_status step_impl(mh_ctx* c, int32_t nsteps, double dt, double t_stop, double* dt_out,
                           const double* dt_sched = nullptr, long long sched_stride = 0,
                           T* keep_u1 = nullptr, T* keep_ub = nullptr) {
  const mh_grid_desc& g = c->g;
  const mh_physics_desc& p = c->p;
  StageGeom geom{g.n[0], g.n[1], g.n[2], {g.bc[0], g.bc[1], g.bc[2]}};
  const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
  const bool force = (p.flags & MH_SRC_FORCING) != 0;
  const bool grav = (p.flags & MH_SRC_GRAVITY) != 0;
  const bool table = c->cool_table();
  // the exact two-branch cooling is fused into the last stage kernel
  const bool cool = (p.flags & MH_SRC_COOLING) != 0 && !table;
  T* U = c->at<T>(c->L.U);
  T* U1 = c->at<T>(c->L.U1);
  const CoolTable<T> ctab = table ? c->cool_table_args<T>() : CoolTable<T>{};
  DevClock* clk = c->clk();
  StageArgs<T> a = base_stage_args<T>(c, clk, c->at<T>(c->L.ou_rows));

  PrologueArgs pa{};
  pa.clk = clk;
  pa.dt_log = c->at<double>(c->L.dtlog);
  pa.f64 = g.dtype == MH_F64;
  pa.dt_fixed = dt;
  pa.cfl = g.cfl;
  pa.ccool = table ? p.cool_ccool : 0.0;
  pa.t_stop = t_stop;
  pa.forcing = force;
  if (force) pa.ou = ou_args(c);
  pa.dt_sched = dt_sched;
  pa.sched_stride = sched_stride;
  const bool cfl = !(dt > 0.0) && !dt_sched;

  MH_HIP(c, launch_clock_reset_health(clk, c->stream));
  for (int s = 0; s < nsteps; ++s) {
    if (!c->smax_valid && cfl) {
      const long tk = time_begin(c, MH_TIME_OTHER);
      MH_HIP(c, launch_smax<T>(U, geom, (T)g.gamma, ih, clk, c->stream));
      if (table && ctab.rate)
        MH_HIP(c, launch_cool_rate<T>(U, geom, (T)g.gamma, ctab, clk, c->stream));
      time_end(c, tk);
      c->smax_valid = true;
    }
    pa.log_index = s % DTLOG_CAP;
    long tk = time_begin(c, MH_TIME_PROLOGUE);
    MH_HIP(c, launch_prologue(pa, c->stream));
    if (force)
      MH_HIP(c, launch_force_rows<T>(c->at<T>(c->L.ou_coef), c->at<int>(c->L.ou_n), c->nmodes,
                                     a.ou_tab[1], a.ou_tab[2], g.n[1], g.n[2], a.ou_R,
                                     c->at<T>(c->L.ou_rows), c->stream));
    time_end(c, tk);
    // all stages but the last
    T* U1s = keep_u1 ? keep_u1 : U1;
    if (g.integrator != MH_RK_EULER) {
      a.uin = U;
      a.un = nullptr;
      a.uout = U1s;
      tk = time_begin(c, MH_TIME_STAGE1);
      MH_HIP(c, launch_stage<T>(1, g.limiter, false, false, a, geom, c->stream));
      time_end(c, tk);
    }
    if (g.integrator == MH_RK_SSP3) {
      T* U2 = c->at<T>(c->L.U2);
      a.uin = U1;
      a.un = U;
      a.uout = U2;
      a.ca = T(0.75);
      a.cb = T(0.25);
      tk = time_begin(c, MH_TIME_OTHER);
      MH_HIP(c, launch_stage<T>(3, g.limiter, false, false, a, geom, c->stream));
      time_end(c, tk);
      a.uin = U2;
      a.uout = U;
      a.ca = T(1.0 / 3.0);
      a.cb = T(2.0 / 3.0);
    } else if (g.integrator == MH_RK_EULER) {
      a.uin = U;  // the lone stage reads U with its stencil, so it writes U1
      a.un = U;
      a.uout = U1;
      a.ca = T(0);
      a.cb = T(1);
    } else {
      a.uin = U1s;
      a.un = U;
      a.uout = U;
    }
    // the last stage, with the sources
    if (keep_ub) {
      // the state after the forcing kick is kept; cooling and the epilogue
      // (or the sources kernels after it) finish the step from it
      StageArgs<T> ak = a;
      ak.uout = keep_ub;
      ak.epilogue = 0;
      tk = time_begin(c, MH_TIME_STAGE2);
      MH_HIP(c, launch_stage<T>(2, g.limiter, force, false, ak, geom, c->stream));
      if (grav || table)
        MH_HIP(c, hipMemcpyAsync(U, keep_ub, 5 * (size_t)c->cells() * sizeof(T),
                                 hipMemcpyDeviceToDevice, c->stream));
      else
        MH_HIP(c, launch_stage2_finish<T>(cool, a, keep_ub, geom, c->stream));
      time_end(c, tk);
    } else if (grav) {
      // forcing fused into the last stage; gravity needs the new density
      // everywhere first, then the kick, cooling and CFL run in the sources
      // kernel
      tk = time_begin(c, MH_TIME_STAGE2);
      MH_HIP(c, launch_stage<T>(2, g.limiter, force, false, a, geom, c->stream));
      time_end(c, tk);
    } else {
      tk = time_begin(c, MH_TIME_STAGE2);
      MH_HIP(c, launch_stage<T>(2, g.limiter, force, cool, a, geom, c->stream));
      time_end(c, tk);
    }
    if (g.integrator == MH_RK_EULER)
      MH_HIP(c, hipMemcpyAsync(U, U1, 5 * (size_t)c->cells() * sizeof(T),
                               hipMemcpyDeviceToDevice, c->stream));
    a.ca = T(0.5);
    a.cb = T(0.5);
    if (grav) {
      tk = time_begin(c, MH_TIME_OTHER);
      MH_HIP(c, mg_gravity_step<T>(c->ws, c->L.mg, c->g, c->p, a.cool, U, clk, !table,
                                   c->stream));
      time_end(c, tk);
    }
    if (table) {
      tk = time_begin(c, MH_TIME_OTHER);
      MH_HIP(c, launch_cool_table<T>(U, geom, (T)g.gamma, ih, ctab, clk, c->stream));
      time_end(c, tk);
    }
    c->smax_valid = true;
    if (dt_out && ((s + 1) % DTLOG_CAP == 0 || s + 1 == nsteps)) {
      const int n0 = (s / DTLOG_CAP) * DTLOG_CAP;
      MH_HIP(c, hipMemcpyAsync(dt_out + n0, pa.dt_log, (size_t)(s + 1 - n0) * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      MH_HIP(c, hipStreamSynchronize(c->stream));
    }
  }
  return MH_OK;
}

extern "C" mh_status mh_step_keep(mh_ctx* c, double dt, void* U1_out, void* Ub_out,
                                  double* dt_out) {
  if (!c || !U1_out || !Ub_out || U1_out == Ub_out) return MH_E_INVALID;
  if (std::isnan(dt)) return set_err(c, MH_E_INVALID, "mh_step_keep: NaN dt");
  if (c->g.integrator != MH_RK_SSP2)
    return set_err(c, MH_E_INVALID, "mh_step_keep: the kept stages are those of SSP-RK2");
  mh_status s = c->g.dtype == MH_F64
                    ? step_impl<double>(c, 1, dt, INFINITY, dt_out, nullptr, 0,
                                        static_cast<double*>(U1_out), static_cast<double*>(Ub_out))
                    : step_impl<float>(c, 1, dt, INFINITY, dt_out, nullptr, 0,
                                       static_cast<float*>(U1_out), static_cast<float*>(Ub_out));
  return s;
}

extern "C" mh_status mh_step(mh_ctx* c, int32_t nsteps, double dt, double t_stop,
                             double* dt_out, double* t_out) {
  if (!c) return MH_E_INVALID;
  if (nsteps < 0) return set_err(c, MH_E_INVALID, "mh_step: nsteps < 0");
  if (std::isnan(dt) || std::isnan(t_stop)) return set_err(c, MH_E_INVALID, "mh_step: NaN dt");
  mh_status s = c->g.dtype == MH_F64 ? step_impl<double>(c, nsteps, dt, t_stop, dt_out)
                                     : step_impl<float>(c, nsteps, dt, t_stop, dt_out);
  if (s != MH_OK) return s;
  if (t_out) {
    DevClock hc;
    MH_HIP(c, hipMemcpyAsync(&hc, c->clk(), sizeof hc, hipMemcpyDeviceToHost, c->stream));
    MH_HIP(c, hipStreamSynchronize(c->stream));
    *t_out = hc.t;
  }
  return MH_OK;
}

// ------------------------------------------------- batched corrected steps

// One corrected step of the B contexts: each context's plain step, the
// gather of the B states into `in`, the corrector's batched pass into `out`,
// the scatter back, and (CFL steps) the signal speed of the corrected states
// for the next step's dt.  The corrector part runs on `main`; with `fork`
// events (a captured step) the plain steps run on the contexts' own streams
// as parallel branches (fork[0] ends the previous work on `main`, fork[1 + b]
// ends context b's step), otherwise on `main` in turn.
template <typename T>
static mh_status corrected_step(mh_ctx* const* ctxs, int B, mh_corr* corr, T* in, T* out,
                                const double* dts, hipStream_t main, const hipEvent_t* fork) {
  const size_t bytes = 5 * (size_t)ctxs[0]->cells() * sizeof(T);
  if (fork) MH_HIP(ctxs[0], hipEventRecord(fork[0], main));
  for (int b = 0; b < B; ++b) {
    if (fork) MH_HIP(ctxs[b], hipStreamWaitEvent(ctxs[b]->stream, fork[0], 0));
    mh_status st = step_impl<T>(ctxs[b], 1, 0.0, INFINITY, nullptr, dts ? dts + b : nullptr, B);
    if (st != MH_OK) return st;
    if (fork) {
      MH_HIP(ctxs[b], hipEventRecord(fork[1 + b], ctxs[b]->stream));
      MH_HIP(ctxs[0], hipStreamWaitEvent(main, fork[1 + b], 0));
    }
  }
  for (int b = 0; b < B; ++b)
    MH_HIP(ctxs[0], launch_copy(ctxs[b]->ws + ctxs[b]->L.U, in + (size_t)b * bytes / sizeof(T),
                                bytes, main));
  MH_HIP(ctxs[0], corr_apply_enqueue(corr, in, out, main));
  for (int b = 0; b < B; ++b)
    MH_HIP(ctxs[0], launch_copy(out + (size_t)b * bytes / sizeof(T), ctxs[b]->ws + ctxs[b]->L.U,
                                bytes, main));
  if (!dts) {
    for (int b = 0; b < B; ++b) {
      mh_ctx* c = ctxs[b];
      const mh_grid_desc& g = c->g;
      StageGeom geom{g.n[0], g.n[1], g.n[2], {g.bc[0], g.bc[1], g.bc[2]}};
      const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
      MH_HIP(c, launch_smax<T>(c->at<T>(c->L.U), geom, (T)g.gamma, ih, c->clk(), main));
    }
  }
  return MH_OK;
}

template <typename T>
static mh_status step_corrected_impl(mh_ctx* const* ctxs, int B, mh_corr* corr, void* stage,
                                     int nsteps, const double* dts, bool graph) {
  mh_ctx* c0 = ctxs[0];
  const size_t per = 5 * (size_t)c0->cells() * (size_t)B;
  T* in = (T*)stage;
  T* out = in + per;
  MH_HIP(c0, corr_fallbacks_reset(corr));
  for (int b = 0; b < B; ++b) {
    MH_HIP(c0, launch_sched_reset(ctxs[b]->clk(), c0->stream));
    if (!dts && !ctxs[b]->smax_valid) {
      // CFL speed of a state that no step has produced yet
      mh_ctx* c = ctxs[b];
      const mh_grid_desc& g = c->g;
      StageGeom geom{g.n[0], g.n[1], g.n[2], {g.bc[0], g.bc[1], g.bc[2]}};
      const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
      MH_HIP(c, launch_smax<T>(c->at<T>(c->L.U), geom, (T)g.gamma, ih, c->clk(), c->stream));
      c->smax_valid = true;
    }
  }
  if (!graph || nsteps == 0) {
    for (int s = 0; s < nsteps; ++s) {
      mh_status st = corrected_step<T>(ctxs, B, corr, in, out, dts, c0->stream, nullptr);
      if (st != MH_OK) return st;
    }
    return MH_OK;
  }
  // One corrected step captured into a graph (kernel nodes only) and replayed
  // on the contexts' stream.  The capture records on streams of its own (the
  // contexts' stream may be the null stream, which cannot capture): the B
  // plain steps on B branch streams, joined before the corrector, so that the
  // graph runs them concurrently (one 64^3 step fills a small part of the
  // GPU).  Nothing runs during the capture.
  const hipStream_t user = c0->stream;
  std::vector<hipStream_t> bs(B + 1, nullptr);
  std::vector<hipEvent_t> ev(B + 1, nullptr);
  hipError_t ec = hipSuccess;
  for (int b = 0; b <= B && ec == hipSuccess; ++b) {
    ec = hipStreamCreateWithFlags(&bs[b], hipStreamNonBlocking);
    if (ec == hipSuccess) ec = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming);
  }
  std::vector<int> timing(B);
  for (int b = 0; b < B; ++b) {
    timing[b] = ctxs[b]->timing;
    ctxs[b]->timing = false;
    ctxs[b]->stream = bs[1 + b];
  }
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  mh_status st = MH_OK;
  if (ec == hipSuccess) ec = hipStreamBeginCapture(bs[0], hipStreamCaptureModeThreadLocal);
  if (ec == hipSuccess) {
    st = corrected_step<T>(ctxs, B, corr, in, out, dts, bs[0], ev.data());
    ec = hipStreamEndCapture(bs[0], &gr);
  }
  for (int b = 0; b < B; ++b) {
    ctxs[b]->timing = timing[b];
    ctxs[b]->stream = user;
  }
  for (int b = 0; b <= B; ++b) {
    if (ev[b]) (void)hipEventDestroy(ev[b]);
    if (bs[b]) (void)hipStreamDestroy(bs[b]);
  }
  if (st != MH_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return st;
  }
  MH_HIP(c0, ec);
  hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  for (int s = 0; e == hipSuccess && s < nsteps; ++s) e = hipGraphLaunch(ex, c0->stream);
  // the executable graph is released once its launches have run
  const hipError_t es = hipStreamSynchronize(c0->stream);
  if (ex) (void)hipGraphExecDestroy(ex);
  (void)hipGraphDestroy(gr);
  MH_HIP(c0, e);
  MH_HIP(c0, es);
  return MH_OK;
}

extern "C" mh_status mh_step_corrected(mh_ctx* const* ctxs, int32_t B, mh_corr* corr,
                                       void* stage, int32_t nsteps, const double* dts,
                                       int32_t use_graph, int64_t* fallbacks) {
  if (!ctxs || B < 1 || !ctxs[0]) return MH_E_INVALID;
  mh_ctx* c0 = ctxs[0];
  if (!corr || !stage || nsteps < 0 || (use_graph != 0 && use_graph != 1))
    return set_err(c0, MH_E_INVALID, "mh_step_corrected: null corrector or stage, nsteps < 0 "
                                     "or use_graph not 0/1");
  const mh_grid_desc& g = c0->g;
  if (g.n[0] != g.n[1] || g.n[0] != g.n[2])
    return set_err(c0, MH_E_SHAPE, "mh_step_corrected: the grid must be a cube");
  for (int b = 0; b < B; ++b) {
    mh_ctx* c = ctxs[b];
    if (!c) return set_err(c0, MH_E_INVALID, "mh_step_corrected: context %d is null", b);
    for (int q = 0; q < b; ++q)
      if (ctxs[q] == c) return set_err(c0, MH_E_INVALID, "mh_step_corrected: context %d repeats", b);
    if (c->g.dtype != g.dtype || c->g.n[0] != g.n[0] || c->g.n[1] != g.n[1] || c->g.n[2] != g.n[2])
      return set_err(c0, MH_E_SHAPE, "mh_step_corrected: context %d differs in grid or dtype", b);
    if (c->stream != c0->stream || corr_stream(corr) != c0->stream)
      return set_err(c0, MH_E_INVALID, "mh_step_corrected: contexts and corrector must share "
                                       "one stream");
    if (use_graph && (c->p.flags & MH_SRC_GRAVITY))
      return set_err(c0, MH_E_UNSUPPORTED, "mh_step_corrected: a captured step cannot hold the "
                                           "gravity solve (its convergence test reads the host)");
  }
  if (!corr_matches(corr, g.n[0], B, g.dtype))
    return set_err(c0, MH_E_SHAPE, "mh_step_corrected: the corrector is not a state corrector "
                                   "of this cube, batch %d and dtype", B);
  mh_status st = g.dtype == MH_F64
                     ? step_corrected_impl<double>(ctxs, B, corr, stage, nsteps, dts, use_graph)
                     : step_corrected_impl<float>(ctxs, B, corr, stage, nsteps, dts, use_graph);
  if (st != MH_OK) return st;
  if (fallbacks) MH_HIP(c0, corr_fallbacks_read(corr, fallbacks));
  return MH_OK;
}

extern "C" mh_status mh_adam(void* theta, void* m, void* v, const void* grad, int64_t count,
                             int32_t dtype, int64_t it, double lr, double beta1, double beta2,
                             double eps, void* stream) {
  if (!theta || !m || !v || !grad || count < 0 || it < 1 || !(lr >= 0.0) ||
      !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return MH_E_INVALID;
  if (count == 0) return MH_OK;
  hipError_t e;
  if (dtype == MH_F64)
    e = launch_adam<double>((double*)theta, (double*)m, (double*)v, (const double*)grad, count,
                            lr, beta1, beta2, eps, it, (hipStream_t)stream);
  else if (dtype == MH_F32)
    e = launch_adam<float>((float*)theta, (float*)m, (float*)v, (const float*)grad, count, lr,
                           beta1, beta2, eps, it, (hipStream_t)stream);
  else
    return MH_E_DTYPE;
  return e == hipSuccess ? MH_OK : MH_E_DEVICE;
}

extern "C" mh_status mh_get_clock(mh_ctx* c, double* t, int64_t* step) {
  if (!c) return MH_E_INVALID;
  DevClock hc;
  MH_HIP(c, hipMemcpyAsync(&hc, c->clk(), sizeof hc, hipMemcpyDeviceToHost, c->stream));
  MH_HIP(c, hipStreamSynchronize(c->stream));
  if (t) *t = hc.t;
  if (step) *step = hc.step;
  return MH_OK;
}

extern "C" mh_status mh_set_clock(mh_ctx* c, double t, int64_t step) {
  if (!c) return MH_E_INVALID;
  if (!std::isfinite(t) || step < 0) return set_err(c, MH_E_INVALID, "mh_set_clock: bad value");
  MH_HIP(c, launch_clock_set(c->clk(), t, step, c->stream));
  return MH_OK;
}

extern "C" mh_status mh_get_ou_state(mh_ctx* c, int32_t* nmodes, double* ahat) {
  if (!c) return MH_E_INVALID;
  if (nmodes) *nmodes = c->nmodes;
  if (ahat && c->nmodes > 0) {
    MH_HIP(c, hipMemcpyAsync(ahat, c->ws + c->L.ou_ahat, 6 * c->nmodes * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    MH_HIP(c, hipStreamSynchronize(c->stream));
  }
  return MH_OK;
}

extern "C" mh_status mh_set_ou_state(mh_ctx* c, const double* ahat) {
  if (!c) return MH_E_INVALID;
  if (c->nmodes == 0) return set_err(c, MH_E_INVALID, "mh_set_ou_state: forcing is off");
  if (!ahat) return set_err(c, MH_E_INVALID, "mh_set_ou_state: null pointer");
  MH_HIP(c, hipMemcpyAsync(c->ws + c->L.ou_ahat, ahat, 6 * c->nmodes * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  MH_HIP(c, hipStreamSynchronize(c->stream));
  return MH_OK;
}

extern "C" mh_status mh_check(mh_ctx* c, int64_t* bad_cells, int64_t* first_bad) {
  if (!c) return MH_E_INVALID;
  DevClock hc;
  MH_HIP(c, hipMemcpyAsync(&hc, c->clk(), sizeof hc, hipMemcpyDeviceToHost, c->stream));
  MH_HIP(c, hipStreamSynchronize(c->stream));
  if (bad_cells) *bad_cells = (int64_t)hc.bad_count;
  const int64_t fb = hc.bad_count ? (int64_t)hc.bad_first : -1;
  if (first_bad) *first_bad = fb;
  if (hc.bad_count)
    return set_err(c, MH_E_NONFINITE, "%llu unphysical cell(s); first at flat index %lld",
                   (unsigned long long)hc.bad_count, (long long)fb);
  return MH_OK;
}

extern "C" mh_status mh_last_mg_cycles(mh_ctx* c, int32_t* cycles) {
  if (!c || !cycles) return MH_E_INVALID;
  DevClock hc;
  MH_HIP(c, hipMemcpyAsync(&hc, c->clk(), sizeof hc, hipMemcpyDeviceToHost, c->stream));
  MH_HIP(c, hipStreamSynchronize(c->stream));
  *cycles = hc.mg_cycles;
  return MH_OK;
}

extern "C" mh_status mh_get_potential(mh_ctx* c, void* phi, int where) {
  if (!c) return MH_E_INVALID;
  if (!(c->p.flags & MH_SRC_GRAVITY))
    return set_err(c, MH_E_INVALID, "mh_get_potential: gravity is off");
  if (!phi || (where != MH_HOST && where != MH_DEVICE))
    return set_err(c, MH_E_INVALID, "mh_get_potential: null pointer or bad location");
  MH_HIP(c, hipMemcpyAsync(phi, c->ws + mg_phi_offset(c->L.mg), (size_t)c->cells() * c->esize(),
                           where == MH_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           c->stream));
  if (where == MH_HOST) MH_HIP(c, hipStreamSynchronize(c->stream));
  return MH_OK;
}

// ------------------------------------------------------------------ adjoint

namespace {

struct AdjLayout {
  size_t clk = 0, dtlog = 0, U1 = 0, U2 = 0, Ua = 0, Uc = 0, lamA = 0, lamB = 0;
  size_t lam1 = 0, lam2 = 0;
  size_t Wacc = 0, wbar = 0, flags = 0, accb = 0, phib = 0, ahat = 0, coef = 0, rows = 0;
  MGLayout mg;
  size_t total = 0;
};

AdjLayout make_adj_layout(const mh_grid_desc& g, const mh_physics_desc& p) {
  AdjLayout A;
  const size_t es = g.dtype == MH_F64 ? 8 : 4;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  size_t faces = 0;
  for (int a = 0; a < 3; ++a) {
    const size_t nf = g.bc[a] == MH_BC_PERIODIC ? g.n[a] : g.n[a] + 1;
    const size_t f = nf * (N / g.n[a]);
    if (f > faces) faces = f;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  A.clk = take(sizeof(DevClock));
  A.dtlog = take(sizeof(double));
  A.U1 = take(5 * N * es);
  A.Ua = take(5 * N * es);
  if (p.flags & MH_SRC_GRAVITY) A.Uc = take(5 * N * es);  // the state after the gravity kick
  A.lamA = take(5 * N * es);
  A.lamB = take(5 * N * es);
  A.lam1 = take(5 * N * es);
  if (g.integrator == MH_RK_SSP3) {
    A.U2 = take(5 * N * es);
    A.lam2 = take(5 * N * es);
  }
  A.Wacc = take(5 * N * es);
  A.wbar = take((adj_runtime_scheme(g.limiter, g.riemann) ? 20 : 10) * faces * es);
  A.flags = take(faces * sizeof(int));
  if (p.flags & MH_SRC_FORCING) {
    const int R = (int)std::floor(p.ou_kmax);
    A.ahat = take(6 * MAX_MODES * sizeof(double));
    A.coef = take(6 * MAX_MODES * es);
    A.rows = take((size_t)g.n[1] * g.n[2] * (R + 1) * 6 * es);
  }
  if (p.flags & MH_SRC_GRAVITY) {
    A.accb = take(3 * N * es);
    A.phib = take(N * es);
    off = mg_layout(&g, &p, off, es, A.mg);
  }
  A.total = off;
  return A;
}

}  // namespace

extern "C" mh_status mh_query_adjoint_workspace(mh_ctx* c, size_t* bytes) {
  if (!c || !bytes) return MH_E_INVALID;
  *bytes = make_adj_layout(c->g, c->p).total;
  return MH_OK;
}

// kept_u1, kept_ub (or null): the step's first-stage result and its state
// after the forcing kick, kept by mh_step_keep; the recomputation of the two
// stages is skipped.  kept_phi (or null): the potential the step's multigrid
// solve returned; the solve is skipped
template <typename T>
static mh_status adjoint_impl(mh_ctx* c, char* ws, AdjLayout& A, const T* Un, double dt,
                              int64_t step, const double* ou_ahat, const T* phi_n,
                              const T* lam_np1, T* lam_n, const T* kept_u1 = nullptr,
                              const T* kept_ub = nullptr, const T* kept_phi = nullptr) {
  const mh_grid_desc& g = c->g;
  const mh_physics_desc& p = c->p;
  const bool force = (p.flags & MH_SRC_FORCING) != 0;
  const bool grav = (p.flags & MH_SRC_GRAVITY) != 0;
  const bool cool = (p.flags & MH_SRC_COOLING) != 0;
  const long long N = c->cells();
  const size_t sbytes = 5 * (size_t)N * sizeof(T);
  StageGeom geom{g.n[0], g.n[1], g.n[2], {g.bc[0], g.bc[1], g.bc[2]}};
  auto at = [&](size_t off) { return reinterpret_cast<T*>(ws + off); };
  DevClock* aclk = reinterpret_cast<DevClock*>(ws + A.clk);
  T *U1 = at(A.U1), *Ua = at(A.Ua), *Ub = nullptr, *Uc = nullptr;
  T *lamA = at(A.lamA), *lamB = at(A.lamB), *lam1 = at(A.lam1);
  AdjointBuffers<T> B{at(A.Wacc), at(A.wbar), reinterpret_cast<int*>(ws + A.flags),
                      grav ? at(A.accb) : nullptr, grav ? at(A.phib) : nullptr};

  // private clock at the step being differentiated; the OU amplitudes of the
  // step start from the caller's copy
  DevClock hc{};
  hc.step = step;
  hc.bad_first = ~0ull;
  MH_HIP(c, hipMemcpyAsync(aclk, &hc, sizeof hc, hipMemcpyHostToDevice, c->stream));
  PrologueArgs pa{};
  pa.clk = aclk;
  pa.dt_log = reinterpret_cast<double*>(ws + A.dtlog);
  pa.f64 = g.dtype == MH_F64;
  pa.dt_fixed = dt;
  pa.cfl = g.cfl;
  pa.t_stop = INFINITY;
  pa.forcing = force;
  if (force) {
    MH_HIP(c, hipMemcpyAsync(ws + A.ahat, ou_ahat, 6 * c->nmodes * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    pa.ou = ou_args(c);
    pa.ou.clk = aclk;
    pa.ou.ahat = reinterpret_cast<double*>(ws + A.ahat);
    pa.ou.coef = ws + A.coef;
  }
  MH_HIP(c, launch_prologue(pa, c->stream));
  StageArgs<T> a = base_stage_args<T>(c, aclk, force ? at(A.rows) : nullptr);
  if (force)
    MH_HIP(c, launch_force_rows<T>(at(A.coef), c->at<int>(c->L.ou_n), c->nmodes, a.ou_tab[1],
                                   a.ou_tab[2], g.n[1], g.n[2], a.ou_R, at(A.rows), c->stream));

  // forward recomputation: U1 (and U2), Ua (the RK update), Ub (after the
  // forcing kick), Uc (after the gravity kick)
  T* U2 = g.integrator == MH_RK_SSP3 ? at(A.U2) : nullptr;
  if (kept_u1) {
    // the stages kept by the forward step (SSP-RK2): U1 and the state after
    // the forcing kick, read only
    U1 = const_cast<T*>(kept_u1);
    Ua = const_cast<T*>(kept_ub);
  } else if (g.integrator == MH_RK_EULER) {
    a.uin = Un;
    a.un = Un;
    a.ca = T(0);
    a.cb = T(1);
  } else {
    a.uin = Un;
    a.un = nullptr;
    a.uout = U1;
    MH_HIP(c, launch_stage<T>(1, g.limiter, false, false, a, geom, c->stream));
    a.uin = U1;
    a.un = Un;
  }
  if (U2) {
    a.uout = U2;
    a.ca = T(0.75);
    a.cb = T(0.25);
    MH_HIP(c, launch_stage<T>(3, g.limiter, false, false, a, geom, c->stream));
    a.uin = U2;
    a.ca = T(1.0 / 3.0);
    a.cb = T(2.0 / 3.0);
  }
  // the last stage applies the forcing kick as the forward step does (the RK
  // update itself is not read again), so Ua is the state after forcing,
  // bitwise; only gravity needs the states before (Ub) and after (Uc) a kick
  if (!kept_u1) {
    a.uout = Ua;
    MH_HIP(c, launch_stage<T>(2, g.limiter, force, false, a, geom, c->stream));
  }
  Ub = Ua;
  Uc = Ub;
  if (grav) {
    Uc = at(A.Uc);
    MH_HIP(c, hipMemcpyAsync(Uc, Ub, sbytes, hipMemcpyDeviceToDevice, c->stream));
  }
  const T* phi_sol = nullptr;
  if (grav) {
    if (kept_phi && !A.mg.fft) {
      // the solve from phi_n on Ub would return these bits
      MH_HIP(c, mg_set_guess<T>(ws, A.mg, kept_phi, c->stream));
    } else {
      MH_HIP(c, mg_set_guess<T>(ws, A.mg, phi_n, c->stream));
      MH_HIP(c, mg_set_rhs<T>(ws, A.mg, Ub, 4.0 * M_PI * p.grav_G, aclk, c->stream));
      MH_HIP(c, mg_solve<T>(ws, A.mg, p, aclk, nullptr, c->stream));
    }
    MH_HIP(c, mg_kick<T>(ws, A.mg, g, Uc, aclk, c->stream));
    phi_sol = reinterpret_cast<const T*>(ws + mg_phi_offset(A.mg));
  }

  // reverse sweep: cooling, gravity, forcing, then the RK update
  const T* cur = lam_np1;
  // without gravity, exact cooling and forcing reverse in one pass
  const bool cool_force = cool && force && !grav && !c->cool_table();
  if (cool_force) {
    MH_HIP(c, adj_cool_force_vjp<T>(Uc, (T)(g.gamma - 1.0), (T)dt, a.cool, at(A.rows),
                                    a.ou_tab[0], a.ou_R, geom, cur, lamA, c->stream));
    cur = lamA;
  } else if (cool) {
    if (c->cool_table())
      MH_HIP(c, launch_cool_table_vjp<T>(Uc, N, (T)g.gamma, (T)dt, c->cool_table_args<T>(), cur,
                                         lamA, c->stream));
    else
      MH_HIP(c, adj_cool_vjp<T>(Uc, N, (T)(g.gamma - 1.0), (T)dt, a.cool, cur, lamA, c->stream));
    cur = lamA;
  }
  if (grav) {
    MH_HIP(c, adj_gravity_vjp<T>(B, A.mg, ws, p, Ub, phi_sol, g.n[0], g.h[0], (T)dt, cur, lamB,
                                 aclk, c->stream));
    cur = lamB;
  }
  if (force && !cool_force) {
    T* dst = cur == lamA ? lamB : lamA;
    MH_HIP(c, adj_force_kick_vjp<T>(at(A.rows), a.ou_tab[0], a.ou_R, geom, (T)dt, cur, dst,
                                    c->stream));
    cur = dst;
  }
  const int lim = g.limiter;
  const T gam = (T)g.gamma;
  T* gflux = static_cast<T*>(c->dflux_grad);
  if (g.integrator == MH_RK_EULER) {
    // lam_n = cur + dt J(U^n)^T cur
    if (gflux) MH_HIP(c, adj_flux_corr_vjp<T>(cur, geom, g.h, dt, gflux, c->stream));
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, Un, cur, (T)dt, T(1), cur, T(0), nullptr, T(0),
                         nullptr, lam_n, c->stream));
  } else if (g.integrator == MH_RK_SSP3) {
    // lam2 = 2/3 (cur + dt J(U2)^T cur);  lam1 = 1/4 (lam2 + dt J(U1)^T lam2);
    // lam_n = cur/3 + 3/4 lam2 + lam1 + dt J(U^n)^T lam1
    T* lam2 = at(A.lam2);
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, U2, cur, (T)(2.0 / 3.0 * dt), (T)(2.0 / 3.0),
                         cur, T(0), nullptr, T(0), nullptr, lam2, c->stream));
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, U1, lam2, (T)(0.25 * dt), T(0.25), lam2, T(0),
                         nullptr, T(0), nullptr, lam1, c->stream));
    if (gflux) {
      MH_HIP(c, adj_flux_corr_vjp<T>(cur, geom, g.h, 2.0 / 3.0 * dt, gflux, c->stream));
      MH_HIP(c, adj_flux_corr_vjp<T>(lam2, geom, g.h, 0.25 * dt, gflux, c->stream));
      MH_HIP(c, adj_flux_corr_vjp<T>(lam1, geom, g.h, dt, gflux, c->stream));
    }
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, Un, lam1, (T)dt, (T)(1.0 / 3.0), cur, T(0.75),
                         lam2, T(1), lam1, lam_n, c->stream));
  } else {
    // lam1 = cur/2 + (dt/2) J(U1)^T cur;  lam_n = cur/2 + lam1 + dt J(U^n)^T lam1
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, U1, cur, (T)(0.5 * dt), T(0.5), cur, T(0),
                         nullptr, T(0), nullptr, lam1, c->stream));
    if (gflux) {
      MH_HIP(c, adj_flux_corr_vjp<T>(cur, geom, g.h, 0.5 * dt, gflux, c->stream));
      MH_HIP(c, adj_flux_corr_vjp<T>(lam1, geom, g.h, dt, gflux, c->stream));
    }
    MH_HIP(c, adj_jtv<T>(B, geom, lim, g.riemann, gam, g.h, Un, lam1, (T)dt, T(0.5), cur, T(1), lam1, T(0),
                         nullptr, lam_n, c->stream));
  }
  return MH_OK;
}

extern "C" mh_status mh_adjoint_step(mh_ctx* c, void* adj_workspace, size_t adj_workspace_bytes,
                                     const void* U_n, double dt, int64_t step,
                                     const double* ou_ahat, const void* phi_n,
                                     const void* lam_np1, void* lam_n) {
  if (!c) return MH_E_INVALID;
  if (!U_n || !lam_np1 || !lam_n)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step: null state or adjoint pointer");
  if ((c->p.flags & MH_SRC_FORCING) && !ou_ahat)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step: forcing is on but ou_ahat is NULL");
  if (!(dt >= 0.0) || step < 0) return set_err(c, MH_E_INVALID, "mh_adjoint_step: bad dt or step");
  AdjLayout A = make_adj_layout(c->g, c->p);
  A.mg.graphs = &c->adj_graphs;
  if (!adj_workspace || adj_workspace_bytes < A.total || ((uintptr_t)adj_workspace % ALIGN) != 0)
    return set_err(c, MH_E_WORKSPACE, "mh_adjoint_step: adjoint workspace too small or misaligned");
  char* ws = (char*)adj_workspace;
  if (c->g.dtype == MH_F64)
    return adjoint_impl<double>(c, ws, A, (const double*)U_n, dt, step, ou_ahat,
                                (const double*)phi_n, (const double*)lam_np1, (double*)lam_n);
  return adjoint_impl<float>(c, ws, A, (const float*)U_n, dt, step, ou_ahat, (const float*)phi_n,
                             (const float*)lam_np1, (float*)lam_n);
}

extern "C" mh_status mh_adjoint_step_kept(mh_ctx* c, void* adj_workspace,
                                          size_t adj_workspace_bytes, const void* U_n,
                                          const void* U1, const void* Ub, double dt, int64_t step,
                                          const double* ou_ahat, const void* phi_n,
                                          const void* phi_np1, const void* lam_np1,
                                          void* lam_n) {
  if (!c) return MH_E_INVALID;
  if (!U_n || !U1 || !Ub || !lam_np1 || !lam_n)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step_kept: null state or adjoint pointer");
  if (c->g.integrator != MH_RK_SSP2)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step_kept: the kept stages are those of SSP-RK2");
  if ((c->p.flags & MH_SRC_FORCING) && !ou_ahat)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step_kept: forcing is on but ou_ahat is NULL");
  if (!(dt >= 0.0) || step < 0)
    return set_err(c, MH_E_INVALID, "mh_adjoint_step_kept: bad dt or step");
  AdjLayout A = make_adj_layout(c->g, c->p);
  A.mg.graphs = &c->adj_graphs;
  if (!adj_workspace || adj_workspace_bytes < A.total || ((uintptr_t)adj_workspace % ALIGN) != 0)
    return set_err(c, MH_E_WORKSPACE,
                   "mh_adjoint_step_kept: adjoint workspace too small or misaligned");
  char* ws = (char*)adj_workspace;
  if (c->g.dtype == MH_F64)
    return adjoint_impl<double>(c, ws, A, (const double*)U_n, dt, step, ou_ahat,
                                (const double*)phi_n, (const double*)lam_np1, (double*)lam_n,
                                (const double*)U1, (const double*)Ub, (const double*)phi_np1);
  return adjoint_impl<float>(c, ws, A, (const float*)U_n, dt, step, ou_ahat, (const float*)phi_n,
                             (const float*)lam_np1, (float*)lam_n, (const float*)U1,
                             (const float*)Ub, (const float*)phi_np1);
}

extern "C" mh_status mh_set_timing(mh_ctx* c, int enable) {
  if (!c) return MH_E_INVALID;
  c->timing = enable != 0;
  return MH_OK;
}

extern "C" mh_status mh_get_timing(mh_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return MH_E_INVALID;
  MH_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < MH_TIME_KINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (size_t i = 0; i < c->kinds.size(); ++i) {
    float t = 0.0f;
    MH_HIP(c, hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]));
    ms[c->kinds[i]] += (double)t;
    launches[c->kinds[i]] += 1;
  }
  launches[MH_TIME_OTHER] += c->untimed;
  c->kinds.clear();
  c->untimed = 0;
  return MH_OK;
}

extern "C" mh_status mh_set_potential(mh_ctx* c, const void* phi, int where) {
  if (!c) return MH_E_INVALID;
  if (!(c->p.flags & MH_SRC_GRAVITY))
    return set_err(c, MH_E_INVALID, "mh_set_potential: gravity is off");
  if (!phi || (where != MH_HOST && where != MH_DEVICE))
    return set_err(c, MH_E_INVALID, "mh_set_potential: null pointer or bad location");
  MH_HIP(c, hipMemcpyAsync(c->ws + mg_phi_offset(c->L.mg), phi, (size_t)c->cells() * c->esize(),
                           where == MH_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->stream));
  if (where == MH_HOST) MH_HIP(c, hipStreamSynchronize(c->stream));
  return MH_OK;
}

extern "C" const char* mh_last_error(const mh_ctx* c) { return c ? c->err.c_str() : ""; }

extern "C" mh_status mh_set_flux_correction(mh_ctx* c, const void* field, void* grad) {
  if (!c) return MH_E_INVALID;
  if (!field && grad)
    return set_err(c, MH_E_INVALID, "mh_set_flux_correction: a gradient buffer needs a field");
  c->dflux = field;
  c->dflux_grad = grad;
  return MH_OK;
}

extern "C" mh_status mh_set_graphs(mh_ctx* c, int enable) {
  if (!c) return MH_E_INVALID;
  MH_HIP(c, hipStreamSynchronize(c->stream));
  for (MGGraphCache* G : {&c->mg_graphs, &c->adj_graphs}) {
    G->enabled = enable != 0;
    if (!G->enabled) G->reset();
  }
  return MH_OK;
}

extern "C" void mh_destroy(mh_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  c->mg_graphs.destroy();
  c->adj_graphs.destroy();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}
