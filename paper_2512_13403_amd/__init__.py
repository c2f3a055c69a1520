"""mihydro: MI355X (gfx950) finite-volume step of diffhydro (arXiv 2512.13403).

Thin Python binding of the C ABI in ``include/mihydro.h`` (``libmihydro.so``,
built in-tree by ``build.py``).  The binding only marshals arguments: every
step of the method runs in the library's HIP kernels.  PyTorch provides the
device memory (the workspace is a torch uint8 tensor) and the stream.  There
is no CPU fallback: constructing a ``Solver`` without the built library or
without a GPU raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmihydro.so")

OK, E_INVALID, E_SHAPE, E_DTYPE, E_DEVICE, E_NONFINITE, E_UNSUPPORTED, E_WORKSPACE = range(8)
STATUS_NAMES = ["MH_OK", "MH_E_INVALID", "MH_E_SHAPE", "MH_E_DTYPE", "MH_E_DEVICE",
                "MH_E_NONFINITE", "MH_E_UNSUPPORTED", "MH_E_WORKSPACE"]
BC_PERIODIC, BC_OUTFLOW = 0, 1
F32, F64 = 0, 1
LIM_MINMOD, LIM_NONE, LIM_VANLEER, LIM_MC, LIM_SUPERBEE = 0, 1, 2, 3, 4
RS_HLLC, RS_HLL, RS_RUSANOV = 0, 1, 2
RK_SSP2, RK_SSP3, RK_EULER = 0, 1, 2
MG_V, MG_W = 0, 1
SMOOTH_JACOBI, SMOOTH_RBGS = 0, 1
GRAV_MG, GRAV_FFT = 0, 1
CORR_STATE, CORR_FLUX = 0, 1
COOL_EXACT2, COOL_TABLE = 0, 1
COOLINT_TRAPEZOID, COOLINT_SUBCYCLE, COOLINT_AUTO = 0, 1, 2
COOL_TABMAX = 64
SRC_COOLING, SRC_FORCING, SRC_GRAVITY = 1, 2, 4
HOST, DEVICE = 0, 1

EXPORTED = [
    "mh_query_workspace", "mh_init", "mh_set_state", "mh_get_state", "mh_step", "mh_get_clock",
    "mh_set_clock", "mh_get_ou_state", "mh_set_ou_state", "mh_check", "mh_last_mg_cycles",
    "mh_get_potential", "mh_set_potential", "mh_set_timing", "mh_get_timing",
    "mh_query_adjoint_workspace", "mh_adjoint_step", "mh_last_error", "mh_destroy",
    "mh_corr_query_workspace", "mh_corr_init", "mh_corr_set_params", "mh_corr_get_params",
    "mh_corr_apply", "mh_corr_loss_grad", "mh_corr_train_step", "mh_corr_get_activation",
    "mh_corr_destroy", "mh_block_average", "mh_corr_zero_grad", "mh_corr_backward",
    "mh_corr_adam_step", "mh_corr_get_grad", "mh_set_graphs", "mh_fft3_query_workspace",
    "mh_fft3", "mh_set_flux_correction", "mh_fft3_noalloc", "mh_step_corrected", "mh_adam",
    "mh_step_keep", "mh_adjoint_step_kept",
]
TIME_STAGE1, TIME_STAGE2, TIME_PROLOGUE, TIME_OTHER = range(4)


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3), ("bc", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3),
        ("dtype", ctypes.c_int32), ("limiter", ctypes.c_int32), ("riemann", ctypes.c_int32),
        ("integrator", ctypes.c_int32), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
    ]


class PhysicsDesc(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32), ("ou_every", ctypes.c_int32),
        ("cool_lambda0", ctypes.c_double), ("cool_tc", ctypes.c_double),
        ("cool_ts", ctypes.c_double), ("cool_tfloor", ctypes.c_double),
        ("ou_seed", ctypes.c_uint64), ("ou_tau", ctypes.c_double), ("ou_arms", ctypes.c_double),
        ("ou_zeta", ctypes.c_double), ("ou_kmin", ctypes.c_double), ("ou_kmax", ctypes.c_double),
        ("grav_G", ctypes.c_double), ("mg_pre", ctypes.c_int32), ("mg_post", ctypes.c_int32),
        ("mg_max_cycles", ctypes.c_int32), ("mg_coarsest", ctypes.c_int32),
        ("mg_tol", ctypes.c_double), ("mg_coarse_sweeps", ctypes.c_int32),
        ("mg_cycle", ctypes.c_int32), ("mg_smoother", ctypes.c_int32),
        ("grav_solver", ctypes.c_int32), ("cool_model", ctypes.c_int32),
        ("cool_integrator", ctypes.c_int32), ("cool_nsub_max", ctypes.c_int32),
        ("cool_ntab", ctypes.c_int32), ("cool_frac", ctypes.c_double),
        ("cool_ccool", ctypes.c_double), ("cool_L1", ctypes.c_double),
        ("cool_a1", ctypes.c_double), ("cool_L2", ctypes.c_double), ("cool_a2", ctypes.c_double),
        ("cool_heat", ctypes.c_double), ("cool_logT", ctypes.c_double * 64),
        ("cool_logL", ctypes.c_double * 64),
    ]


class CorrDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("batch", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("gamma", ctypes.c_double),
        ("mean", ctypes.c_double * 5), ("std", ctypes.c_double * 5),
        ("scale", ctypes.c_double * 5), ("loss_w", ctypes.c_double * 5),
        ("floor_rel", ctypes.c_double), ("fallback_frac", ctypes.c_double),
    ]


class MHError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


_lib = None


def load_library():
    """Loads libmihydro.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "mh_query_workspace": [ctypes.POINTER(GridDesc), ctypes.POINTER(PhysicsDesc),
                                   ctypes.POINTER(ctypes.c_size_t)],
            "mh_init": [ctypes.POINTER(GridDesc), ctypes.POINTER(PhysicsDesc), vp, ctypes.c_size_t,
                        vp, ctypes.POINTER(vp)],
            "mh_set_state": [vp, vp, ctypes.c_int],
            "mh_get_state": [vp, vp, ctypes.c_int],
            "mh_step": [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, dp, dp],
            "mh_get_clock": [vp, dp, i64p],
            "mh_set_clock": [vp, ctypes.c_double, ctypes.c_int64],
            "mh_get_ou_state": [vp, ctypes.POINTER(ctypes.c_int32), dp],
            "mh_set_ou_state": [vp, dp],
            "mh_check": [vp, i64p, i64p],
            "mh_last_mg_cycles": [vp, ctypes.POINTER(ctypes.c_int32)],
            "mh_get_potential": [vp, vp, ctypes.c_int],
            "mh_set_timing": [vp, ctypes.c_int],
            "mh_get_timing": [vp, dp, i64p],
            "mh_set_potential": [vp, vp, ctypes.c_int],
            "mh_query_adjoint_workspace": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "mh_adjoint_step": [vp, vp, ctypes.c_size_t, vp, ctypes.c_double, ctypes.c_int64, dp,
                                vp, vp, vp],
            "mh_step_keep": [vp, ctypes.c_double, vp, vp, dp],
            "mh_adjoint_step_kept": [vp, vp, ctypes.c_size_t, vp, vp, vp, ctypes.c_double,
                                     ctypes.c_int64, dp, vp, vp, vp, vp],
            "mh_corr_query_workspace": [ctypes.POINTER(CorrDesc), ctypes.POINTER(ctypes.c_size_t)],
            "mh_corr_init": [ctypes.POINTER(CorrDesc), vp, ctypes.c_size_t, vp,
                             ctypes.POINTER(vp)],
            "mh_corr_set_params": [vp, vp, ctypes.c_int],
            "mh_corr_get_params": [vp, vp, ctypes.c_int],
            "mh_corr_apply": [vp, vp, vp, i64p, ctypes.POINTER(ctypes.c_int32)],
            "mh_corr_loss_grad": [vp, vp, vp, dp, vp, ctypes.c_int],
            "mh_corr_train_step": [vp, vp, vp, ctypes.c_float, dp],
            "mh_corr_get_activation": [vp, ctypes.c_int, vp, ctypes.c_int],
            "mh_block_average": [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32, vp],
            "mh_corr_zero_grad": [vp],
            "mh_set_graphs": [vp, ctypes.c_int],
            "mh_corr_backward": [vp, vp, vp, vp, dp, vp],
            "mh_corr_adam_step": [vp, ctypes.c_float],
            "mh_corr_get_grad": [vp, vp, ctypes.c_int],
            "mh_fft3_query_workspace": [ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_size_t)],
            "mh_fft3": [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_size_t,
                        vp],
            "mh_set_flux_correction": [vp, vp, vp],
            "mh_fft3_noalloc": [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp],
            "mh_step_corrected": [ctypes.POINTER(vp), ctypes.c_int32, vp, vp, ctypes.c_int32,
                                  vp, ctypes.c_int32, i64p],
            "mh_adam": [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.mh_last_error.argtypes = [vp]
        L.mh_last_error.restype = ctypes.c_char_p
        L.mh_destroy.argtypes = [vp]
        L.mh_destroy.restype = None
        L.mh_corr_destroy.argtypes = [vp]
        L.mh_corr_destroy.restype = None
        _lib = L
    return _lib


def grid_desc(shape, h, bc=(BC_PERIODIC,) * 3, dtype="f32", gamma=5.0 / 3.0, cfl=0.4,
              limiter=LIM_MINMOD, riemann=RS_HLLC, integrator=RK_SSP2) -> GridDesc:
    """shape = (nz, ny, nx); h and bc per (x, y, z); integrator RK_SSP2 (default),
    RK_SSP3 or RK_EULER."""
    g = GridDesc()
    nz, ny, nx = shape
    g.n[:] = [nx, ny, nz]
    g.bc[:] = list(bc)
    g.h[:] = list(h)
    g.dtype = F64 if dtype in ("f64", "float64", F64) else F32
    g.limiter, g.riemann, g.gamma, g.cfl = limiter, riemann, gamma, cfl
    g.integrator = integrator
    return g


def physics_desc(flags=0, cool=(0.3, 1e-2, 1e-3, 1e-4), ou_seed=0, ou_tau=0.5, ou_arms=1.0,
                 ou_zeta=1.0, ou_kmin=1.0, ou_kmax=2.0, ou_every=1, grav_G=0.0, mg_pre=2,
                 mg_post=2, mg_max_cycles=20, mg_coarsest=4, mg_tol=1e-10,
                 mg_coarse_sweeps=200, mg_cycle=MG_V, mg_smoother=SMOOTH_RBGS,
                 grav_solver=GRAV_MG, cool_model=COOL_EXACT2, cool_integrator=COOLINT_TRAPEZOID,
                 cool_nsub_max=1000, cool_frac=0.1, cool_ccool=0.0,
                 cool_ki=(0.0, 0.0, 0.0, 0.0), cool_heat=0.0, cool_table=None) -> PhysicsDesc:
    """cool_table: (log10 T, log10 Lambda) arrays of the tabulated model."""
    p = PhysicsDesc()
    p.flags = flags
    p.cool_lambda0, p.cool_tc, p.cool_ts, p.cool_tfloor = cool
    p.ou_seed, p.ou_tau, p.ou_arms, p.ou_zeta = ou_seed, ou_tau, ou_arms, ou_zeta
    p.ou_kmin, p.ou_kmax, p.ou_every = ou_kmin, ou_kmax, ou_every
    p.grav_G = grav_G
    p.mg_pre, p.mg_post, p.mg_max_cycles, p.mg_coarsest = mg_pre, mg_post, mg_max_cycles, mg_coarsest
    p.mg_tol, p.mg_coarse_sweeps = mg_tol, mg_coarse_sweeps
    p.mg_cycle, p.mg_smoother, p.grav_solver = mg_cycle, mg_smoother, grav_solver
    p.cool_model, p.cool_integrator, p.cool_nsub_max = cool_model, cool_integrator, cool_nsub_max
    p.cool_frac, p.cool_ccool, p.cool_heat = cool_frac, cool_ccool, cool_heat
    p.cool_L1, p.cool_a1, p.cool_L2, p.cool_a2 = cool_ki
    if cool_table is not None:
        logT, logL = cool_table
        if len(logT) != len(logL) or not 2 <= len(logT) <= COOL_TABMAX:
            raise ValueError("cool_table needs 2..64 matching (log10 T, log10 Lambda) points")
        p.cool_ntab = len(logT)
        p.cool_logT[:len(logT)] = [float(v) for v in logT]
        p.cool_logL[:len(logL)] = [float(v) for v in logL]
    return p


def query_workspace(grid: GridDesc, phys: PhysicsDesc) -> int:
    L = load_library()
    n = ctypes.c_size_t(0)
    st = L.mh_query_workspace(ctypes.byref(grid), ctypes.byref(phys), ctypes.byref(n))
    if st != OK:
        raise MHError(st, "mh_query_workspace rejected the descriptors")
    return n.value


class Solver:
    """One simulation on one GPU: owns a torch workspace tensor and an mh_ctx."""

    def __init__(self, grid: GridDesc, phys: PhysicsDesc | None = None, device="cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("mihydro needs a GPU (no CPU fallback)")
        self._torch = torch
        self.lib = load_library()
        self.grid = grid
        self.phys = phys if phys is not None else physics_desc()
        self.device = torch.device(device)
        self.shape = (grid.n[2], grid.n[1], grid.n[0])
        self.np_dtype = np.float64 if grid.dtype == F64 else np.float32
        self.torch_dtype = torch.float64 if grid.dtype == F64 else torch.float32
        nbytes = query_workspace(grid, self.phys)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            ctx = ctypes.c_void_p()
            st = self.lib.mh_init(ctypes.byref(grid), ctypes.byref(self.phys),
                                  ctypes.c_void_p(aligned), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != OK:
            raise MHError(st, "mh_init failed")
        self.ctx = ctx

    # -- helpers
    def _check(self, st, what):
        if st != OK:
            raise MHError(st, f"{what}: {self.lib.mh_last_error(self.ctx).decode()}")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state
    def set_state(self, U):
        torch = self._torch
        if isinstance(U, torch.Tensor) and U.is_cuda:
            t = U.to(self.torch_dtype).contiguous()
            assert tuple(t.shape) == (5,) + self.shape
            self._keep = t  # keep alive until the copy has run
            self._check(self.lib.mh_set_state(self.ctx, ctypes.c_void_p(t.data_ptr()), DEVICE),
                        "mh_set_state")
        else:
            a = np.ascontiguousarray(np.asarray(U), dtype=self.np_dtype)
            assert a.shape == (5,) + self.shape, (a.shape, self.shape)
            self._check(self.lib.mh_set_state(self.ctx, a.ctypes.data_as(ctypes.c_void_p), HOST),
                        "mh_set_state")

    def get_state(self) -> np.ndarray:
        out = np.empty((5,) + self.shape, dtype=self.np_dtype)
        self._check(self.lib.mh_get_state(self.ctx, out.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_get_state")
        return out

    def get_state_into(self, out):
        """Copies the state into an existing CUDA tensor (enqueued)."""
        assert out.is_contiguous() and out.dtype == self.torch_dtype and out.numel() == 5 * int(
            np.prod(self.shape))
        self._check(self.lib.mh_get_state(self.ctx, ctypes.c_void_p(out.data_ptr()), DEVICE),
                    "mh_get_state")
        return out

    def new_state_tensor(self):
        """An uninitialised CUDA tensor of the state's shape and dtype."""
        return self._torch.empty((5,) + self.shape, dtype=self.torch_dtype, device=self.device)

    def get_state_device(self):
        torch = self._torch
        out = torch.empty((5,) + self.shape, dtype=self.torch_dtype, device=self.device)
        self._check(self.lib.mh_get_state(self.ctx, ctypes.c_void_p(out.data_ptr()), DEVICE),
                    "mh_get_state")
        return out

    # -- stepping
    def step(self, nsteps: int = 1, dt: float = 0.0, t_stop: float = math.inf,
             record: bool = False):
        """Advances nsteps; dt > 0 fixed, else CFL.  With record=True returns
        the per-step dt array (synchronises)."""
        dts = np.zeros(max(nsteps, 1)) if record else None
        st = self.lib.mh_step(self.ctx, nsteps, dt, t_stop,
                              dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if record else None,
                              None)
        self._check(st, "mh_step")
        return dts[:nsteps] if record else None

    def step_keep(self, dt: float, U1_out, Ub_out, record: bool = False):
        """One SSP-RK2 step (dt > 0 fixed, else CFL) that also writes its first
        stage to U1_out and its state after the forcing kick to Ub_out (CUDA
        tensors of the state's shape and dtype), for adjoint_step(kept=...).
        With record=True returns the step's dt (synchronises)."""
        d = np.zeros(1) if record else None
        U1_out, Ub_out = U1_out.contiguous(), Ub_out.contiguous()
        self._keep_step = (U1_out, Ub_out)
        st = self.lib.mh_step_keep(self.ctx, dt, ctypes.c_void_p(U1_out.data_ptr()),
                                   ctypes.c_void_p(Ub_out.data_ptr()),
                                   d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if record
                                   else None)
        self._check(st, "mh_step_keep")
        return d if record else None

    def run_to(self, t_stop: float, max_steps: int = 1_000_000):
        """Steps under CFL until the clock reaches t_stop; returns the dt list."""
        dts = []
        while True:
            t, _ = self.clock()
            if t >= t_stop or len(dts) >= max_steps:
                return np.array(dts)
            dts.extend(self.step(1, 0.0, t_stop, record=True))

    def clock(self):
        t = ctypes.c_double()
        s = ctypes.c_int64()
        self._check(self.lib.mh_get_clock(self.ctx, ctypes.byref(t), ctypes.byref(s)), "mh_get_clock")
        return t.value, s.value

    def set_clock(self, t: float, step: int):
        self._check(self.lib.mh_set_clock(self.ctx, t, step), "mh_set_clock")

    def ou_state(self) -> np.ndarray:
        n = ctypes.c_int32()
        self._check(self.lib.mh_get_ou_state(self.ctx, ctypes.byref(n), None), "mh_get_ou_state")
        a = np.zeros(6 * n.value)
        if n.value:
            self._check(self.lib.mh_get_ou_state(self.ctx, ctypes.byref(n),
                                                 a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                        "mh_get_ou_state")
        return a

    def set_ou_state(self, ahat):
        a = np.ascontiguousarray(ahat, dtype=np.float64)
        self._check(self.lib.mh_set_ou_state(self.ctx, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "mh_set_ou_state")

    def check(self):
        """(bad_cells, first_bad_flat_index) of the last step call."""
        b = ctypes.c_int64()
        f = ctypes.c_int64()
        st = self.lib.mh_check(self.ctx, ctypes.byref(b), ctypes.byref(f))
        if st not in (OK, E_NONFINITE):
            self._check(st, "mh_check")
        return b.value, f.value

    def mg_cycles(self) -> int:
        c = ctypes.c_int32()
        self._check(self.lib.mh_last_mg_cycles(self.ctx, ctypes.byref(c)), "mh_last_mg_cycles")
        return c.value

    def set_flux_correction(self, field=None, grad=None):
        """Attaches a learned flux-correction field (CUDA tensor [5][nz][ny][nx]
        of the state dtype) added to each cell's upper-face fluxes in every
        later step, and optionally a gradient tensor of the same shape that
        later adjoint steps accumulate into; None detaches.  The solver keeps
        references to both."""
        for t in (field, grad):
            if t is not None and (tuple(t.shape) != (5,) + self.shape or not t.is_contiguous()
                                  or t.dtype != self.torch_dtype):
                raise ValueError("flux correction tensors must be contiguous [5][nz][ny][nx] "
                                 "of the state dtype")
        self._dflux, self._dflux_grad = field, grad
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(self.lib.mh_set_flux_correction(self.ctx, ptr(field), ptr(grad)),
                    "mh_set_flux_correction")

    def set_graphs(self, enable: bool):
        """Multigrid V-cycles from captured HIP graphs (default) or launched
        kernel by kernel."""
        self._check(self.lib.mh_set_graphs(self.ctx, int(bool(enable))), "mh_set_graphs")

    def set_timing(self, enable: bool):
        """Records HIP events around every kernel launch of step()."""
        self._check(self.lib.mh_set_timing(self.ctx, 1 if enable else 0), "mh_set_timing")

    def timing(self):
        """(ms, launches) per kind (stage 1, stage 2, prologue, other) since
        the last read; synchronises and clears the records."""
        ms = np.zeros(4)
        n = np.zeros(4, dtype=np.int64)
        self._check(self.lib.mh_get_timing(self.ctx, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                    "mh_get_timing")
        return ms, n

    def set_potential(self, phi):
        """Multigrid warm start for the next step (torch CUDA tensor or host array)."""
        torch = self._torch
        if isinstance(phi, torch.Tensor) and phi.is_cuda:
            t = phi.to(self.torch_dtype).contiguous()
            self._keep_phi = t
            self._check(self.lib.mh_set_potential(self.ctx, ctypes.c_void_p(t.data_ptr()), DEVICE),
                        "mh_set_potential")
        else:
            a = np.ascontiguousarray(np.asarray(phi), dtype=self.np_dtype)
            self._check(self.lib.mh_set_potential(self.ctx, a.ctypes.data_as(ctypes.c_void_p), HOST),
                        "mh_set_potential")

    def potential_device(self):
        out = self._torch.empty(self.shape, dtype=self.torch_dtype, device=self.device)
        self._check(self.lib.mh_get_potential(self.ctx, ctypes.c_void_p(out.data_ptr()), DEVICE),
                    "mh_get_potential")
        return out

    def adjoint_step(self, U_n, dt: float, step: int, lam, ou_ahat=None, phi_n=None, out=None,
                     kept=None):
        """lam_n = (dU^{n+1}/dU^n)^T lam for the step from U_n (CUDA tensors of
        the solver's shape and dtype) with fixed dt at global index `step`;
        ou_ahat: OU amplitudes before the step (host), phi_n: potential before
        the step (CUDA tensor) or None; kept: (U1, Ub) written by step_keep for
        this step, which spares recomputing the two stages, or (U1, Ub,
        phi_np1) with the potential right after the step, which with
        multigrid gravity also spares the step's Poisson solve.  Returns lam_n
        (a new tensor unless `out` is given; `out` may be `lam`)."""
        torch = self._torch
        if getattr(self, "_adj_ws", None) is None:
            n = ctypes.c_size_t(0)
            self._check(self.lib.mh_query_adjoint_workspace(self.ctx, ctypes.byref(n)),
                        "mh_query_adjoint_workspace")
            self._adj_bytes = n.value
            self._adj_ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = (self._adj_ws.data_ptr() + 255) // 256 * 256
        U_n = U_n.contiguous()
        lam = lam.contiguous()
        if out is None:
            out = torch.empty_like(lam)
        ah = None
        if ou_ahat is not None:
            # kept alive on self until the next call: the copy is enqueued
            self._keep_ahat = np.ascontiguousarray(ou_ahat, dtype=np.float64)
            ah = self._keep_ahat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if phi_n is not None:
            phi_n = phi_n.contiguous()
        ph = ctypes.c_void_p(phi_n.data_ptr()) if phi_n is not None else None
        self._keep_adj = (U_n, lam, phi_n, kept)
        if kept is not None:
            U1, Ub = kept[0], kept[1]
            phi_np1 = kept[2].contiguous() if len(kept) > 2 and kept[2] is not None else None
            self._keep_adj += (phi_np1,)
            p1 = ctypes.c_void_p(phi_np1.data_ptr()) if phi_np1 is not None else None
            st = self.lib.mh_adjoint_step_kept(self.ctx, ctypes.c_void_p(base), self._adj_bytes,
                                               ctypes.c_void_p(U_n.data_ptr()),
                                               ctypes.c_void_p(U1.data_ptr()),
                                               ctypes.c_void_p(Ub.data_ptr()), dt, step, ah, ph,
                                               p1, ctypes.c_void_p(lam.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()))
            self._check(st, "mh_adjoint_step_kept")
            return out
        st = self.lib.mh_adjoint_step(self.ctx, ctypes.c_void_p(base), self._adj_bytes,
                                      ctypes.c_void_p(U_n.data_ptr()), dt, step, ah, ph,
                                      ctypes.c_void_p(lam.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()))
        self._check(st, "mh_adjoint_step")
        return out

    def potential(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.np_dtype)
        self._check(self.lib.mh_get_potential(self.ctx, out.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_get_potential")
        return out


# ---------------------------------------------------------------- corrector

NPARAM_CORRECTOR = 36357


def corr_desc(n: int, batch: int, dtype="f32", gamma=5.0 / 3.0, mean=(0.0,) * 5, std=(1.0,) * 5,
              scale=(1.0,) * 5, loss_w=(1.0,) * 5, floor_rel=1e-6,
              fallback_frac=1e-3, mode=0) -> CorrDesc:
    """mode: CORR_STATE (corrected state) or CORR_FLUX (the learned flux field)."""
    d = CorrDesc()
    d.mode = mode
    d.n, d.batch = n, batch
    d.dtype = F64 if dtype in ("f64", "float64", F64) else F32
    d.gamma = gamma
    d.mean[:], d.std[:], d.scale[:], d.loss_w[:] = list(mean), list(std), list(scale), list(loss_w)
    d.floor_rel, d.fallback_frac = floor_rel, fallback_frac
    return d


class Corrector:
    """The learned state corrector on one GPU (mh_corr_*): a torch workspace
    tensor and an mh_corr handle; states are CUDA tensors [batch][5][n][n][n]."""

    def __init__(self, desc: CorrDesc, device="cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("mihydro needs a GPU (no CPU fallback)")
        self._torch = torch
        self.lib = load_library()
        self.desc = desc
        self.device = torch.device(device)
        self.torch_dtype = torch.float64 if desc.dtype == F64 else torch.float32
        self.cells = desc.batch * desc.n ** 3
        n = ctypes.c_size_t(0)
        st = self.lib.mh_corr_query_workspace(ctypes.byref(desc), ctypes.byref(n))
        if st != OK:
            raise MHError(st, "mh_corr_query_workspace rejected the descriptor")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            st = self.lib.mh_corr_init(ctypes.byref(desc), ctypes.c_void_p(aligned), n.value,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise MHError(st, "mh_corr_init failed")
        self.h = h

    def _check(self, st, what):
        if st != OK:
            raise MHError(st, what)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mh_corr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _state(self, U):
        U = U.contiguous()
        if U.dtype != self.torch_dtype or U.device != self.device or U.numel() != 5 * self.cells:
            raise ValueError("state must be a contiguous CUDA tensor [batch][5][n][n][n] of the "
                             "corrector's dtype")
        return U

    def set_params(self, theta):
        a = np.ascontiguousarray(np.asarray(theta), dtype=np.float32)
        if a.size != NPARAM_CORRECTOR:
            raise ValueError(f"expected {NPARAM_CORRECTOR} parameters")
        self._check(self.lib.mh_corr_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_corr_set_params")

    def params(self) -> np.ndarray:
        out = np.empty(NPARAM_CORRECTOR, dtype=np.float32)
        self._check(self.lib.mh_corr_get_params(self.h, out.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_corr_get_params")
        return out

    def apply(self, U, out=None, stats: bool = True):
        """Returns (U_corrected, floored_cells, fell_back); with stats=False the
        call only enqueues and the two counts are None."""
        U = self._state(U)
        if out is None:
            out = self._torch.empty_like(U)
        fl = ctypes.c_int64(0)
        fb = ctypes.c_int32(0)
        self._keep_apply = (U, out)
        self._check(self.lib.mh_corr_apply(self.h, ctypes.c_void_p(U.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()),
                                           ctypes.byref(fl) if stats else None,
                                           ctypes.byref(fb) if stats else None), "mh_corr_apply")
        if not stats:
            return out, None, None
        return out, fl.value, bool(fb.value)

    def loss_grad(self, U, target):
        """Returns (loss, gradient as a float32 numpy array in canonical order)."""
        U, target = self._state(U), self._state(target)
        loss = ctypes.c_double(0.0)
        g = np.empty(NPARAM_CORRECTOR, dtype=np.float32)
        self._check(self.lib.mh_corr_loss_grad(self.h, ctypes.c_void_p(U.data_ptr()),
                                               ctypes.c_void_p(target.data_ptr()),
                                               ctypes.byref(loss),
                                               g.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_corr_loss_grad")
        return loss.value, g

    def train_step(self, U, target, lr: float, want_loss: bool = True):
        U, target = self._state(U), self._state(target)
        self._keep = (U, target)
        loss = ctypes.c_double(0.0)
        self._check(self.lib.mh_corr_train_step(self.h, ctypes.c_void_p(U.data_ptr()),
                                                ctypes.c_void_p(target.data_ptr()), lr,
                                                ctypes.byref(loss) if want_loss else None),
                    "mh_corr_train_step")
        return loss.value if want_loss else None

    def zero_grad(self):
        self._check(self.lib.mh_corr_zero_grad(self.h), "mh_corr_zero_grad")

    def backward(self, U, target=None, gUc=None, want_loss: bool = False,
                 input_grad: bool = False):
        """Adds the parameter gradient of one reverse pass at U to the
        accumulated one; returns (loss or None, dL/dU tensor or None)."""
        U = self._state(U)
        tg = self._state(target) if target is not None else None
        gu = self._state(gUc) if gUc is not None else None
        gU = self._torch.empty_like(U) if input_grad else None
        self._keep_bw = (U, tg, gu, gU)
        loss = ctypes.c_double(0.0)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(self.lib.mh_corr_backward(self.h, ptr(U), ptr(tg), ptr(gu),
                                              ctypes.byref(loss) if want_loss else None, ptr(gU)),
                    "mh_corr_backward")
        return (loss.value if want_loss else None), gU

    def adam_step(self, lr: float):
        self._check(self.lib.mh_corr_adam_step(self.h, lr), "mh_corr_adam_step")

    def grad(self) -> np.ndarray:
        out = np.empty(NPARAM_CORRECTOR, dtype=np.float32)
        self._check(self.lib.mh_corr_get_grad(self.h, out.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_corr_get_grad")
        return out

    def activation(self, which: int) -> np.ndarray:
        """0 x, 1 z1, 2 h1, 3 z2, 4 h2, 5 y of the last forward pass, or 6 dY,
        7 dZ2, 8 dZ1, 9 the first layer's input gradient of the last reverse
        pass, as float64 arrays [cells][channels] (bf16 ones widened exactly)."""
        ch = 16 if which in (5, 6, 9) else 32
        if which in (0, 2, 4, 6, 7, 8):
            raw = np.empty((self.cells, ch), dtype=np.uint16)
        else:
            raw = np.empty((self.cells, ch), dtype=np.float32)
        self._check(self.lib.mh_corr_get_activation(self.h, which,
                                                    raw.ctypes.data_as(ctypes.c_void_p), HOST),
                    "mh_corr_get_activation")
        if raw.dtype == np.uint16:
            return (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return raw.astype(np.float64)


def fft3(x, inverse: bool = False):
    """In-place 3D DFT (mh_fft3) of a CUDA tensor [n][n][n][2] of interleaved
    (re, im) float32/float64 values, x fastest; forward exp(-i), inverse
    unnormalised.  Returns x."""
    import torch

    lib = load_library()
    n = x.shape[0]
    if x.shape != (n, n, n, 2) or not x.is_contiguous() or x.device.type != "cuda":
        raise ValueError("fft3 needs a contiguous CUDA tensor [n][n][n][2]")
    dt = F64 if x.dtype == torch.float64 else F32
    need = ctypes.c_size_t(0)
    st = lib.mh_fft3_query_workspace(n, dt, ctypes.byref(need))
    if st != OK:
        raise MHError(st, "mh_fft3_query_workspace")
    ws = torch.empty(need.value, dtype=torch.uint8, device=x.device)
    st = lib.mh_fft3(ctypes.c_void_p(x.data_ptr()), n, dt, int(bool(inverse)),
                     ctypes.c_void_p(ws.data_ptr()), need.value,
                     ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if st != OK:
        raise MHError(st, "mh_fft3")
    return x


def step_corrected(solvers, corrector, nsteps: int, dts=None, use_graph: bool = True,
                   stage=None, count_fallbacks: bool = False):
    """mh_step_corrected: advances the solvers (one per batch member of the
    state-mode corrector, all on one stream) by nsteps corrected steps.  dts:
    CUDA float64 tensor [nsteps][B] of step sizes, or None for CFL steps.
    stage: optional CUDA buffer of 2 B 5 n^3 values of the dtype (allocated
    here when None).  Returns the number of fallbacks when count_fallbacks
    (synchronises), else None."""
    import torch

    lib = load_library()
    B = len(solvers)
    s0 = solvers[0]
    need = 2 * B * 5 * int(np.prod(s0.shape))
    if stage is None:
        stage = torch.empty(need, dtype=s0.torch_dtype, device=s0.device)
    elif stage.numel() < need or stage.dtype != s0.torch_dtype or not stage.is_contiguous():
        raise ValueError("stage must be a contiguous tensor of 2 B 5 n^3 values of the dtype")
    if dts is not None:
        if (tuple(dts.shape) != (nsteps, B) or dts.dtype != torch.float64 or not dts.is_cuda
                or not dts.is_contiguous()):
            raise ValueError("dts must be a contiguous CUDA float64 tensor [nsteps][B]")
    arr = (ctypes.c_void_p * B)(*[s.ctx.value for s in solvers])
    fb = ctypes.c_int64(0)
    corrector._keep_step = (stage, dts)
    st = lib.mh_step_corrected(arr, B, corrector.h, ctypes.c_void_p(stage.data_ptr()), nsteps,
                               ctypes.c_void_p(dts.data_ptr()) if dts is not None else None,
                               int(bool(use_graph)), ctypes.byref(fb) if count_fallbacks else None)
    if st != OK:
        raise MHError(st, f"mh_step_corrected: {lib.mh_last_error(solvers[0].ctx).decode()}")
    return fb.value if count_fallbacks else None


class Adam:
    """ADAM on one CUDA tensor (float32 or float64) through mh_adam: the
    moments live in tensors of the same shape, the update runs in the
    library.  step(grad) applies one iteration to the parameter in place."""

    def __init__(self, param, lr: float, betas=(0.9, 0.999), eps: float = 1e-8):
        import torch

        if not (param.is_cuda and param.is_contiguous()
                and param.dtype in (torch.float32, torch.float64)):
            raise ValueError("Adam needs a contiguous CUDA float32/float64 tensor")
        self.param, self.lr, self.betas, self.eps = param, lr, betas, eps
        self.m = torch.zeros_like(param)
        self.v = torch.zeros_like(param)
        self.it = 0
        self.lib = load_library()

    def step(self, grad):
        import torch

        g = grad.detach().to(self.param.dtype).contiguous()
        self.it += 1
        self._keep = g
        dt = F64 if self.param.dtype == torch.float64 else F32
        st = self.lib.mh_adam(ctypes.c_void_p(self.param.data_ptr()),
                              ctypes.c_void_p(self.m.data_ptr()),
                              ctypes.c_void_p(self.v.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                              self.param.numel(), dt, self.it, self.lr, self.betas[0],
                              self.betas[1], self.eps,
                              ctypes.c_void_p(torch.cuda.current_stream(self.param.device)
                                              .cuda_stream))
        if st != OK:
            raise MHError(st, "mh_adam")


def fft3_noalloc(x, inverse: bool = False):
    """fft3 through mh_fft3_noalloc: the twiddle table in the library's own
    device array, no workspace and no allocation (calls on one GPU must not
    overlap).  Returns x."""
    import torch

    lib = load_library()
    n = x.shape[0]
    if x.shape != (n, n, n, 2) or not x.is_contiguous() or x.device.type != "cuda":
        raise ValueError("fft3_noalloc needs a contiguous CUDA tensor [n][n][n][2]")
    dt = F64 if x.dtype == torch.float64 else F32
    with torch.cuda.device(x.device):
        st = lib.mh_fft3_noalloc(ctypes.c_void_p(x.data_ptr()), n, dt, int(bool(inverse)),
                                 ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if st != OK:
        raise MHError(st, "mh_fft3_noalloc")
    return x


def block_average(fine, r: int):
    """Conservative r^3 block average of a fine CUDA state [5][nf][nf][nf]."""
    import torch

    lib = load_library()
    fine = fine.contiguous()
    nf = fine.shape[-1]
    if fine.shape != (5, nf, nf, nf) or nf % r:
        raise ValueError("fine state must be [5][nf][nf][nf] with nf divisible by r")
    nc = nf // r
    out = torch.empty((5, nc, nc, nc), dtype=fine.dtype, device=fine.device)
    dt = F64 if fine.dtype == torch.float64 else F32
    st = lib.mh_block_average(ctypes.c_void_p(fine.data_ptr()), nf, r,
                              ctypes.c_void_p(out.data_ptr()), dt,
                              ctypes.c_void_p(torch.cuda.current_stream(fine.device).cuda_stream))
    if st != OK:
        raise MHError(st, "mh_block_average")
    return out
