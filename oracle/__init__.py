"""FP64 CPU oracle of the diffhydro finite-volume step (arXiv 2512.13403).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It loads
``liboracle.so`` (plain C, built by ``oracle/build.py``) through ctypes and
shares no code with the HIP library ``paper_2512_13403_amd``.

Each wrapper names the paper passage its C function follows:

* ``cfl_dt``        -- App. A.4 (CFL condition)
* ``rhs``           -- App. A.1-A.3 (MUSCL on primitives, HLLC, rhs_unsplit)
* ``rk2``           -- App. A.3 (RK2 / Heun in Shu-Osher form)
* ``ssprk3``/``euler``/``integrate`` -- App. A.3 (the other explicit RK options)
* ``cool``          -- Sec. 4 (operator-split cooling, exact per cell)
* ``ou_*``/``kick`` -- Sec. 3.1.1 (Ornstein-Uhlenbeck forcing)
* ``mg_*``/``gravity_accel`` -- Sec. 6, 6.2, App. C (multigrid self-gravity)
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_OUTFLOW = 0, 1
LIM_MINMOD, LIM_NONE, LIM_VANLEER, LIM_MC, LIM_SUPERBEE = 0, 1, 2, 3, 4
RS_HLLC, RS_HLL, RS_RUSANOV = 0, 1, 2
RK_SSP2, RK_SSP3, RK_EULER = 0, 1, 2
MG_V, MG_W = 0, 1
SMOOTH_JACOBI, SMOOTH_RBGS = 0, 1
GRAV_MG, GRAV_FFT = 0, 1
COOL_EXACT2, COOL_TABLE = 0, 1
COOLINT_TRAPEZOID, COOLINT_SUBCYCLE, COOLINT_AUTO = 0, 1, 2
COOL_TABMAX = 64
SRC_COOLING, SRC_FORCING, SRC_GRAVITY = 1, 2, 4
OU_MAXMODES = 64


class Config(ctypes.Structure):
    """Mirror of ``or_config`` in oracle.h."""

    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 3),
        ("h", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("ou_every", ctypes.c_int32),
        ("cool_lambda0", ctypes.c_double),
        ("cool_tc", ctypes.c_double),
        ("cool_ts", ctypes.c_double),
        ("cool_tfloor", ctypes.c_double),
        ("ou_seed", ctypes.c_uint64),
        ("ou_tau", ctypes.c_double),
        ("ou_arms", ctypes.c_double),
        ("ou_zeta", ctypes.c_double),
        ("ou_kmin", ctypes.c_double),
        ("ou_kmax", ctypes.c_double),
        ("grav_G", ctypes.c_double),
        ("mg_pre", ctypes.c_int32),
        ("mg_post", ctypes.c_int32),
        ("mg_max_cycles", ctypes.c_int32),
        ("mg_coarsest", ctypes.c_int32),
        ("mg_tol", ctypes.c_double),
        ("mg_coarse_sweeps", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("mg_cycle", ctypes.c_int32),
        ("mg_smoother", ctypes.c_int32),
        ("grav_solver", ctypes.c_int32),
        ("cool_model", ctypes.c_int32),
        ("cool_integrator", ctypes.c_int32),
        ("cool_nsub_max", ctypes.c_int32),
        ("cool_ntab", ctypes.c_int32),
        ("pad2_", ctypes.c_int32),
        ("cool_frac", ctypes.c_double),
        ("cool_ccool", ctypes.c_double),
        ("cool_L1", ctypes.c_double),
        ("cool_a1", ctypes.c_double),
        ("cool_L2", ctypes.c_double),
        ("cool_a2", ctypes.c_double),
        ("cool_heat", ctypes.c_double),
        ("cool_logT", ctypes.c_double * 64),
        ("cool_logL", ctypes.c_double * 64),
        ("flux_corr", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        cp = ctypes.POINTER(Config)
        sig = {
            "or_primitives": (None, [cp, dp, dp]),
            "or_cfl_dt": (ctypes.c_double, [cp, dp]),
            "or_rhs": (None, [cp, dp, dp]),
            "or_rk2": (None, [cp, dp, ctypes.c_double]),
            "or_euler": (None, [cp, dp, ctypes.c_double]),
            "or_ssprk3": (None, [cp, dp, ctypes.c_double]),
            "or_cool_lambda": (ctypes.c_double, [cp, ctypes.c_double]),
            "or_cool_edot": (ctypes.c_double, [cp, ctypes.c_double, ctypes.c_double]),
            "or_cool_eth_step": (ctypes.c_double, [cp, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double]),
            "or_cool_dt_limit": (ctypes.c_double, [cp, dp]),
            "or_cool_eth_step_d": (ctypes.c_double, [cp, ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_double, dp, dp]),
            "or_integrate": (None, [cp, dp, ctypes.c_double]),
            "or_cool_temperature": (ctypes.c_double, [ctypes.c_double] * 8),
            "or_cool": (None, [cp, dp, ctypes.c_double]),
            "or_ou_gauss": (None, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, dp]),
            "or_ou_modes": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ip]),
            "or_ou_init": (None, [cp, ctypes.c_int, ip, dp]),
            "or_ou_advance": (None, [cp, ctypes.c_int, ip, dp, ctypes.c_int64, ctypes.c_double]),
            "or_ou_scale": (ctypes.c_double, [cp, ctypes.c_int, dp]),
            "or_ou_accel": (None, [cp, ctypes.c_int, ip, dp, dp]),
            "or_ou_accel_at": (None, [cp, ctypes.c_int, ip, dp, ctypes.c_long, ctypes.c_long,
                                      ctypes.c_long, dp]),
            "or_kick": (None, [cp, dp, dp, ctypes.c_double]),
            "or_laplacian": (None, [ctypes.c_int, ctypes.c_double, dp, dp]),
            "or_mg_vcycle": (None, [cp, ctypes.c_int, ctypes.c_double, dp, dp]),
            "or_mg_solve": (ctypes.c_int, [cp, ctypes.c_int, ctypes.c_double, dp, dp]),
            "or_mg_smooth": (None, [cp, ctypes.c_int, ctypes.c_double, dp, dp]),
            "or_dft3": (None, [ctypes.c_int, ctypes.c_int, dp, dp]),
            "or_fft_gravity": (None, [cp, dp, dp, dp]),
            "or_fft_gravity_vjp": (None, [cp, dp, dp]),
            "or_gravity_accel": (ctypes.c_int, [cp, dp, dp, dp]),
            "or_num_threads": (ctypes.c_int, []),
            "or_set_num_threads": (None, [ctypes.c_int]),
            "or_rhs_vjp": (None, [cp, dp, dp, dp]),
            "or_rk2_vjp": (None, [cp, dp, ctypes.c_double, dp, dp]),
            "or_euler_vjp": (None, [cp, dp, ctypes.c_double, dp, dp]),
            "or_ssprk3_vjp": (None, [cp, dp, ctypes.c_double, dp, dp]),
            "or_integrate_vjp": (None, [cp, dp, ctypes.c_double, dp, dp]),
            "or_kick_vjp": (None, [cp, dp, dp, ctypes.c_double, dp, dp, dp]),
            "or_cool_vjp": (None, [cp, dp, ctypes.c_double, dp, dp]),
            "or_gravity_vjp": (ctypes.c_int, [cp, dp, ctypes.c_double, dp, dp, dp]),
            "or_step_vjp": (None, [cp, dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int, ip, dp, dp,
                                   dp, dp]),
            "or_step_vjp_flux": (None, [cp, dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int, ip, dp,
                                        dp, dp, dp, dp]),
            "or_flux_corr_vjp": (None, [cp, dp, ctypes.c_double, dp]),
            "or_step": (ctypes.c_double, [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                          ctypes.c_int, ip, dp, dp, ip]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def make_config(shape, h, bc=(BC_PERIODIC,) * 3, gamma=5.0 / 3.0, cfl=0.4, limiter=LIM_MINMOD,
                riemann=RS_HLLC, flags=0, cool=(0.3, 1e-2, 1e-3, 1e-4), ou_seed=0, ou_tau=0.5,
                ou_arms=1.0, ou_zeta=1.0, ou_kmin=1.0, ou_kmax=2.0, ou_every=1, grav_G=0.0,
                mg_pre=2, mg_post=2, mg_max_cycles=20, mg_coarsest=4, mg_tol=1e-10,
                mg_coarse_sweeps=200, integrator=RK_SSP2, mg_cycle=MG_V, mg_smoother=SMOOTH_JACOBI,
                grav_solver=GRAV_MG, cool_model=COOL_EXACT2, cool_integrator=COOLINT_TRAPEZOID,
                cool_nsub_max=1000, cool_frac=0.1, cool_ccool=0.0, cool_ki=(0.0, 0.0, 0.0, 0.0),
                cool_heat=0.0, cool_table=None, flux_corr=None) -> Config:
    """shape = (nz, ny, nx) of the state arrays; h = (hx, hy, hz); bc per (x, y, z)."""
    nz, ny, nx = shape
    c = Config()
    c.n[:] = [nx, ny, nz]
    c.bc[:] = list(bc)
    c.h[:] = list(h)
    c.gamma, c.cfl, c.limiter, c.riemann, c.flags = gamma, cfl, limiter, riemann, flags
    c.cool_lambda0, c.cool_tc, c.cool_ts, c.cool_tfloor = cool
    c.ou_seed, c.ou_tau, c.ou_arms, c.ou_zeta = ou_seed, ou_tau, ou_arms, ou_zeta
    c.ou_kmin, c.ou_kmax, c.ou_every = ou_kmin, ou_kmax, ou_every
    c.grav_G = grav_G
    c.mg_pre, c.mg_post, c.mg_max_cycles, c.mg_coarsest = mg_pre, mg_post, mg_max_cycles, mg_coarsest
    c.mg_tol, c.mg_coarse_sweeps = mg_tol, mg_coarse_sweeps
    c.integrator = integrator
    c.mg_cycle, c.mg_smoother, c.grav_solver = mg_cycle, mg_smoother, grav_solver
    c.cool_model, c.cool_integrator, c.cool_nsub_max = cool_model, cool_integrator, cool_nsub_max
    c.cool_frac, c.cool_ccool, c.cool_heat = cool_frac, cool_ccool, cool_heat
    c.cool_L1, c.cool_a1, c.cool_L2, c.cool_a2 = cool_ki
    if cool_table is not None:
        logT, logL = (np.asarray(a, dtype=np.float64) for a in cool_table)
        assert logT.shape == logL.shape and 2 <= len(logT) <= COOL_TABMAX
        c.cool_ntab = len(logT)
        c.cool_logT[:len(logT)] = list(logT)
        c.cool_logL[:len(logL)] = list(logL)
    set_flux_corr(c, flux_corr)
    return c


def set_flux_corr(c, field):
    """Attach a flux-correction field [5][nz][ny][nx] (or None) to c; c keeps
    a reference to the array it points at."""
    if field is None:
        c.flux_corr = None
        c._flux_ref = None
        return c
    a = np.ascontiguousarray(field, dtype=np.float64)
    assert a.shape == (5,) + _shape(c)
    c._flux_ref = a
    c.flux_corr = a.ctypes.data
    return c


def _shape(c: Config):
    return (c.n[2], c.n[1], c.n[0])


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls in this process."""
    lib().or_set_num_threads(int(n))


def primitives(c, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.empty_like(U)
    lib().or_primitives(ctypes.byref(c), _dp(U), _dp(W))
    return W


def cfl_dt(c, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().or_cfl_dt(ctypes.byref(c), _dp(U))


def rhs(c, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    L = np.empty_like(U)
    lib().or_rhs(ctypes.byref(c), _dp(U), _dp(L))
    return L


def rk2(c, U, dt):
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().or_rk2(ctypes.byref(c), _dp(U), dt)
    return U


def euler(c, U, dt):
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().or_euler(ctypes.byref(c), _dp(U), dt)
    return U


def ssprk3(c, U, dt):
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().or_ssprk3(ctypes.byref(c), _dp(U), dt)
    return U


def integrate(c, U, dt):
    """One update by the configuration's integrator (c.integrator)."""
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().or_integrate(ctypes.byref(c), _dp(U), dt)
    return U


def cool_lambda(c, T):
    return lib().or_cool_lambda(ctypes.byref(c), T)


def cool_edot(c, rho, Eth):
    return lib().or_cool_edot(ctypes.byref(c), rho, Eth)


def cool_eth_step(c, rho, Eth, dt):
    """One step of the tabulated model's integrator (oracle_cool.c)."""
    return lib().or_cool_eth_step(ctypes.byref(c), rho, Eth, dt)


def cool_eth_step_d(c, rho, Eth, dt):
    """(E', dE'/dEth, dE'/drho) of the tabulated model's step."""
    dE = ctypes.c_double(0.0)
    dr = ctypes.c_double(0.0)
    v = lib().or_cool_eth_step_d(ctypes.byref(c), rho, Eth, dt, ctypes.byref(dE), ctypes.byref(dr))
    return v, dE.value, dr.value


def cool_dt_limit(c, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().or_cool_dt_limit(ctypes.byref(c), _dp(U))


def cool_temperature(rho, T, dt, gamma, L0, Tc, Ts, Tfloor):
    return lib().or_cool_temperature(rho, T, dt, gamma, L0, Tc, Ts, Tfloor)


def cool(c, U, dt):
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    lib().or_cool(ctypes.byref(c), _dp(U), dt)
    return U


def ou_gauss(seed, group, mode, comp):
    out = np.zeros(2)
    lib().or_ou_gauss(seed, group, mode, comp, _dp(out))
    return complex(out[0], out[1])


def ou_modes(kmin=1.0, kmax=2.0):
    nv = np.zeros(3 * OU_MAXMODES, dtype=np.int32)
    m = lib().or_ou_modes(kmin, kmax, _ip(nv))
    if m < 0:
        raise ValueError("too many OU modes")
    return nv[: 3 * m].reshape(m, 3).copy()


def ou_init(c, nvec):
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    a = np.zeros(6 * len(nvec))
    lib().or_ou_init(ctypes.byref(c), len(nvec), _ip(nvec), _dp(a))
    return a


def ou_advance(c, nvec, ahat, group, dt):
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    a = np.array(ahat, dtype=np.float64, copy=True)
    lib().or_ou_advance(ctypes.byref(c), len(nvec), _ip(nvec), _dp(a), group, dt)
    return a


def ou_scale(c, ahat):
    a = np.ascontiguousarray(ahat, dtype=np.float64)
    return lib().or_ou_scale(ctypes.byref(c), len(a) // 6, _dp(a))


def ou_accel(c, nvec, ahat):
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    a = np.ascontiguousarray(ahat, dtype=np.float64)
    acc = np.zeros((3,) + _shape(c))
    lib().or_ou_accel(ctypes.byref(c), len(nvec), _ip(nvec), _dp(a), _dp(acc))
    return acc


def ou_accel_at(c, nvec, ahat, i, j, k):
    """Acceleration at the centre of cell (i, j, k) (x index first)."""
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    a = np.ascontiguousarray(ahat, dtype=np.float64)
    out = np.zeros(3)
    lib().or_ou_accel_at(ctypes.byref(c), len(nvec), _ip(nvec), _dp(a), i, j, k, _dp(out))
    return out


def kick(c, U, acc, dt):
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    lib().or_kick(ctypes.byref(c), _dp(U), _dp(acc), dt)
    return U


def laplacian(n, h, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.empty_like(phi)
    lib().or_laplacian(n, h, _dp(phi), _dp(out))
    return out


def mg_vcycle(c, n, h, phi, F):
    phi = np.array(phi, dtype=np.float64, copy=True)
    F = np.ascontiguousarray(F, dtype=np.float64)
    lib().or_mg_vcycle(ctypes.byref(c), n, h, _dp(phi), _dp(F))
    return phi


def mg_solve(c, n, h, phi, F):
    phi = np.array(phi, dtype=np.float64, copy=True)
    F = np.ascontiguousarray(F, dtype=np.float64)
    cyc = lib().or_mg_solve(ctypes.byref(c), n, h, _dp(phi), _dp(F))
    return phi, cyc


def mg_smooth(c, n, h, phi, F):
    """One sweep of the configured smoother (c.mg_smoother)."""
    phi = np.array(phi, dtype=np.float64, copy=True)
    F = np.ascontiguousarray(F, dtype=np.float64)
    lib().or_mg_smooth(ctypes.byref(c), n, h, _dp(phi), _dp(F))
    return phi


def dft3(x, inverse=False):
    """3D DFT of an n^3 complex array by its definition (oracle_fft.c)."""
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    lib().or_dft3(x.shape[0], int(inverse), _dp(re), _dp(im))
    return re + 1j * im


def fft_gravity(c, rho):
    """Spectral potential and acceleration of a density field (Sec. 6.1)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.empty_like(rho)
    acc = np.empty((3,) + rho.shape)
    lib().or_fft_gravity(ctypes.byref(c), _dp(rho), _dp(phi), _dp(acc))
    return phi, acc


def fft_gravity_vjp(c, accb):
    accb = np.ascontiguousarray(accb, dtype=np.float64)
    rhob = np.empty(accb.shape[1:])
    lib().or_fft_gravity_vjp(ctypes.byref(c), _dp(accb), _dp(rhob))
    return rhob


def gravity_accel(c, U, phi):
    U = np.ascontiguousarray(U, dtype=np.float64)
    phi = np.array(phi, dtype=np.float64, copy=True)
    acc = np.zeros((3,) + _shape(c))
    cyc = lib().or_gravity_accel(ctypes.byref(c), _dp(U), _dp(phi), _dp(acc))
    return acc, phi, cyc


# ---------------------------------------------------------------- adjoints
# Reverse-mode derivatives with dt held fixed (oracle_adjoint.c).

def rhs_vjp(c, U, v):
    """(dL/dU)^T v for L = rhs (App. A.1-A.3)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(U)
    lib().or_rhs_vjp(ctypes.byref(c), _dp(U), _dp(v), _dp(out))
    return out


def rk2_vjp(c, U, dt, lam):
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty_like(U)
    lib().or_rk2_vjp(ctypes.byref(c), _dp(U), dt, _dp(lam), _dp(out))
    return out


def _vjp(fn, c, U, dt, lam):
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty_like(U)
    fn(ctypes.byref(c), _dp(U), dt, _dp(lam), _dp(out))
    return out


def euler_vjp(c, U, dt, lam):
    return _vjp(lib().or_euler_vjp, c, U, dt, lam)


def ssprk3_vjp(c, U, dt, lam):
    return _vjp(lib().or_ssprk3_vjp, c, U, dt, lam)


def integrate_vjp(c, U, dt, lam):
    return _vjp(lib().or_integrate_vjp, c, U, dt, lam)


def kick_vjp(c, U, acc, dt, lam):
    U = np.ascontiguousarray(U, dtype=np.float64)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty_like(U)
    accb = np.empty_like(acc)
    lib().or_kick_vjp(ctypes.byref(c), _dp(U), _dp(acc), dt, _dp(lam), _dp(out), _dp(accb))
    return out, accb


def cool_vjp(c, U, dt, lam):
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty_like(U)
    lib().or_cool_vjp(ctypes.byref(c), _dp(U), dt, _dp(lam), _dp(out))
    return out


def gravity_vjp(c, U, dt, phi, lam):
    """Reverse of U' = kick(U, -grad A^+ 4 pi G (rho - <rho>)); phi = warm start."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    phi = np.array(phi, dtype=np.float64, copy=True)
    out = np.empty_like(U)
    lib().or_gravity_vjp(ctypes.byref(c), _dp(U), dt, _dp(phi), _dp(lam), _dp(out))
    return out


def step_vjp(c, Un, dt, step, nvec, ahat, phi, lam):
    """(dU^{n+1}/dU^n)^T lam for one full step at fixed dt; ahat and phi are
    the OU modes and potential before the step."""
    Un = np.ascontiguousarray(Un, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nv = np.ascontiguousarray(nvec, dtype=np.int32).reshape(-1)
    if nv.size == 0:
        nv = np.zeros(3, dtype=np.int32)
    a = np.array(ahat, dtype=np.float64, copy=True)
    ph = np.array(phi, dtype=np.float64, copy=True)
    out = np.empty_like(Un)
    lib().or_step_vjp(ctypes.byref(c), _dp(Un), dt, step, len(nvec), _ip(nv), _dp(a), _dp(ph),
                      _dp(lam), _dp(out))
    return out


def step_vjp_flux(c, Un, dt, step, nvec, ahat, phi, lam):
    """step_vjp that also returns the adjoint of the flux-correction field
    attached to c: (lam_n, gflux)."""
    Un = np.ascontiguousarray(Un, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nv = np.ascontiguousarray(nvec, dtype=np.int32).reshape(-1)
    if nv.size == 0:
        nv = np.zeros(3, dtype=np.int32)
    a = np.array(ahat, dtype=np.float64, copy=True)
    ph = np.array(phi, dtype=np.float64, copy=True)
    out = np.empty_like(Un)
    g = np.zeros_like(Un)
    lib().or_step_vjp_flux(ctypes.byref(c), _dp(Un), dt, step, len(nvec), _ip(nv), _dp(a),
                           _dp(ph), _dp(lam), _dp(out), _dp(g))
    return out, g


def flux_corr_vjp(c, v, weight=1.0):
    """weight (dL/dflux_corr)^T v for L = rhs."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros_like(v)
    lib().or_flux_corr_vjp(ctypes.byref(c), _dp(v), weight, _dp(g))
    return g


@dataclass
class Simulation:
    """Host-side driver around ``or_step``: the state, time, step index, OU
    mode state and gravitational potential of one run."""

    cfg: Config
    U: np.ndarray
    t: float = 0.0
    step_index: int = 0
    nvec: np.ndarray = field(default=None)
    ahat: np.ndarray = field(default=None)
    phi: np.ndarray = field(default=None)
    dts: list = field(default_factory=list)
    mg_cycles: list = field(default_factory=list)

    def __post_init__(self):
        self.U = np.array(self.U, dtype=np.float64, order="C", copy=True)
        if self.nvec is None:
            if self.cfg.flags & SRC_FORCING:
                self.nvec = ou_modes(self.cfg.ou_kmin, self.cfg.ou_kmax)
                self.ahat = ou_init(self.cfg, self.nvec)
            else:
                self.nvec = np.zeros((0, 3), dtype=np.int32)
                self.ahat = np.zeros(6)
        if self.phi is None:
            self.phi = np.zeros(_shape(self.cfg))

    def advance(self, nsteps: int, dt: float = 0.0, t_stop: float = math.inf):
        L = lib()
        nv = np.ascontiguousarray(self.nvec, dtype=np.int32).reshape(-1)
        if nv.size == 0:
            nv = np.zeros(3, dtype=np.int32)
        cyc = np.zeros(1, dtype=np.int32)
        for _ in range(nsteps):
            cap = t_stop - self.t
            used = L.or_step(ctypes.byref(self.cfg), _dp(self.U), dt, cap, self.step_index,
                             len(self.nvec), _ip(nv), _dp(self.ahat), _dp(self.phi), _ip(cyc))
            self.dts.append(used)
            self.mg_cycles.append(int(cyc[0]))
            self.t += used
            self.step_index += 1
        return self

    def run_to(self, t_stop: float, max_steps: int = 1_000_000):
        n = 0
        while self.t < t_stop and n < max_steps:
            self.advance(1, 0.0, t_stop)
            n += 1
        return n
