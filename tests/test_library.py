"""Host-only checks of the C-ABI library: it loads without a GPU, exports
every entry point that include/mihydro.h declares, and its argument
validation (mh_query_workspace is pure host code) rejects bad descriptors
with the documented status codes."""
import ctypes
import os
import re

import pytest

import paper_2512_13403_amd as mh
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    text = open(os.path.join(ROOT, "include", "mihydro.h")).read()
    return sorted(set(re.findall(r"\b(mh_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mh.load_library()
    names = declared_entry_points()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mh.EXPORTED) == names


def ws(grid, phys):
    n = ctypes.c_size_t(0)
    st = mh.load_library().mh_query_workspace(ctypes.byref(grid), ctypes.byref(phys), ctypes.byref(n))
    return st, n.value


def test_workspace_size_of_valid_grids():
    g = mh.grid_desc((16, 16, 128), (1 / 128,) * 3, (1, 0, 0), "f64", 1.4)
    st, n = ws(g, mh.physics_desc())
    assert st == mh.OK and n >= 2 * 5 * 128 * 16 * 16 * 8
    g32 = mh.grid_desc((64, 64, 64), (1 / 64,) * 3, dtype="f32")
    st, n32 = ws(g32, mh.physics_desc(flags=mh.SRC_FORCING | mh.SRC_COOLING))
    assert st == mh.OK and n32 >= 2 * 5 * 64 ** 3 * 4
    st, ng = ws(g32, mh.physics_desc(flags=mh.SRC_GRAVITY, grav_G=1.0))
    assert st == mh.OK and ng > n32  # the multigrid hierarchy adds > 4 fields


@pytest.mark.parametrize("mutate,status", [
    (lambda g, p: setattr(g, "dtype", 7), mh.E_DTYPE),
    (lambda g, p: g.n.__setitem__(0, 0), mh.E_INVALID),
    (lambda g, p: g.h.__setitem__(1, -1.0), mh.E_INVALID),
    (lambda g, p: g.bc.__setitem__(2, 5), mh.E_INVALID),
    (lambda g, p: setattr(g, "gamma", 1.0), mh.E_INVALID),
    (lambda g, p: setattr(g, "cfl", 0.0), mh.E_INVALID),
    (lambda g, p: setattr(g, "limiter", 9), mh.E_UNSUPPORTED),
    (lambda g, p: setattr(g, "riemann", 7), mh.E_UNSUPPORTED),
    (lambda g, p: setattr(g, "limiter", -1), mh.E_UNSUPPORTED),
    (lambda g, p: setattr(g, "integrator", 3), mh.E_UNSUPPORTED),
    (lambda g, p: setattr(g, "integrator", -1), mh.E_UNSUPPORTED),
    (lambda g, p: setattr(p, "flags", 64), mh.E_INVALID),
    (lambda g, p: (setattr(p, "flags", mh.SRC_FORCING), setattr(p, "ou_tau", 0.0)), mh.E_INVALID),
    (lambda g, p: (setattr(p, "flags", mh.SRC_FORCING), setattr(p, "ou_kmin", 3.0),
                   setattr(p, "ou_kmax", 2.0)), mh.E_INVALID),
    (lambda g, p: (setattr(p, "flags", mh.SRC_FORCING), setattr(p, "ou_kmax", 3.5)), mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_COOLING), setattr(p, "cool_ts", 0.0)), mh.E_INVALID),
    (lambda g, p: (setattr(p, "flags", mh.SRC_COOLING), setattr(p, "cool_model", 3)),
     mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_COOLING), setattr(p, "cool_ccool", 0.3)),
     mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_COOLING), setattr(p, "cool_model", 1)),
     mh.E_INVALID),  # no table points

    # an x-y plane of 4 GiB (fp64): lane offsets inside a plane are 32-bit
    (lambda g, p: (g.n.__setitem__(0, 65536), g.n.__setitem__(1, 8192), g.n.__setitem__(2, 1)),
     mh.E_SHAPE),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), g.bc.__setitem__(0, 1)), mh.E_SHAPE),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), g.n.__setitem__(0, 32)), mh.E_SHAPE),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), setattr(p, "mg_coarsest", 0)), mh.E_INVALID),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), setattr(p, "mg_cycle", 2)), mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), setattr(p, "mg_smoother", 5)),
     mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), setattr(p, "grav_solver", 4)),
     mh.E_UNSUPPORTED),
    (lambda g, p: (setattr(p, "flags", mh.SRC_GRAVITY), setattr(p, "grav_solver", mh.GRAV_FFT),
                   g.n.__setitem__(0, 12), g.n.__setitem__(1, 12), g.n.__setitem__(2, 12)),
     mh.E_SHAPE),
])
def test_validation_rejects(mutate, status):
    g = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f64")
    p = mh.physics_desc()
    mutate(g, p)
    st, _ = ws(g, p)
    assert st == status


def test_scheme_variants_are_accepted():
    for lim in (mh.LIM_MINMOD, mh.LIM_NONE, mh.LIM_VANLEER, mh.LIM_MC, mh.LIM_SUPERBEE):
        for rs in (mh.RS_HLLC, mh.RS_HLL, mh.RS_RUSANOV):
            g = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f32", limiter=lim, riemann=rs)
            assert ws(g, mh.physics_desc())[0] == mh.OK


def test_fft3_workspace_query_checks_its_arguments():
    L = mh.load_library()
    n = ctypes.c_size_t(0)
    assert L.mh_fft3_query_workspace(64, mh.F64, ctypes.byref(n)) == mh.OK and n.value == 32 * 16
    assert L.mh_fft3_query_workspace(48, mh.F64, ctypes.byref(n)) == mh.E_SHAPE
    assert L.mh_fft3_query_workspace(2048, mh.F32, ctypes.byref(n)) == mh.E_SHAPE
    assert L.mh_fft3_query_workspace(64, 9, ctypes.byref(n)) == mh.E_DTYPE


def test_tabulated_cooling_is_accepted_and_checked():
    g = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f32")
    kw = dict(flags=mh.SRC_COOLING, cool_model=mh.COOL_TABLE, cool_table=wl.synthetic_cie_table(),
              **wl.COOLING_TABLE_MODEL)
    assert ws(g, mh.physics_desc(**kw))[0] == mh.OK
    assert ws(g, mh.physics_desc(cool_ccool=0.2, cool_integrator=mh.COOLINT_AUTO, **kw))[0] == mh.OK
    bad = mh.physics_desc(**kw)
    bad.cool_logT[3] = bad.cool_logT[2]
    assert ws(g, bad)[0] == mh.E_INVALID
    assert ws(g, mh.physics_desc(cool_frac=0.0, **kw))[0] == mh.E_INVALID


def test_ssprk3_workspace_holds_one_more_state():
    p = mh.physics_desc()
    g2 = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f32")
    g3 = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f32", integrator=mh.RK_SSP3)
    ge = mh.grid_desc((16, 16, 16), (1 / 16,) * 3, dtype="f32", integrator=mh.RK_EULER)
    (s2, n2), (s3, n3), (se, ne) = ws(g2, p), ws(g3, p), ws(ge, p)
    assert s2 == s3 == se == mh.OK
    assert n3 >= n2 + 5 * 16 ** 3 * 4 and ne == n2


def test_gravity_coarsest_grid_limit():
    # 3 * 2^k grids coarsen to 3^3; 25 * 4 = 100 coarsens to 25^3 > 2048 cells
    g = mh.grid_desc((96, 96, 96), (1 / 96,) * 3, dtype="f64")
    assert ws(g, mh.physics_desc(flags=mh.SRC_GRAVITY))[0] == mh.OK
    g = mh.grid_desc((100, 100, 100), (1 / 100,) * 3, dtype="f64")
    assert ws(g, mh.physics_desc(flags=mh.SRC_GRAVITY))[0] == mh.E_SHAPE


def test_null_arguments():
    lib = mh.load_library()
    assert lib.mh_query_workspace(None, None, None) == mh.E_INVALID
    assert lib.mh_step(None, 1, 0.0, 1.0, None, None) == mh.E_INVALID
    assert lib.mh_step_keep(None, 0.0, None, None, None) == mh.E_INVALID
    assert lib.mh_adjoint_step_kept(None, None, 0, None, None, None, 0.0, 0, None, None, None,
                                    None, None) == mh.E_INVALID
    assert lib.mh_set_state(None, None, 0) == mh.E_INVALID
    assert lib.mh_last_error(None) == b""
    lib.mh_destroy(None)


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = mh.grid_desc((8, 8, 8), (1 / 8,) * 3)
    with pytest.raises(RuntimeError):
        mh.Solver(g)


def corr_ws(d):
    n = ctypes.c_size_t(0)
    st = mh.load_library().mh_corr_query_workspace(ctypes.byref(d), ctypes.byref(n))
    return st, n.value


def test_corrector_workspace_and_validation():
    st, n = corr_ws(mh.corr_desc(64, 2, "f32"))
    cells = 2 * 64 ** 3
    # activations alone: x, h1, h2, dY, dZ (bf16, 32 ch) + z1, z2 (fp32) + y
    assert st == mh.OK and n >= cells * (32 * 2 * 6 + 32 * 4 * 2 + 16 * 4)
    bad = [
        (lambda d: setattr(d, "n", 24), mh.E_SHAPE),
        (lambda d: setattr(d, "n", 8), mh.E_SHAPE),
        (lambda d: setattr(d, "batch", 0), mh.E_SHAPE),
        (lambda d: setattr(d, "dtype", 3), mh.E_DTYPE),
        (lambda d: setattr(d, "gamma", 0.5), mh.E_INVALID),
        (lambda d: d.std.__setitem__(2, 0.0), mh.E_INVALID),
        (lambda d: setattr(d, "floor_rel", -1.0), mh.E_INVALID),
        (lambda d: setattr(d, "mode", 2), mh.E_UNSUPPORTED),
    ]
    assert corr_ws(mh.corr_desc(32, 1, "f64", mode=mh.CORR_FLUX))[0] == mh.OK
    for mutate, status in bad:
        d = mh.corr_desc(32, 1, "f64")
        mutate(d)
        assert corr_ws(d)[0] == status
    lib = mh.load_library()
    assert lib.mh_corr_query_workspace(None, None) == mh.E_INVALID
    assert lib.mh_corr_apply(None, None, None, None, None) == mh.E_INVALID
    assert lib.mh_corr_train_step(None, None, None, 1e-3, None) == mh.E_INVALID
    assert lib.mh_block_average(None, 8, 2, None, mh.F32, None) == mh.E_INVALID
    lib.mh_corr_destroy(None)


def test_corrector_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        mh.Corrector(mh.corr_desc(16, 1))
