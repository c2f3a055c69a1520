"""The allocation-free transform entry point (mh_fft3_noalloc) against the
workspace one (mh_fft3), called through the C ABI: two calls in a row per
dtype and direction, the second on a smaller cube, each bitwise equal to
mh_fft3 on the same input (same kernels, same twiddle values), plus the
argument checks of the new entry point."""
import ctypes

import numpy as np
import pytest

import paper_2512_13403_amd as mh

pytestmark = pytest.mark.gpu


def _cube(n, dtype, seed):
    import torch

    g = np.random.default_rng(seed).standard_normal((n, n, n, 2))
    return torch.tensor(g, dtype=dtype, device="cuda:0")


def _with_workspace(x, inverse):
    import torch

    lib = mh.load_library()
    n = x.shape[0]
    dt = mh.F64 if x.dtype == torch.float64 else mh.F32
    need = ctypes.c_size_t(0)
    assert lib.mh_fft3_query_workspace(n, dt, ctypes.byref(need)) == mh.OK
    ws = torch.empty(need.value, dtype=torch.uint8, device=x.device)
    st = lib.mh_fft3(ctypes.c_void_p(x.data_ptr()), n, dt, int(inverse),
                     ctypes.c_void_p(ws.data_ptr()), need.value,
                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == mh.OK
    return x


def _no_alloc(x, inverse):
    import torch

    lib = mh.load_library()
    dt = mh.F64 if x.dtype == torch.float64 else mh.F32
    st = lib.mh_fft3_noalloc(ctypes.c_void_p(x.data_ptr()), x.shape[0], dt, int(inverse),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == mh.OK, mh.STATUS_NAMES[st]
    return x


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
@pytest.mark.parametrize("inverse", [0, 1])
def test_no_alloc_transform_equals_workspace_transform(dtype_name, inverse):
    import torch

    dtype = getattr(torch, dtype_name)
    # a larger cube first, then a smaller one: the second call rewrites the
    # head of the table and must not read what the first call left behind
    for call, n in enumerate((64, 16)):
        x = _cube(n, dtype, seed=10 * call + inverse)
        print(f"no-alloc fft: {dtype_name} n={n} inverse={inverse} call {call}", flush=True)
        ref = _with_workspace(x.clone(), inverse)
        got = _no_alloc(x.clone(), inverse)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, (got - ref).abs().max().item())
        # and against numpy's transform (the tolerances of the fft3 tests)
        xn = x.cpu().numpy()
        z = xn[..., 0] + 1j * xn[..., 1]
        zr = np.fft.ifftn(z) * n ** 3 if inverse else np.fft.fftn(z)
        g = got.cpu().numpy()
        err = np.abs(g[..., 0] + 1j * g[..., 1] - zr).max() / np.abs(zr).max()
        assert err < (1e-12 if dtype == torch.float64 else 2e-5), err


def test_no_alloc_rejects_bad_arguments():
    import torch

    lib = mh.load_library()
    x = _cube(8, torch.float32, seed=0)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(x.data_ptr())
    assert lib.mh_fft3_noalloc(None, 8, mh.F32, 0, s) == mh.E_INVALID
    assert lib.mh_fft3_noalloc(p, 8, mh.F32, 2, s) == mh.E_INVALID
    assert lib.mh_fft3_noalloc(p, 12, mh.F32, 0, s) == mh.E_SHAPE
    assert lib.mh_fft3_noalloc(p, 2048, mh.F32, 0, s) == mh.E_SHAPE
    assert lib.mh_fft3_noalloc(p, 8, 5, 0, s) == mh.E_DTYPE
    torch.cuda.synchronize()
