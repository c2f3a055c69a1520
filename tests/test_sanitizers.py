"""CPU builds under the address and undefined-behaviour sanitizers: the FP64
oracle driven through every scheme, source and gravity option
(tests/sanitize/oracle_driver.c), and the C ABI's host-side argument
validation (tests/sanitize/abi_driver.c) with the sanitizers on the host pass
of the library sources that hold it.  No GPU is touched: the ABI driver only
calls what returns before a device is needed."""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2512_13403_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2512_13403_amd", "_build")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
ORACLE = ["oracle.c", "oracle_mg.c", "oracle_adjoint.c", "oracle_fft.c", "oracle_cool.c"]
# library sources holding C-ABI entry points, built with host sanitizers
ABI_SOURCES = ["api.hip", "corrector_api.hip", "fft_kernels.hip"]
LIB_SOURCES = ["api.hip", "hydro_kernels.hip", "step_kernels.hip", "mg_kernels.hip",
               "fft_kernels.hip", "cool_kernels.hip", "adjoint_kernels.hip",
               "corrector_kernels.hip", "corrector_api.hip"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", os.path.join(SAN, "oracle_driver.c")]
            + [os.path.join(ROOT, "oracle", f) for f in ORACLE] + ["-lm", "-o", exe])
        env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
        r = run([exe], env=env)
        assert "oracle driver: ok" in r.stdout


def test_abi_validation_under_sanitizers():
    others = [s for s in LIB_SOURCES if s not in ABI_SOURCES]
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in others]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the library has not been built (its kernel objects are reused)")
    with tempfile.TemporaryDirectory() as d:
        def compile_one(src):
            out = os.path.join(d, os.path.splitext(src)[0] + ".o")
            run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN
                + ["-c", os.path.join(CSRC, src), "-o", out])
            return out

        with ThreadPoolExecutor(max_workers=3) as ex:
            san_objs = list(ex.map(compile_one, ABI_SOURCES))
        drv = os.path.join(d, "abi_driver.o")
        run(["gcc", "-c", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", os.path.join(SAN, "abi_driver.c"), "-o", drv])
        exe = os.path.join(d, "abi_driver")
        run([HIPCC, "-O1", "-g", "--offload-arch=gfx950"] + HOST_SAN[:4]
            + [drv] + san_objs + objs + ["-o", exe])
        # the HIP runtime's own allocations are not this code's: no leak report
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        r = run([exe], env=env)
        assert "abi driver: ok" in r.stdout
