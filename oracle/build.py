"""Builds liboracle.so (plain C, gcc, OpenMP) next to this file.

Test infrastructure: the oracle is compiled here so that the checker exists
wherever the tests run; nothing in the product library links it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.c", "oracle_mg.c", "oracle_adjoint.c", "oracle_fft.c", "oracle_cool.c"]


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
