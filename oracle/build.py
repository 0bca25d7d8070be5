"""Build the FP64 oracle shared library with gcc.

Test infrastructure only: the oracle is the independent reference for the
parity tests, the smoke check and the CPU-baseline timing.  The product
library never loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(force=True):
    """Compile lbm_oracle.c -> liblbm_oracle.so (OpenMP, strict IEEE FP64)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-std=c11",
           "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
