"""Build liblbm_em.so (gfx950) with hipcc, in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_em.so")
SOURCES = [os.path.join(CSRC, "lbm_em.hip")]
DEPENDS = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + [
    os.path.join(os.path.dirname(HERE), "include", "lbm_em.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every operation rounded on its own: results do not depend on where the
    # shared per-cell update is inlined (single, batched, any tile)
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(force=True, verbose=False):
    """Compile every HIP source into paper_2510_11042_amd/liblbm_em.so."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in DEPENDS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
