"""Build liblbm_em.so (gfx950) with hipcc, in-tree.

Every HIP source in csrc/ is compiled to an object of its own, in parallel
(the kernel families live in separate translation units), then linked.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_em.so")
SOURCES = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
DEPENDS = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h", ".inc"))] + [
    os.path.join(os.path.dirname(HERE), "include", "lbm_em.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every operation rounded on its own: results do not depend on where the
    # shared per-cell update is inlined (single, batched, any tile)
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def _jobs():
    try:
        return max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))
    except ValueError:
        return 1


def build(force=True, verbose=False):
    """Compile every HIP source into paper_2510_11042_amd/liblbm_em.so."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in DEPENDS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    with tempfile.TemporaryDirectory(prefix="lbm_em_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s)[:-4] + ".o") for s in SOURCES]
        cmds = [["hipcc", *HIPCC_FLAGS, "-c", s, "-o", o] for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd).returncode

        with ThreadPoolExecutor(_jobs()) as ex:
            codes = list(ex.map(run, cmds))
        if any(codes):
            raise subprocess.CalledProcessError(max(codes), "hipcc")
        tmp = LIB + ".tmp"
        link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
