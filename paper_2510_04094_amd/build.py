"""Build libnyls.so (all HIP sources, gfx950) in-tree with hipcc.

    python -m paper_2510_04094_amd.build

Packed FP32 instructions are disabled on purpose (-packed-fp32-ops): the kernels'
FP32 work runs as scalar VALU or MFMA.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnyls.so")
SOURCES = ["api.hip", "eig.hip", "gram64.hip", "gram32.hip", "kkt.hip", "points.hip",
           "features.hip", "explicit.hip", "newton.hip", "adjoint.hip"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def command(out=LIB):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    return [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + INCLUDE, "-I" + CSRC, "-o", out] + srcs + ["-lrocblas"]


def build(verbose=False):
    """Compile every source into libnyls.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnyls.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
