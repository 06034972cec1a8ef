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
           "features.hip", "explicit.hip", "newton.hip", "newton_gen.hip", "adjoint.hip", "adjoint_split.hip",
           "leverage.hip"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def command(out=LIB, csrc=CSRC):
    """Single-invocation compile-and-link command (for reference and tools)."""
    srcs = [os.path.join(csrc, s) for s in SOURCES]
    return [hipcc()] + FLAGS + ["-shared", "-I" + INCLUDE, "-I" + csrc, "-o", out] + srcs + ["-lrocblas"]


def build(verbose=False, out=LIB, csrc=CSRC, jobs=None):
    """Compile every source (in parallel) and link libnyls.so; always recompiles."""
    import concurrent.futures
    import tempfile
    cc = hipcc()
    objdir = tempfile.mkdtemp(prefix="nyls_build_")
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + FLAGS + ["-I" + INCLUDE, "-I" + csrc, "-c", os.path.join(csrc, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, res

    try:
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for src, _, res in results:
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed compiling " + src)
            if verbose:
                sys.stderr.write(res.stderr)
        tmp = out + ".tmp"
        link = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results] + ["-lrocblas"]
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libnyls.so")
        os.replace(tmp, out)
    finally:
        for name in os.listdir(objdir):
            os.remove(os.path.join(objdir, name))
        os.rmdir(objdir)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
