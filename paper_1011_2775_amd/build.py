"""Build libwcmg.so (HIP, gfx950) in-tree.

Usage: python -m paper_1011_2775_amd.build   (or build() from Python)

Every source under csrc/ is compiled with hipcc for gfx950 into
paper_1011_2775_amd/lib/libwcmg.so.  Packed FP32 instructions are disabled
(-target-feature -packed-fp32-ops) for all device code.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libwcmg.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["dslash.hip", "fields.hip", "blas.hip", "blas_batch.hip", "transfer.hip", "coarse.hip", "coarse_mfma.hip", "coarse_multilevel.hip", "coarse_persist.hip", "random.hip", "force.hip", "noalloc.hip",
           "runtime.cpp", "solvers.cpp", "capi.cpp"]

ARCH = os.environ.get("WCMG_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["-x", "hip", "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + INCLUDE, "-I" + CSRC]


def _compile(src, objdir, verbose):
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), p.stdout, p.stderr))
    if verbose and p.stderr.strip():
        err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l
                        and "not a recognized feature" not in l)
        if err.strip():
            print(err, file=sys.stderr)
    return obj


def build(verbose=False, jobs=None):
    """Compile all sources and link lib/libwcmg.so; returns the library path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (p.stdout, p.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
