"""Compile libpipe.so (HIP for gfx950) in-tree.

Usage: python -m paper_1111_4971_amd.build   (or build() from Python).
Object files go to _build/ at the repository root; the shared library is
written next to this file.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpipe.so")
# (source, unit): the kernel files are compiled as two units each, FP32 kernels
# with the precision-independent code (PIPE_TU=1) and FP64 kernels (PIPE_TU=2)
SOURCES = [("xprod.hip", 1), ("xprod.hip", 2), ("passes.hip", 1), ("passes.hip", 2), ("band.hip", 1),
           ("band.hip", 2), ("fft3d.hip", 1), ("fft3d.hip", 2), ("green.hip", 0), ("pipe_api.cpp", 0)]
ARCH = os.environ.get("PIPE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            # never emit packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


def _compile(unit):
    src, tu = unit
    out = os.path.join(OBJ, "%s.%d.o" % (src, tu))
    cmd = [hipcc()] + flags() + (["-DPIPE_TU=%d" % tu] if tu else []) + ["-x", "hip", "-c",
                                                                        os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return out


def build(verbose=True):
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
