"""Build libauxprec.so (host setup with g++, HIP kernels with hipcc for gfx950) in-tree."""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libauxprec.so")

HOST_SOURCES = ["host/fem.cpp", "host/amg.cpp", "host/formats.cpp", "host/fuse.cpp", "host/stokes.cpp"]
HIP_SOURCES = ["hip/kernels.hip", "hip/prolong.hip", "hip/batched.hip", "hip/mfree.hip", "hip/krylov.hip", "hip/blockcg.hip",
               "hip/assemble.hip", "hip/amgsetup.hip", "hip/stokes.hip", "hip/solver.hip"]
ARCH = os.environ.get("AUXPREC_ARCH", "gfx950")

CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]) + " ...")
    return r


def build(verbose=False, jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    cmds, objs = [], []
    for s in HOST_SOURCES:
        o = os.path.join(OBJ, os.path.basename(s) + ".o")
        cmds.append(["g++"] + CXXFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(OBJ, os.path.basename(s) + ".o")
        cmds.append(["hipcc"] + HIPFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs, verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
