"""Build liblb.so (HIP kernels for gfx950 + host C++) in place.

Host sources are compiled with g++ (OpenMP), HIP sources with hipcc for
gfx950, and everything is linked against the HIP runtime.  Run as
``python -m paper_2111_10743_amd.build`` or through ``__graft_entry__.build``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblb.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SRC = ["refelem.cpp", "surface.cpp", "quadrature.cpp", "octree.cpp", "harmonics.cpp"]
HIP_HOST_SRC = ["api.cpp"]
HIP_SRC = ["kernels.hip", "octree.hip", "quadrature.hip", "calculus.hip", "noalloc.hip"]

CXXFLAGS = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-Wall", "-Wno-unused-function"]
HIPFLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    for s in HOST_SRC:
        o = os.path.join(OUT, s + ".o")
        jobs.append(["g++"] + CXXFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_HOST_SRC:
        o = os.path.join(OUT, s + ".o")
        jobs.append(["g++"] + CXXFLAGS + ["-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
                                         "-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SRC:
        o = os.path.join(OUT, s + ".o")
        jobs.append([os.path.join(ROCM, "bin", "hipcc")] + HIPFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    workers = min(8, int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(OUT, s + ".o") for s in HOST_SRC + HIP_HOST_SRC + HIP_SRC]
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-fopenmp", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
