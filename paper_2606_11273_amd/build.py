"""Build the HIP library libmfs_hip.so in-tree for gfx950 (hipcc, no JIT).

Usage: python -m paper_2606_11273_amd.build   (or build() from Python).
Every call recompiles.  Objects go to paper_2606_11273_amd/_build/.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmfs_hip.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_SOURCES = ["kernels.hip", "precompute.hip", "capi.hip", "gmres.hip", "flow.hip", "server.hip", "fmm_tree.hip"]
CXX_SOURCES = ["geometry.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{ROCM}/include", f"-I{os.path.join(HERE, '..', 'include')}",
    # the ROCm library directory the library is built against (its rocSOLVER is resolved there)
    f"-DMFS_ROCM_LIB=\"{os.path.realpath(os.path.join(ROCM, 'lib'))}\"",
]


def _hipcc():
    p = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; the HIP library needs ROCm")
    return p


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    for f in HIP_SOURCES:
        obj = os.path.join(BUILD, f + ".o")
        jobs.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(SRC, f), "-o", obj])
    for f in CXX_SOURCES:
        obj = os.path.join(BUILD, f + ".o")
        jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(SRC, f), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    objs = [j[-1] for j in jobs]
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp, f"-L{ROCM}/lib",
          "-lrocsolver", "-lrocblas", "-ldl", "-pthread", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
