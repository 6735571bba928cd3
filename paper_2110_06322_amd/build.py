"""Build the HIP/C++ library libcpm.so in-tree for gfx950.

Host C++ (band build, setup, solver orchestration) is compiled by g++ with
OpenMP and without floating-point contraction; HIP kernels by hipcc for
gfx950 with packed-FP32 instructions disabled; hipcc links the shared object.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcpm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("CPM_OFFLOAD_ARCH", "gfx950")

CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def sources():
    files = sorted(os.listdir(CSRC))
    return ([os.path.join(CSRC, f) for f in files if f.endswith(".cpp")],
            [os.path.join(CSRC, f) for f in files if f.endswith(".hip")])


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link libcpm.so; returns the library path."""
    os.makedirs(OBJ, exist_ok=True)
    cpp, hip = sources()
    cmds = []
    for s in cpp:
        o = os.path.join(OBJ, os.path.basename(s) + ".o")
        cmds.append((["g++"] + CXX_FLAGS + ["-c", s, "-o", o], o))
    for s in hip:
        o = os.path.join(OBJ, os.path.basename(s) + ".o")
        cmds.append(([f"{ROCM}/bin/hipcc"] + HIP_FLAGS + ["-c", s, "-o", o], o))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(lambda c: _run(c[0]), cmds))
    if verbose:
        for (c, _), o in zip(cmds, outs):
            print(" ".join(c))
            if o.strip():
                print(o)
    gomp = subprocess.run(["g++", "-print-file-name=libgomp.so"], stdout=subprocess.PIPE,
                          text=True).stdout.strip()
    tmp = LIB + ".tmp"
    link = [f"{ROCM}/bin/hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + \
        [o for _, o in cmds] + [gomp, f"-Wl,-rpath,{os.path.dirname(gomp)}", f"-L{ROCM}/lib", "-lamdhip64"]
    _run(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
