"""Builds liblt.so (host runtime + gfx950 kernels) in-tree.

Host C++ is compiled with g++ against the HIP runtime headers; the kernels
with hipcc for gfx950.  Packed FP32 instructions are disabled for the GPU
code (``-Xclang -target-feature -Xclang -packed-fp32-ops``) and no multiply
and add are fused unless the source writes fmaf (``-ffp-contract=off``).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "liblt.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SRC = ["annot.cpp", "plan.cpp", "memory.cpp", "exec.cpp", "api.cpp", "serve.cpp", "rtc.cpp", "bounce.cpp"]
HIP_SRC = ["kernels.hip", "gemm.hip", "drain.hip", "reduce.hip"]

HOST_FLAGS = ["-O2", "-g", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-D__HIP_PLATFORM_AMD__", "-I" + INC, "-I" + CSRC, "-I" + os.path.join(ROCM, "include")]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INC, "-I" + CSRC, "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), p.stdout))
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for f in HOST_SRC:
        src = os.path.join(CSRC, f)
        if not os.path.exists(src):
            continue
        obj = os.path.join(BUILD, f + ".o")
        jobs.append((["g++"] + HOST_FLAGS + ["-c", src, "-o", obj], obj))
    for f in HIP_SRC:
        src = os.path.join(CSRC, f)
        if not os.path.exists(src):
            continue
        obj = os.path.join(BUILD, f + ".o")
        jobs.append(([os.path.join(ROCM, "bin", "hipcc")] + HIP_FLAGS + ["-c", src, "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([os.path.join(ROCM, "bin", "hipcc"), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp]
         + [j[1] for j in jobs] + ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lhiprtc",
                                   "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
