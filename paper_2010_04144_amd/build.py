"""Build ``libhemelb_hip.so`` (the C-ABI library) for gfx950 with hipcc.

The library is built in-tree next to this file.  Flags:
  --offload-arch=gfx950        MI355X (CDNA4) code objects only
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no packed FP32 instructions (v_pk_*_f32)
  -fno-gpu-flush-denormals-to-zero
                               keep FP32 subnormals (small offsets in the
                               FP16/FP32 offset storage)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhemelb_hip.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-I", INC, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-flush-denormals-to-zero", "-Wall", "-Wno-unused-result"]
SOURCES = ["hl_kernels.hip", "hl_api.cpp", "hl_layout.cpp", "hl_ceiling.hip"]


def build(verbose=False, extra=()):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
