"""Build of the HIP library libcog.so (gfx950) in-tree.

The flags fix the numerics the method's discrete decisions depend on:
no floating-point contraction, IEEE denormals, correctly rounded fp32
division; packed-fp32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcog.so")
SOURCES = [os.path.join(CSRC, "cog_kernels.hip"), os.path.join(CSRC, "cog_api.cpp"),
           os.path.join(CSRC, "cog_batch.cpp"), os.path.join(CSRC, "cog_server.cpp")]
HEADERS = [os.path.join(CSRC, "cog_device.h"), os.path.join(CSRC, "cog_ctx.h"),
           os.path.join(ROOT, "include", "cog.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
