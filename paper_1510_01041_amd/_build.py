"""Build step for the HIP library (gfx950 only).

    python -m paper_1510_01041_amd._build

Compiles csrc/lms.hip into liblms.so next to this file. Packed FP32 VALU
instructions are disabled on purpose (-packed-fp32-ops), and contraction is
off so that every FP64 multiply-add is an explicit fma, as in the reference.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("lms.hip", "lms_batched.hip", "lms_net.hip", "lms_alg1.hip", "lms_sample.hip", "lms_hough.hip",
                                                    "lms_host.cpp")]
LIB = os.path.join(HERE, "liblms.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-pass-failed",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC, *FLAGS, *extra, "-o", LIB + ".tmp", *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
