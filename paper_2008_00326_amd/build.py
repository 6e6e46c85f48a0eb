"""Builds the gfx950 HIP library libperch.so (in-tree) and the sensor simulator."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libperch.so")
ARCH = os.environ.get("PERCH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",                       # bit-exact geometry: no FMA contraction
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build_hip(verbose: bool = False) -> str:
    src = [os.path.join(HERE, "csrc", "perch_runtime.cpp"), os.path.join(HERE, "csrc", "perch_kernels.hip"),
           os.path.join(HERE, "csrc", "perch_icp.hip"), os.path.join(HERE, "csrc", "perch_msg.hip"),
           os.path.join(HERE, "csrc", "perch_knn1.hip")]
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", tmp, *src,
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build(verbose: bool = False) -> None:
    from .workloads import sensor
    sensor.build(verbose)
    build_hip(verbose)


if __name__ == "__main__":
    build(verbose=True)
