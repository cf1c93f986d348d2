"""Build the synthetic-workload generator (plain C + OpenMP, gcc)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "plummer.c")
LIB = os.path.join(HERE, "libcsk_workloads.so")
GPU_SRC = os.path.join(HERE, "plummer_gpu.hip")
GPU_LIB = os.path.join(HERE, "libcsk_workloads_gpu.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    gcmd = ["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", GPU_LIB + ".tmp", GPU_SRC]
    if verbose:
        print(" ".join(gcmd), flush=True)
    subprocess.run(gcmd, check=True)
    os.replace(GPU_LIB + ".tmp", GPU_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
