"""Build libfvna.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fvna_runtime.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "fvna_device.hpp"), os.path.join(HERE, "csrc", "fvna_step.hpp"),
        os.path.join(os.path.dirname(HERE), "include", "fvna.h")]
LIB = os.path.join(HERE, "libfvna.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every rounding is the one written in the source: no FMA contraction
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # instruction scheduling for ILP: the step kernel is bound by VALU issue
    # (measured 1-2% faster FP32 step kernels than the default strategy;
    # scheduling only reorders, results are bitwise unchanged)
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, extra=()):
    """Compile every time it is called (the caller decides when)."""
    cmd = ["hipcc", *FLAGS, *extra, "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
