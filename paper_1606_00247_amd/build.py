"""Build libtetfmm.so (HIP kernels for gfx950 + host plan + C ABI) in-tree.

    python -m paper_1606_00247_amd.build [-v]

The host plan is compiled with g++ and no floating-point contraction (its
discrete decisions must be reproducible); the HIP sources with hipcc for
gfx950 with hardware FP64 atomics and packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtetfmm.so")
ARCH = os.environ.get("TFMM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False, jobs=4):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    plan_o = os.path.join(BUILD, "plan.o")
    cmds = [["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o]]
    objs.append(plan_o)
    for src in ("kernels.hip", "surrogate.hip", "capi.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmds.append(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        procs.append(subprocess.Popen(c))
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError(f"compilation failed: {rc}")
    _run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
