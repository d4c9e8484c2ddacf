"""Build ``libssa.so`` (the C-ABI library of include/ssa.h) for gfx950 with hipcc, in-tree.

Flags that matter for the arithmetic contract: -ffp-contract=off (clang's HIP default
would fuse a*b+c), no fast-math.  Packed FP32 instructions are disabled (the code is FP64
and integer; the flag keeps the compiler from forming them anywhere).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ssa_api.hip")
DEPS = [os.path.join(HERE, "csrc", f) for f in ("ssa_api.hip", "ssa_kernels.hpp", "ssa_sim.hpp", "ssa_jit.hpp",
                                                "ssa_device.hpp", "ssa_wave.hpp")] + \
    [os.path.join(ROOT, "include", "ssa.h")]
LIB = os.path.join(HERE, "libssa.so")
ARCH = os.environ.get("SSA_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-c23-extensions"]


def build(verbose=True, extra=()):
    """Always compiles (the build check is that this succeeds)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + list(extra) + ["-o", tmp, SRC, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("hipcc failed (exit %d)" % r.returncode)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


def is_stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    build()
