"""Build ``libspgm.so`` (HIP, gfx950) in place from ``csrc/spgm.hip``.

Packed FP32 instructions are disabled (``-packed-fp32-ops``): the kernels are written with
scalar float arithmetic and must not be turned into v_pk_* forms by the compiler.

The machine scheduler runs its instruction-level-parallelism strategy (``max-ilp``): the tile
kernels are bound by VALU issue, and ordering each row's independent sin/cos and FMA chains
for latency rather than register pressure made the adjoint tile about 5 % faster on gfx950
(forward unchanged) with no change of occupancy.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "spgm.hip")
LIB = os.path.join(HERE, "libspgm.so")
ARCH = os.environ.get("SPGM_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out):
    return ["hipcc", "-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-sched-strategy=max-ilp",
            "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-o", out, SRC]


def build(verbose: bool = False) -> str:
    """Compile ``libspgm.so`` (always recompiles) and return its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libspgm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
