"""Compile the HIP library libgrlbm.so for gfx950 with hipcc (in-tree).

The library holds every kernel of the solver and the C ABI of include/grlbm.h.
Packed-FP32 instructions are disabled for all device code.  Multiply-adds are
fused only inside one source expression (-ffp-contract=on): the collision is
inlined into several kernels (the two AA parities, the row-staged odd step, the
batch kernel) and with the compiler's default cross-statement fusion
each copy could round differently; this way every kernel computes a cell update
with the same FP32 operations and the paths agree bit for bit.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgrlbm.so")
SOURCES = ["grlbm_kernels.hip", "grlbm_api.hip", "grlbm_batch.hip", "grlbm_mms.hip"]
ARCH = "gfx950"


def hipcc_cmd(out, extra=()):
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
             "-Wall", "-Wno-unused-function", f"-I{os.path.join(HERE, '..', 'include')}"]
            + list(extra) + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def build(verbose: bool = False) -> str:
    """Always recompile; returns the path of the shared library."""
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
