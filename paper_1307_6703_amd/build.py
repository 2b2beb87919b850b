"""Build the HIP library liblbvdw.so (gfx950) in-tree.

Compiles the HIP sources of csrc/ (lattice step, C ABI, batch, the D2Q17
variant, surrogate) with hipcc for gfx950 only.
Packed FP32 instructions are disabled for device code. Multiply-adds fuse only
within one source expression (-ffp-contract=on), so the arithmetic of a node
does not depend on how the compiler lays out a kernel instance: every launch
shape gives bitwise-identical results.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbvdw.so")
SOURCES = ["lb_device.hip", "lb_api.hip", "lb_batch.hip", "d17_device.hip", "d17_api.hip",
           "sg_device.hip", "sg_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def build(verbose: bool = False) -> str:
    """Compile every HIP source into liblbvdw.so next to this file."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
