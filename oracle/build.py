"""Compile the oracle's C sources into a shared library (test infrastructure).

The oracle is plain C99 built with -O2 and -ffp-contract=off so that no
multiply-add is fused; OpenMP only splits the row loops across host threads.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "lb_oracle.c"), os.path.join(HERE, "d2q17_oracle.c")]
HDRS = [os.path.join(HERE, "lb_oracle.h")]
LIB = os.path.join(HERE, "liblb_oracle.so")


def build(force: bool = True) -> str:
    """Build liblb_oracle.so next to this file and return its path."""
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(f) for f in SRCS + HDRS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, *SRCS, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
