"""Compile the C oracle into oracle/libraysh_oracle.so (test infrastructure).

The flags keep every floating-point operation a single IEEE-rounded one:
no fast-math, no FMA contraction, no vectorisation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "raysh_oracle.c")
LIB = os.path.join(HERE, "libraysh_oracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fno-tree-vectorize",
          "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build_oracle(extra_flags=(), out=LIB, src=SRC):
    """Compile the oracle; returns the path of the shared library."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle())
