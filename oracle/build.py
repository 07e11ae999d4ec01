"""Compile the C oracle (test infrastructure) into oracle/liborc.so.

gcc -O2 -ffp-contract=off: no fused multiply-add, so the oracle rounds every
product and sum exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cg_oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build(out=LIB, extra=()):
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out, SRC, "-lm", *extra]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
