"""Compile the C oracle (test infrastructure) into oracle/liborc.so.

gcc -O2 -ffp-contract=off: no fused multiply-add, so the oracle rounds every
product and sum exactly as written.  -fopenmp only serves the timing mode
(orc_cg_csr_omp); every other function is serial.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cg_oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build(out=LIB, extra=()):
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm", *extra]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)  # a new file: a process that has the old one loaded keeps it
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
