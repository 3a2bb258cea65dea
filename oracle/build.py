"""Compile the oracle's C source into ``oracle/liblsh_oracle.so`` (gcc, OpenMP).

-ffp-contract=off keeps every FP64 product and sum separately rounded, as the
source is written; no -ffast-math.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsh_oracle.c")
LIB_PATH = os.path.join(HERE, "liblsh_oracle.so")


def build() -> str:
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build())
