"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so.

Flags matter for parity: -ffp-contract=off keeps every multiply and add
separately rounded, and -ffast-math is never used (it would flush denormals
on x86 and allow reassociation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mknn_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-pthread", "-Wall", "-Wextra"]


def build(verbose=False):
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
