"""Compile the plain-C oracle into ``oracle/liboracle.so`` (gcc, OpenMP).

Test infrastructure only: the product library never links or loads it.
The default build is generic x86-64 code (no ``-march=native``) so the
library built here also runs on any host it is copied to; ``native=True``
builds ``liboracle_native.so`` with ``-O3 -march=native`` for the host it
runs on (the timed CPU baseline builds it there).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NATIVE_LIB = os.path.join(HERE, "liboracle_native.so")


def build(verbose: bool = False, native: bool = False) -> str:
    out = NATIVE_LIB if native else LIB
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
