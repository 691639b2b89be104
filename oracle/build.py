"""Builds the oracle's shared library (``oracle/liboracle.so``) with g++.

Portable x86-64 code (no -march=native: the library may run on another host),
IEEE double with FP contraction off and no fast-math, so every result is the
plainly rounded value of the written expression.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tl_oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wextra"]


def build(src=SRC, out=OUT, verbose=False):
    """Compile ``src`` into the shared library ``out``; returns ``out``."""
    tmp = out + ".tmp"
    cmd = ["g++", *FLAGS, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
