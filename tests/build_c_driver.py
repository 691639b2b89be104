"""Builds tests/c_abi_driver.cpp (a test of the C ABI without Python, checked
against the oracle) into tests/_build/c_abi_driver, linked against the
in-tree libtl.so and oracle/liboracle.so through $ORIGIN-relative run paths."""
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_abi_driver.cpp")
OUT = os.path.join(HERE, "_build", "c_abi_driver")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
STAMP = OUT + ".sources"
SOURCES = (SRC, os.path.join(ROOT, "include", "tl.h"))


def sources_digest():
    """sha256 of the driver's source and of the header it is compiled against."""
    h = hashlib.sha256()
    for path in SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), SRC, "-o", OUT + ".tmp",
           "-L", os.path.join(ROOT, "paper_1804_10120_amd"), "-ltl",
           "-L", os.path.join(ROOT, "oracle"), "-loracle",
           "-Wl,-rpath,$ORIGIN/../../paper_1804_10120_amd", "-Wl,-rpath,$ORIGIN/../../oracle"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(OUT + ".tmp", OUT)
    with open(STAMP, "w") as f:
        f.write(sources_digest())
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
