"""Build the FP64 CPU oracle (test infrastructure) with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "matcha_oracle.c")
OUT = os.path.join(HERE, "libmatcha_oracle.so")
# built on the machine that times it (the portable library above may be built elsewhere)
OUT_NATIVE = os.path.join(HERE, "libmatcha_oracle_native.so")


def build(verbose: bool = False, native: bool = False) -> str:
    """native: -march=native for the CPU timing on the host that runs it; otherwise a portable
    x86-64 build (the same library is loaded on other hosts)."""
    out = OUT_NATIVE if native else OUT
    arch = ["-march=native"] if native else []
    cmd = ["gcc", "-O3", *arch, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unused-function",
           SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
