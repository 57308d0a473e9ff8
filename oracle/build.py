"""Build the oracle shared library with gcc (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
          "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, "-o", SO + ".tmp", os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
