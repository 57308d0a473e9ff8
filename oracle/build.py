"""Build the oracle shared library with gcc/g++ (test infrastructure only):
oracle.c (the plain C oracle), compress.c (cluster compression) and
adjoint.cc (the double-precision refit differentiated by a recorded tape)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")
# -mfma: the explicit fmaf/fma calls of the Kalman arithmetic become the x86
# fused multiply-add instruction (the same single rounding as the library
# call); with contraction off nothing else is fused
FPFLAGS = ["-O2", "-Wall", "-Wextra", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-mfma"]


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    c_obj = os.path.join(objdir, "oracle.o")
    z_obj = os.path.join(objdir, "compress.o")
    cc_obj = os.path.join(objdir, "adjoint.o")
    cmds = [
        ["gcc", "-std=c11", *FPFLAGS, "-fexcess-precision=standard", "-c", os.path.join(HERE, "oracle.c"), "-o", c_obj],
        ["gcc", "-std=c11", *FPFLAGS, "-fexcess-precision=standard", "-Wno-unused-function",
         "-c", os.path.join(HERE, "compress.c"), "-o", z_obj],
        ["g++", "-std=c++17", *FPFLAGS, "-Wno-unused-function", "-c",
         os.path.join(HERE, "adjoint.cc"), "-o", cc_obj],
        ["g++", "-shared", "-fPIC", "-o", SO + ".tmp", c_obj, z_obj, cc_obj, "-lm"],
    ]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
