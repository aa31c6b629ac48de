"""Compile the CPU oracle (mpref.c) into oracle/libmpref.so with gcc.

Strict IEEE binary64: -ffp-contract=off (no fused multiply-add except the
explicit fma() calls), no fast-math; x86-64 scalar SSE2 arithmetic.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpref.c")
OUT = os.path.join(HERE, "libmpref.so")


OUT_SAN = os.path.join(HERE, "libmpref_san.so")
# the checked build: AddressSanitizer and UndefinedBehaviorSanitizer, traps
# on the first report; load it with MPREF_LIB=san and the sanitizer runtime
# preloaded into the Python process (LD_PRELOAD=$(gcc -print-file-name=libasan.so))
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = OUT_SAN if sanitize else OUT
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]
    if sanitize:
        cmd += SAN_FLAGS
    cmd += ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
