"""Build the oracle's C integral engine (test infrastructure only).

    python oracle/build.py

produces ``oracle/liboracle.so`` with gcc -O2 -fopenmp.  No GPU code is
involved and nothing here is shared with the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "md_ints.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose=False, out=None, sanitize=False):
    """Compile md_ints.c to `out` (default liboracle.so).  sanitize=True makes
    an AddressSanitizer + UndefinedBehaviorSanitizer build (-O1, frame
    pointers kept, no OpenMP) for the tests that run the oracle under it."""
    out = out or OUT
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2", "-fopenmp"]
    cmd = ["gcc"] + opt + ["-fPIC", "-shared", "-std=c99", "-Wall", "-Wno-unused-variable",
                           "-Wno-unknown-pragmas", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
