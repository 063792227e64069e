"""Build the FP64 CPU oracle (test infrastructure) into oracle/liborc.so.

Run as ``python oracle/build.py``; ``__graft_entry__.build()`` calls
:func:`build` as well.  The oracle is compiled without floating-point
contraction so that every operation rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
OUT = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
        "-o", OUT + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
