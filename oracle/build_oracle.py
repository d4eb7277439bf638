"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False) -> str:
    """The parity build (single thread) and the timing build with OpenMP over
    the messages of an evaluation (same arithmetic per message)."""
    # -O2 without -ffast-math: the oracle keeps IEEE semantics.
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        cmd = (["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra"] + extra +
               ["-o", out + ".tmp", SRC, "-lm"])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
