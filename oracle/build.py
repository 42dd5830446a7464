"""Build the plain-C FP64 oracle (the Eulerian step in ``sale_oracle.c``, the
pure-Lagrangian step in ``lagrange_oracle.c``) into ``oracle/liboracle.so``
with gcc.

Test infrastructure: the oracle is the checker of the HIP path, never a part
of it. Flags: no fast-math and no FP contraction, so every operation rounds
exactly as written; OpenMP for the independent per-cell/per-node loops.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sale_oracle.c")
SRC_LAG = os.path.join(HERE, "lagrange_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build_oracle(verbose: bool = False) -> str:
    """Compile the oracle (always; it takes about a second) and return the path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, SRC_LAG, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
