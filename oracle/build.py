"""Build the CPU oracle (plain C, OpenMP) into oracle/liboracle.so.

Test infrastructure only; see oracle/__init__.py.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isci_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile the oracle; ``defines`` is only used by the mutation test."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]
    cmd += [f"-D{d}" for d in defines]
    cmd += ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
