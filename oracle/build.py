"""Compile the CPU oracle (oracle.c) into liboracle.so next to this file.

Test infrastructure only.  gcc, -O2, no FMA contraction (-ffp-contract=off):
each product and sum in the oracle is rounded on its own.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src: str | None = None, out: str | None = None) -> str:
    """Compile `src` (default: oracle.c) into `out` (default: liboracle.so)."""
    src = src or os.path.join(HERE, "oracle.c")
    out = out or library_path()
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_timing(out: str, src: str | None = None, verbose: bool = False) -> str:
    """The timing build of the same source: -O3 for the machine it runs on,
    OpenMP on (which adds oracle_cg_classical_omp), still without FMA
    contraction.  Timing only; parity uses the build above."""
    src = src or os.path.join(HERE, "oracle.c")
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-std=c11", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
