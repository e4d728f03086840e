"""Build libfk.so (the HIP kernels and the C ABI) in-tree for gfx950.

hipcc flags: -O3, -ffp-contract=off (every product and sum rounded as
written; fma only where the code asks for it), packed-FP32 instructions
disabled, position-independent shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["fk_kernels.hip", "fk_capi.hip", "fk_net.hip", "fk_batch.hip"]
ARCH = os.environ.get("FK_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def library_path() -> str:
    return os.path.join(HERE, "libfk.so")


def extra_flags() -> list[str]:
    """Additional hipcc flags from FK_HIPCC_FLAGS (tuning experiments)."""
    return os.environ.get("FK_HIPCC_FLAGS", "").split()


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr, flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so.
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"command failed ({res.returncode}): {' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, out: str | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(ROOT, "_build", os.path.basename(out or "libfk.so"))
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, src.replace(".hip", ".o")) for src in SOURCES]
    # the sources compile independently: one hipcc per source, side by side
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        jobs = [pool.submit(_run, [hipcc, *HIPCC_FLAGS, *extra_flags(), "-c", os.path.join(CSRC, src),
                                   "-o", obj], verbose)
                for src, obj in zip(SOURCES, objs)]
        for j in jobs:
            j.result()
    out = out or library_path()
    tmp = out + f".tmp{os.getpid()}"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, out=sys.argv[1] if len(sys.argv) > 1 else None))
