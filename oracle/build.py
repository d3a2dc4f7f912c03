"""Compile the C oracle into ``oracle/libsdm_oracle.so`` with gcc (OpenMP, FP64,
no fast-math, no FMA contraction)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libsdm_oracle.so")
SOURCES = ["sdm_oracle.c", "slab_mc.c", "mlp.c"]


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", SO + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


def ensure_built():
    """Build only when no library is there (``build()`` always rebuilds)."""
    if not os.path.exists(SO):
        build()
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
