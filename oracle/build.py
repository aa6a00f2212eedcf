"""Build the FP64 oracle shared library (test infrastructure).

Compiles ``clbm_oracle.c`` and ``net_oracle.c`` (when present) with gcc into
``liboracle.so`` next to this file. Plain ``-O2``: no fast-math and no FMA
contraction, so the arithmetic is the order written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["clbm_oracle.c", "net_oracle.c"]


def build(verbose: bool = False, src_dir: str = HERE, out: str = LIB) -> str:
    """Compile the sources found in src_dir (default: this directory) into out."""
    srcs = [os.path.join(src_dir, s) for s in SOURCES if os.path.exists(os.path.join(src_dir, s))]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
