"""Compile the FP64 CPU oracle (test infrastructure) into liboracle_vlasov.so.

Run as ``python oracle/build.py`` or through ``__graft_entry__.build()``.
Contraction of a*b+c into fused multiply-adds is switched off so that the
oracle's shift formulas round exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_vlasov.so")
SOURCES = [os.path.join(HERE, "vlasov_oracle.c"), os.path.join(HERE, "vlasov_oracle_adj.c")]


def build(verbose: bool = False) -> str:
    srcs = [s for s in SOURCES if os.path.exists(s)]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
