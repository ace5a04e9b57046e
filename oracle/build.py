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
# the same sources built with AddressSanitizer and UndefinedBehaviorSanitizer
# (gcc's runtimes; a process loading it must preload libasan)
LIB_SAN = os.path.join(HERE, "liboracle_vlasov_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]
SOURCES = [os.path.join(HERE, "vlasov_oracle.c"), os.path.join(HERE, "vlasov_oracle_adj.c")]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    srcs = [s for s in SOURCES if os.path.exists(s)]
    out = out or (LIB_SAN if sanitize else LIB)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas"] + (SAN_FLAGS if sanitize else []) + ["-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
