"""Sanitizer build of the library's host code, for the CPU test run.

The C-ABI layer (argument checks, shift tables, launch sequences) and the
host-only background code are compiled with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only (each sanitizer flag
follows -Xarch_host, so no device code is instrumented) and linked with the
regular objects of the other sources into libvlasov_san.so.  A process that
loads it must preload clang's ASan runtime (san_runtime()).  Run
``python -m paper_2110_15867_amd.build`` first (it leaves the objects).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

from . import build as B

LIB_SAN = os.path.join(B.HERE, "libvlasov_san.so")
HOST_SOURCES = ("capi.hip", "cosmo.hip")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]


def san_runtime() -> str:
    out = subprocess.run([B.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(out):
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        out = hits[0] if hits else out
    return out


def build(verbose: bool = False, out: str = LIB_SAN) -> str:
    objs = []
    for src in sorted(glob.glob(os.path.join(B.CSRC, "*.hip"))):
        name = os.path.basename(src)
        if name in HOST_SOURCES:
            obj = os.path.join(os.path.dirname(out), name + ".san.o")
            cmd = [B.HIPCC] + B.FLAGS + SAN + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        else:
            obj = os.path.join(B.BUILD, name + ".o")
            if not os.path.exists(obj):
                raise RuntimeError(f"{obj} missing: build the library first")
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC"] + SAN + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
