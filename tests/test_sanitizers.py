"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds of the same sources, each exercised by the existing CPU tests in a
child process that preloads the matching sanitizer runtime:
- the FP64 oracle (C, gcc's runtimes) under its pin tests of the scheme and
  the adjoint;
- the library's host code (C-ABI argument checks, shift tables, background
  expansion; clang's runtimes, device code untouched) under the ABI and
  background tests.
Any report aborts the child (recovery is off for undefined behaviour), so the
child's exit status is the verdict.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import build as ob

    lib = ob.build(sanitize=True, out=str(tmp_path / "liboracle_vlasov_san.so"))
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt):
        pytest.skip("gcc's libasan not found")
    _child({"LD_PRELOAD": rt, "VLASOV_ORACLE_LIB": lib},
           ["tests/test_oracle_scheme.py", "tests/test_oracle_adjoint.py"])


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2110_15867_amd import build as B
    from paper_2110_15867_amd import build_san as S

    if not os.path.isdir(B.BUILD) or not any(n.endswith(".hip.o") for n in os.listdir(B.BUILD)):
        pytest.skip("library objects not built (run __graft_entry__.build())")
    lib = S.build(out=str(tmp_path / "libvlasov_san.so"))
    rt = S.san_runtime()
    if not os.path.exists(rt):
        pytest.skip("clang's ASan runtime not found")
    _child({"LD_PRELOAD": rt, "VLASOV_LIB": lib},
           ["tests/test_abi.py", "tests/test_cosmo_host.py"])
