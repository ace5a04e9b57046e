"""The C-ABI library loads and exports every entry point its header declares.

Runs without a GPU: only host-side entry points that return before touching
the device are called (version, error strings, sizes, argument checks).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vlasov.h")
LIB = os.environ.get("VLASOV_LIB", os.path.join(ROOT, "paper_2110_15867_amd", "libvlasov.so"))


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vlasov_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libvlasov.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = _declared()
    for want in ["vlasov_advect_x", "vlasov_advect_uz", "vlasov_step", "vlasov_moments",
                 "vlasov_strerror", "vlasov_abi_version"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_entry_points(lib):
    lib.vlasov_strerror.restype = ctypes.c_char_p
    assert lib.vlasov_abi_version() == 1
    for code in range(-8, 1):
        assert lib.vlasov_strerror(code)
    import sys

    sys.path.insert(0, ROOT)
    from paper_2110_15867_amd import vlasov as V

    g = V.make_grid((4, 4, 4), (8, 8, 8))
    assert V.vlasov_f_bytes(g, V.F32) == 4 ** 3 * 8 ** 3 * 4
    assert V.vlasov_f_bytes(g, V.F16) == 4 ** 3 * 8 ** 3 * 2
    assert V.vlasov_scale_bytes(g, V.BF16) == 4 ** 3 * 8 ** 2 * 4
    assert V.vlasov_scale_bytes(g, V.F32) == 0
    assert V.vlasov_step_workspace_bytes(g, V.F32) % 256 == 0
    # argument checks fail before any device call
    L = V.lib()
    assert L.vlasov_advect_x(None, 0, None, None, None, None, 0.1, None) == -1
    assert L.vlasov_step(ctypes.byref(g), 0, 0, None, None, None, None, None, None, 0.1, 1.0,
                         None, 0, None, None) == -1
    bad = V.make_grid((4, 0, 4), (8, 8, 8))
    assert L.vlasov_moments(ctypes.byref(bad), 0, None, None, None, None, None, None) == -2
    assert L.vlasov_dispersion(None, 0, None, None, None, None, None, None) == -1
    assert L.vlasov_dispersion(ctypes.byref(bad), 0, None, None, None, None, None, None) == -2
    assert L.vlasov_dispersion(ctypes.byref(g), 0, ctypes.c_void_p(256), None,
                               ctypes.c_void_p(512), None, None, None) == -1


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2110_15867_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liboracle" not in text and "vlasov_oracle" not in text, fn
