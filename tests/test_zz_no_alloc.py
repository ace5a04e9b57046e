"""vlasov_field_noalloc (the allocation-free entry point) through the C ABI.

Two calls in a row -- a 32 x 24 x 16 mesh, then a smaller 8 x 12 x 6 one --
each against vlasov_field with a caller workspace on the same input: the same
kernels on the same data, so the results agree bit for bit whatever the
previous call left in the fixed array.  A mesh too large for the array is
refused.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


def _case(n, L, coupling, seed):
    hg = V.make_grid(n, (4, 4, 4), L)
    rng = np.random.default_rng(seed)
    rho = torch.from_numpy(1.0 + 0.3 * rng.standard_normal(n)).cuda()
    ref = torch.empty((3,) + tuple(n), dtype=torch.float32, device="cuda")
    nb = V.vlasov_field_workspace_bytes(hg)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    V.vlasov_field(hg, rho, coupling, ref, work, nb)
    got = torch.full_like(ref, float("nan"))
    lib = V.lib()
    rc = lib.vlasov_field_noalloc(ctypes.byref(hg), ctypes.c_void_p(rho.data_ptr()),
                                  ctypes.c_double(coupling), ctypes.c_void_p(got.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, V.vlasov_strerror(rc)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_field_matches_the_workspace_form_on_two_calls():
    print("case: allocation-free field, 32x24x16 then 8x12x6", flush=True)
    ref1, got1 = _case((32, 24, 16), (1.0, 2.0, 0.5), 3.7, 1)
    assert torch.equal(got1, ref1)
    ref2, got2 = _case((8, 12, 6), (1.5, 1.0, 1.0), -1.25, 2)
    assert torch.equal(got2, ref2)


def test_noalloc_field_refuses_meshes_beyond_its_array():
    lib = V.lib()
    assert V.vlasov_field_noalloc_max_bytes() == 24 << 20
    hg = V.make_grid((128, 64, 64), (4, 4, 4))
    assert V.vlasov_field_workspace_bytes(hg) > V.vlasov_field_noalloc_max_bytes()
    rho = torch.ones((128, 64, 64), dtype=torch.float64, device="cuda")
    out = torch.empty((3, 128, 64, 64), dtype=torch.float32, device="cuda")
    rc = lib.vlasov_field_noalloc(ctypes.byref(hg), ctypes.c_void_p(rho.data_ptr()),
                                  ctypes.c_double(1.0), ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -8
    assert lib.vlasov_field_noalloc(None, None, ctypes.c_double(1.0), None, None) == -1
