"""Position sweeps whose waves hold lines with different integer shifts.

In the y sweep a wave spans eight u_y values of one sign; where their
integer parts differ, the wave cannot share row addresses and each lane
walks its own rows.  Transposing x with y (space and velocity) turns such a
y sweep into an x sweep, whose waves hold one u_x each and share their rows:
with FP32 storage the per-line arithmetic is the same, so the two must agree
to the bit.  Shifts up to 1.4 and 2.6 cells (and -1.4) give waves with two
and with several integer parts.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


@pytest.mark.parametrize("smax", [1.4, 2.6, -1.4])
@pytest.mark.parametrize("ny", [16, 32, 64])
def test_y_sweep_with_two_integer_parts_equals_transposed_x(smax, ny):
    n, nu = (3, ny, 2), (8, 16, 32)
    L, U = (1.0, 2.0, 1.0), (1.0, 0.8, 1.0)
    print("case: lag", ny, smax, flush=True)
    hg = V.make_grid(n, nu, L, U)
    ht = V.make_grid((n[1], n[0], n[2]), (nu[1], nu[0], nu[2]), (L[1], L[0], L[2]),
                     (U[1], U[0], U[2]))
    dy = L[1] / n[1]
    umax_c = U[1] * (1 - 1 / nu[1])                 # largest |u_y| at a cell centre
    dt = smax * dy / umax_c
    rng = np.random.default_rng(81)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    ft = f.permute(1, 0, 2, 4, 3, 5).contiguous()
    a = V.advect("y", V.State(hg, V.F32, f), dt)
    b = V.advect("x", V.State(ht, V.F32, ft), dt)
    torch.cuda.synchronize()
    assert torch.equal(a.f, b.f.permute(1, 0, 2, 4, 3, 5))
