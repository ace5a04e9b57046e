"""The fused velocity kick equals the three single velocity sweeps, bitwise.

vlasov_kick sweeps ux, uy, uz inside LDS for 16^3 and 32^3 velocity blocks;
its result must be exactly that of vlasov_advect_ux, _uy, _uz in sequence,
including the storage rounding between sweeps for FP16/BF16.  Shapes that do
not fit run the three sweeps themselves.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


@pytest.mark.parametrize("prec", [V.F32, V.F16, V.BF16])
@pytest.mark.parametrize("shape", [((3, 4, 5), (16, 16, 16)), ((2, 3, 3), (32, 32, 32)),
                                   ((2, 3, 2), (8, 8, 8))])
@pytest.mark.parametrize("vbc", [V.VBC_OUTFLOW, V.VBC_PERIODIC])
@pytest.mark.parametrize("cfl", [3.3, 45.0])
def test_kick_equals_three_sweeps(prec, shape, vbc, cfl):
    """cfl: largest |shift| in cells; 45 moves whole blocks out (vacuum) or wraps them."""
    n, nu = shape
    print("case: kick", V.PREC_NAME[prec], n, nu, vbc, cfl, flush=True)
    hg = V.make_grid(n, nu, (1.0, 1.0, 1.0), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(5)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    st = V.encode(hg, prec, f)
    cells = int(np.prod(n))
    dt = 0.1
    field = np.zeros((3, cells), np.float32)
    for a in range(3):
        du = 2 * hg.umax[a] / hg.nu[a]
        field[a] = (rng.uniform(-cfl, cfl, cells) * du / dt).astype(np.float32)
    g = torch.from_numpy(field.reshape((3,) + tuple(n))).cuda()
    o1 = torch.zeros(tuple(n), dtype=torch.float64, device="cuda")
    o2 = torch.zeros(tuple(n), dtype=torch.float64, device="cuda")
    a = V.advect("ux", st, dt, g=g, vbc=vbc, outflow=o1)
    b = V.advect("uy", a, dt, g=g, vbc=vbc, outflow=o1)
    c = V.advect("uz", b, dt, g=g, vbc=vbc, outflow=o1)
    k = V.kick(st, g, dt, vbc=vbc, outflow=o2)
    torch.cuda.synchronize()
    assert torch.equal(k.f, c.f)
    if prec != V.F32:
        assert torch.equal(k.scale, c.scale)
    # per-line partial sums are FP32 and grouped differently (4 lines per thread vs 1)
    np.testing.assert_allclose(o2.cpu().numpy(), o1.cpu().numpy(), rtol=1e-6, atol=0)


@pytest.mark.parametrize("prec", [V.F32, V.F16])
def test_step_equals_its_five_launches(prec):
    """vlasov_step is kick(g_n), z, y, x, kick(g_np1); bench.py times those five
    launches one by one, so both must give the same bits."""
    print("case: step vs five launches", V.PREC_NAME[prec], flush=True)
    n, nu = (6, 5, 4), (16, 16, 16)
    hg = V.make_grid(n, nu, (1.0, 1.3, 0.8), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(11)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    st = V.encode(hg, prec, f)
    dt = 0.21
    gs = [torch.from_numpy(rng.uniform(-3, 3, (3,) + n).astype(np.float32)).cuda() for _ in range(2)]
    o1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    o2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    ref = V.step(st, gs[0], gs[1], dt, outflow=o1)
    a = V.kick(st, gs[0], 0.5 * dt, outflow=o2)
    for ax in ("z", "y", "x"):
        a = V.advect(ax, a, dt)
    b = V.kick(a, gs[1], 0.5 * dt, outflow=o2)
    torch.cuda.synchronize()
    assert torch.equal(b.f, ref.f)
    if prec != V.F32:
        assert torch.equal(b.scale, ref.scale)
    assert torch.equal(o1, o2)
