"""The fused velocity kick against the three single velocity sweeps.

vlasov_kick sweeps ux, uy, uz inside LDS for 16^3 and 32^3 velocity blocks.
With FP32 storage its result must be exactly that of vlasov_advect_ux, _uy,
_uz in sequence (and always for shapes that do not fit, which run the three
sweeps themselves).  With FP16/BF16 storage the fused kick keeps the values
between its sweeps in FP32 and rounds only the result: it must agree with
the three sweeps within their two intermediate roundings, and be at least as
close to the FP64 oracle's three sweeps.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402
import oracle  # noqa: E402


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
    fused = nu[0] in (16, 32)
    if prec == V.F32 or not fused:
        assert torch.equal(k.f, c.f)
        if prec != V.F32:
            assert torch.equal(k.scale, c.scale)
        # per-line partial sums are FP32 and grouped differently (4 lines per thread vs 1)
        np.testing.assert_allclose(o2.cpu().numpy(), o1.cpu().numpy(), rtol=1e-6, atol=0)
        return
    # Scaled storage, fused: the two paths differ by the three sweeps' two
    # intermediate roundings (half a code unit of a line scale each), carried
    # through the later sweeps.  A sweep of these rough random lines enlarges
    # a perturbation of its input by up to A ~ 10-20 (measured on the FP64
    # oracle), so the first rounding can grow to A^2/2 units and the second
    # to A/2: the bound takes 64 units.  A wrong line, shift or scale would
    # differ by O(1), and the oracle comparison below is the sharper check.
    unit = {V.F16: 2.0 ** -11, V.BF16: 2.0 ** -8}[prec]
    dk = V.decode(k).double().cpu().numpy()
    dc = V.decode(c).double().cpu().numpy()
    top = np.abs(dc).max()
    assert np.abs(dk - dc).max() <= 64 * unit * top
    o1n, o2n = o1.cpu().numpy(), o2.cpu().numpy()
    np.testing.assert_allclose(o2n, o1n, rtol=0, atol=64 * unit * max(np.abs(o1n).max(), 1e-30))
    # and against the FP64 oracle's three sweeps of the same (decoded) input
    og = oracle.Grid.make(n, nu, (1.0, 1.0, 1.0), (1.0, 0.9, 1.1))
    ref = V.decode(st).double().cpu().numpy()
    fld = field.reshape((3,) + tuple(n))
    for ax in range(3):
        ref = oracle.advect_velocity(og, ax, ref, fld, dt, vbc=vbc)
    err_k = np.linalg.norm(dk - ref)
    err_c = np.linalg.norm(dc - ref)
    print(f"L2 error vs oracle: fused {err_k:.3e}, three sweeps {err_c:.3e}")
    assert err_k <= 1.05 * err_c


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


@pytest.mark.parametrize("prec", [V.F32, V.BF16])
@pytest.mark.parametrize("vbc", [V.VBC_OUTFLOW, V.VBC_PERIODIC])
def test_kick_without_workspace(prec, vbc):
    """Fused shapes run without a workspace (each work-group then splits its own
    shifts); with one they precompute the shift table first.  Same bits."""
    print("case: kick without workspace", V.PREC_NAME[prec], vbc, flush=True)
    n, nu = (4, 3, 5), (32, 32, 32)
    hg = V.make_grid(n, nu, (1.0, 1.0, 1.0), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(12)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    st = V.encode(hg, prec, f)
    g = torch.from_numpy(rng.uniform(-40, 40, (3,) + n).astype(np.float32)).cuda()
    dt = 0.05
    outs = []
    for use_work in (True, False):
        o = torch.zeros(n, dtype=torch.float64, device="cuda")
        k = V.empty_state(hg, prec, st.f.device)
        nbytes = V.vlasov_step_workspace_bytes(hg, prec)
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda") if use_work else None
        V.vlasov_kick(hg, prec, vbc, st.f, st.scale, k.f, k.scale, g, dt, work,
                      nbytes if use_work else 0, o)
        outs.append((k, o))
    torch.cuda.synchronize()
    (k1, o1), (k2, o2) = outs
    assert torch.equal(k1.f, k2.f)
    if prec != V.F32:
        assert torch.equal(k1.scale, k2.scale)
    assert torch.equal(o1, o2)
