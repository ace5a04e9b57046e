"""vlasov_step_moments: a full step that also returns rho and umean of f^{n+1}.

Where the last kick runs fused (cubic velocity blocks of 16 or 32) the
moments are summed while the kick stores each block; otherwise a moments pass
reads f_out.  Either way f_out, its scales and the outflow tally must be the
bits vlasov_step gives, and the moments must be those of f_out: equal to
vlasov_moments' to FP64 rounding (another summation order) and to the FP64
oracle's moments of the same (decoded) values.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

SHAPES = {
    "fused16": ((6, 5, 4), (16, 16, 16), (1.0, 1.3, 0.8), (1.0, 0.9, 1.1)),
    "fused32": ((3, 2, 4), (32, 32, 32), (1.0, 1.0, 2.0), (1.0, 1.2, 0.8)),
    "unfused": ((5, 4, 3), (8, 12, 16), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
}


@pytest.mark.parametrize("prec", [V.F32, V.F16, V.BF16])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_step_moments(prec, shape):
    n, nu, L, U = SHAPES[shape]
    print("case: step moments", V.PREC_NAME[prec], shape, flush=True)
    hg = V.make_grid(n, nu, L, U)
    og = oracle.Grid.make(n, nu, L, U)
    rng = np.random.default_rng(23)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    st = V.encode(hg, prec, f)
    dt = 0.17
    gs = [torch.from_numpy(rng.uniform(-3, 3, (3,) + n).astype(np.float32)).cuda()
          for _ in range(2)]
    o1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    o2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    ref = V.step(st, gs[0], gs[1], dt, outflow=o1)

    nbytes = V.vlasov_step_workspace_bytes(hg, prec)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = V.empty_state(hg, prec, "cuda")
    rho = torch.full(n, np.nan, dtype=torch.float64, device="cuda")
    um = torch.full((3,) + n, np.nan, dtype=torch.float64, device="cuda")
    V.vlasov_step_moments(hg, prec, V.VBC_OUTFLOW, st.f, st.scale, out.f, out.scale, gs[0],
                          gs[1], dt, 1.0, work, nbytes, o2, rho, um)
    torch.cuda.synchronize()
    assert torch.equal(out.f, ref.f)
    if prec != V.F32:
        assert torch.equal(out.scale, ref.scale)
    assert torch.equal(o1, o2)

    rho_k, um_k, _ = V.moments(out)
    torch.cuda.synchronize()
    np.testing.assert_allclose(rho.cpu().numpy(), rho_k.cpu().numpy(), rtol=1e-13, atol=0)
    np.testing.assert_allclose(um.cpu().numpy(), um_k.cpu().numpy(), rtol=1e-11, atol=1e-15)
    rho_o, um_o, _ = oracle.moments(og, V.decode(out).double().cpu().numpy())
    np.testing.assert_allclose(rho.cpu().numpy().reshape(-1), np.reshape(rho_o, -1), rtol=1e-12,
                               atol=0)
    np.testing.assert_allclose(um.cpu().numpy().reshape(-1), np.reshape(um_o, -1), rtol=1e-10,
                               atol=1e-14)


def test_step_moments_without_mean_and_errors():
    n, nu, L, U = SHAPES["fused16"]
    hg = V.make_grid(n, nu, L, U)
    rng = np.random.default_rng(24)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32)).cuda()
    g = torch.from_numpy(rng.uniform(-1, 1, (3,) + n).astype(np.float32)).cuda()
    nbytes = V.vlasov_step_workspace_bytes(hg, V.F32)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(f)
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    V.vlasov_step_moments(hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, g, g, 0.1, 1.0, work,
                          nbytes, None, rho, None)
    rho_k, _, _ = V.moments(V.State(hg, V.F32, out), with_mean=False)
    torch.cuda.synchronize()
    np.testing.assert_allclose(rho.cpu().numpy(), rho_k.cpu().numpy(), rtol=1e-13, atol=0)
    with pytest.raises(V.VlasovError) as e:
        V.vlasov_step_moments(hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, g, g, 0.1, 1.0, work,
                              nbytes, None, None, None)
    assert "NULL" in str(e.value) or e.value.code != 0
    um = torch.empty((3,) + n, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VlasovError):      # umean overlapping rho
        V.vlasov_step_moments(hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, g, g, 0.1, 1.0,
                              work, nbytes, None, um, um)
