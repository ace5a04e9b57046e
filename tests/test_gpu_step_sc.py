"""vlasov_step_sc: the self-consistent step (Eqs. 1, 2, 5).

Two steps of the tiny workload from the field of the initial density,
against the oracle's composition (oracle.step_sc: kick, drifts, density,
field, kick), FP32 at the sweeps' bar; the returned density and field
against the oracle's; argument errors.
"""
import numpy as np
import pytest

import oracle
from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


def test_selfconsistent_steps_against_oracle():
    w = inputs.workload(1)
    print("case: self-consistent steps", w.name, flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    f32 = inputs.initial_f32(w)
    f_ref = f32.astype(np.float64)
    rho0, _, _ = oracle.moments(og, f_ref)
    g1 = oracle.field_from_density(og, rho0, 1.0)
    du = min(2 * w.umax[a] / w.nu[a] for a in range(3))
    # coupling chosen so the half kick moves at most half a cell
    c = 0.5 * du / (0.5 * w.dt * np.abs(g1).max())
    g_ref = oracle.field_from_density(og, rho0, c).astype(np.float32)
    st = V.State(hg, V.F32, torch.from_numpy(f32).cuda())
    rho_d = torch.from_numpy(rho0).cuda()
    g_d = V.field(hg, rho_d, c)
    torch.cuda.synchronize()
    assert np.abs(g_d.cpu().numpy() - g_ref).max() <= 2e-7 * np.abs(g_ref).max()
    nb = V.vlasov_step_sc_workspace_bytes(hg, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for n in range(2):
        f_ref, g_ref, rho_ref = oracle.step_sc(og, f_ref, g_ref, c, w.dt)
        out = V.empty_state(hg, V.F32, "cuda")
        g_new = torch.empty_like(g_d)
        rho_new = torch.empty_like(rho_d)
        V.vlasov_step_sc(hg, V.F32, V.VBC_OUTFLOW, st.f, None, out.f, None, g_d, g_new, rho_new,
                         c, w.dt, 1.0, work, nb, None)
        torch.cuda.synchronize()
        got = out.f.cpu().numpy().astype(np.float64)
        assert np.abs(got - f_ref).max() <= 1e-5 * f_ref.max()
        np.testing.assert_allclose(rho_new.cpu().numpy(), rho_ref, rtol=1e-6, atol=0)
        gs = g_new.cpu().numpy()
        assert np.abs(gs - g_ref).max() <= 1e-5 * np.abs(g_ref).max()
        st, g_d = out, g_new


def test_selfconsistent_step_errors():
    hg = V.make_grid((4, 4, 4), (16, 16, 16))
    f = torch.rand(V.grid_shape(hg), device="cuda")
    out = torch.empty_like(f)
    g0 = torch.zeros((3, 4, 4, 4), dtype=torch.float32, device="cuda")
    g1 = torch.empty_like(g0)
    rho = torch.empty((4, 4, 4), dtype=torch.float64, device="cuda")
    nb = V.vlasov_step_sc_workspace_bytes(hg, V.F32)
    assert nb > V.vlasov_step_workspace_bytes(hg, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    args = [hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, g0, g1, rho, 1.0, 0.1, 1.0, work, nb]
    V.vlasov_step_sc(*args)
    torch.cuda.synchronize()
    for i, bad in ((8, g0), (9, None), (14, nb - 1)):          # aliasing, NULL, workspace
        a = list(args)
        a[i] = bad
        with pytest.raises(V.VlasovError):
            V.vlasov_step_sc(*a)
