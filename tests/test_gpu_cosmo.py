"""A comoving self-consistent run (Eqs. 1, 2 with a(t), Eq. 5): three steps
of the tiny workload from redshift 10 in a flat matter+Lambda background.
The device chain takes its drift factors and couplings from
vlasov_cosmo_steps and calls vlasov_step_sc; the oracle chain
(oracle.cosmology.run_sc) takes its own from the Friedmann quadrature.
FP32 at the sweeps' bar, density and field as in the single self-consistent
step.  And linear theory: a cold growing mode in Einstein-de Sitter grows as
the scale factor."""
import numpy as np
import pytest

import oracle
from oracle import cosmology as C
from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


def test_comoving_selfconsistent_run_against_oracle():
    w = inputs.workload(1)
    om, H0, nsteps = 0.3, 1.0, 3
    print("case: comoving run", w.name, flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    cos = V.vlasov_cosmology()
    cos.omega_m, cos.H0 = om, H0
    a0 = 1.0 / 11.0
    t0 = V.vlasov_cosmo_t(cos, a0)
    dt = w.dt * a0 * a0                  # the drift moves about as far as w.dt does at a = 1
    a, a2inv = V.vlasov_cosmo_steps(cos, t0, dt, nsteps)
    assert a[-1] > 1.05 * a[0]           # the background changes over the run
    f32 = inputs.initial_f32(w)
    rho0, _, _ = oracle.moments(og, f32.astype(np.float64))
    g1 = oracle.field_from_density(og, rho0, 1.0)
    du = min(2 * w.umax[k] / w.nu[k] for k in range(3))
    K = a0 * 0.5 * du / (0.5 * dt * np.abs(g1).max())   # half kicks within half a cell
    f_ref, g_ref, rho_ref, a_o, a2_o = C.run_sc(og, f32.astype(np.float64), K, om, H0, t0, dt,
                                                nsteps)
    np.testing.assert_allclose(a, a_o, rtol=1e-12)
    np.testing.assert_allclose(a2inv, a2_o, rtol=1e-12)

    st = V.State(hg, V.F32, torch.from_numpy(f32).cuda())
    rho = torch.from_numpy(rho0).cuda()
    g = V.field(hg, rho, K / a[0])
    nb = V.vlasov_step_sc_workspace_bytes(hg, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for n in range(nsteps):
        out = V.empty_state(hg, V.F32, "cuda")
        g_new, rho_new = torch.empty_like(g), torch.empty_like(rho)
        V.vlasov_step_sc(hg, V.F32, V.VBC_OUTFLOW, st.f, None, out.f, None, g, g_new, rho_new,
                         K / a[n + 1], dt, a2inv[n], work, nb, None)
        st, g, rho = out, g_new, rho_new
    torch.cuda.synchronize()
    got = st.f.cpu().numpy().astype(np.float64)
    assert np.abs(got - f_ref).max() <= nsteps * 1e-5 * f_ref.max()
    np.testing.assert_allclose(rho.cpu().numpy(), rho_ref, rtol=1e-6, atol=0)
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-5 * np.abs(g_ref).max()


def test_growing_mode_follows_the_scale_factor_on_the_device():
    """A cold density wave's growing mode in Einstein-de Sitter grows as
    a / a0 (tests/growth_setup.py): the device chain to 1 %, and its final
    mode amplitude against the oracle chain's."""
    import growth_setup as G

    print("case: comoving growing mode", G.N, G.NU, flush=True)
    hg = V.make_grid(G.N, G.NU, G.L, G.UMAX)
    og = oracle.Grid.make(G.N, G.NU, G.L, G.UMAX)
    cos = V.vlasov_cosmology()
    cos.omega_m, cos.H0 = G.OMEGA_M, G.H0
    t0 = V.vlasov_cosmo_t(cos, G.A0)
    dt = (V.vlasov_cosmo_t(cos, G.A1) - t0) / G.NSTEPS
    a, a2inv = V.vlasov_cosmo_steps(cos, t0, dt, G.NSTEPS)
    f0 = G.initial_f().astype(np.float32)
    st = V.State(hg, V.F32, torch.from_numpy(f0).cuda())
    rho, _, _ = V.moments(st)
    amp0 = G.mode_amplitude(rho.cpu().numpy())
    g = V.field(hg, rho, G.COUPLING_K / a[0])
    nb = V.vlasov_step_sc_workspace_bytes(hg, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for n in range(G.NSTEPS):
        out = V.empty_state(hg, V.F32, "cuda")
        g_new, rho_new = torch.empty_like(g), torch.empty_like(rho)
        V.vlasov_step_sc(hg, V.F32, V.VBC_OUTFLOW, st.f, None, out.f, None, g, g_new, rho_new,
                         G.COUPLING_K / a[n + 1], dt, a2inv[n], work, nb, None)
        st, g, rho = out, g_new, rho_new
    torch.cuda.synchronize()
    amp1 = G.mode_amplitude(rho.cpu().numpy())
    assert amp1 / amp0 == pytest.approx(G.A1 / G.A0, rel=1e-2)
    _, _, rho_o, _, _ = C.run_sc(og, f0.astype(np.float64), G.COUPLING_K, G.OMEGA_M, G.H0, t0,
                                 dt, G.NSTEPS)
    assert amp1 == pytest.approx(G.mode_amplitude(rho_o), rel=1e-3)
