"""The device's self-consistent loop (vlasov_field, then vlasov_step_sc per
step) against linear theory and the oracle: the kinetic Jeans growth rate of
a Maxwellian (see tests/jeans_setup.py) to 1 %, the damped mode above the
Jeans wavenumber to 2 %, and the mode amplitude of every step against the
oracle chain's."""
import numpy as np
import pytest

import oracle
from jeans_setup import (DT, L, N, NU, UMAX, coupling, damping_rate, fitted_rate, growth_rate,
                         initial_f, mode_amplitude)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


def _device_run(c, nsteps):
    hg = V.make_grid(N, NU, L, UMAX)
    st = V.State(hg, V.F32, torch.from_numpy(initial_f().astype(np.float32)).cuda())
    rho, _, _ = V.moments(st)
    g = V.field(hg, rho, c)
    nb = V.vlasov_step_sc_workspace_bytes(hg, V.F32)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ts, amps = [], []
    for s in range(nsteps):
        out = V.empty_state(hg, V.F32, "cuda")
        g_new, rho_new = torch.empty_like(g), torch.empty_like(rho)
        V.vlasov_step_sc(hg, V.F32, V.VBC_OUTFLOW, st.f, None, out.f, None, g, g_new, rho_new, c,
                         DT, 1.0, work, nb, None)
        st, g, rho = out, g_new, rho_new
        ts.append((s + 1) * DT)
        amps.append(mode_amplitude(rho.cpu().numpy()))
    torch.cuda.synchronize()
    return ts, amps


def _oracle_run(c, nsteps):
    og = oracle.Grid.make(N, NU, L, UMAX)
    fo = initial_f().astype(np.float32).astype(np.float64)
    r, _, _ = oracle.moments(og, fo)
    gf = oracle.field_from_density(og, r, c).astype(np.float32)
    ref = []
    for s in range(nsteps):
        fo, gf, r = oracle.step_sc(og, fo, gf, c, DT)
        ref.append(mode_amplitude(r))
    return ref


def test_kinetic_jeans_growth_on_the_device():
    ratio, nsteps = 0.5, 100
    print("case: Jeans growth", N, NU, flush=True)
    c = coupling(ratio)
    ts, amps = _device_run(c, nsteps)
    got = fitted_rate(ts, amps, t_lo=0.6 * ts[-1])
    assert got == pytest.approx(growth_rate(ratio), rel=1e-2)
    np.testing.assert_allclose(amps, _oracle_run(c, nsteps), rtol=1e-3)


def test_damping_above_the_jeans_wavenumber_on_the_device():
    ratio, nsteps = 1.5, 120
    print("case: Jeans damping", N, NU, flush=True)
    c = coupling(ratio)
    ts, amps = _device_run(c, nsteps)
    got = fitted_rate(ts, amps, t_lo=0.5 * ts[-1])
    assert -got == pytest.approx(damping_rate(ratio), rel=2e-2)
    np.testing.assert_allclose(amps, _oracle_run(c, nsteps), rtol=1e-3)
