"""The oracle's self-consistent step (oracle.step_sc) against linear theory:
the kinetic Jeans growth rate of a Maxwellian (see tests/jeans_setup.py), at
two wavenumbers, to 1 %; the cold-fluid rate omega_J is far off, and a
repulsive coupling does not grow.  Above the Jeans wavenumber the mode decays
at the damped root of the same relation, to 2 %."""
import numpy as np
import pytest

import oracle
from jeans_setup import (DT, L, N, NU, UMAX, coupling, damping_rate, fitted_rate, growth_rate,
                         initial_f, mode_amplitude)


def _run(c, nsteps):
    g = oracle.Grid.make(N, NU, L, UMAX)
    f = initial_f()
    rho, _, _ = oracle.moments(g, f)
    assert rho.mean() == pytest.approx(1.0, rel=1e-12)
    gf = oracle.field_from_density(g, rho, c).astype(np.float32)
    ts, amps = [], []
    for s in range(nsteps):
        f, gf, rho = oracle.step_sc(g, f, gf, c, DT)
        ts.append((s + 1) * DT)
        amps.append(mode_amplitude(rho))
    return ts, amps


@pytest.mark.parametrize("ratio,nsteps", [(0.5, 100), (0.7, 160)])
def test_kinetic_jeans_growth(ratio, nsteps):
    c = coupling(ratio)
    gam = growth_rate(ratio)
    ts, amps = _run(c, nsteps)
    got = fitted_rate(ts, amps, t_lo=0.6 * ts[-1])
    assert got == pytest.approx(gam, rel=1e-2)
    assert abs(got - np.sqrt(c)) > 0.2 * np.sqrt(c)        # not the cold-fluid rate


def test_repulsive_coupling_does_not_grow():
    ts, amps = _run(-coupling(0.5), 100)
    assert max(amps) < 1.5 * amps[0]


def test_damping_above_the_jeans_wavenumber():
    ratio = 1.5
    ts, amps = _run(coupling(ratio), 120)
    got = fitted_rate(ts, amps, t_lo=0.5 * ts[-1])
    assert -got == pytest.approx(damping_rate(ratio), rel=2e-2)
