"""Pins of the oracle's cosmological background (Eqs. 1, 2 with a(t)):

* Einstein-de Sitter (Om = 1): a = (3 H0 t / 2)^(2/3) and the drift integral
  3 (3 H0 / 2)^(-4/3) (t0^(-1/3) - t1^(-1/3)) in closed form;
* the textbook ages H0 t(a=1) = 2/3 (Om = 1) and 0.9641 (Om = 0.3);
* a(t) satisfies the Friedmann equation (central differences);
* the drift integral is additive over split intervals and tends to
  dt / a^2 for a short step;
* the comoving self-consistent loop (run_sc) grows a cold density wave's
  growing mode as a / a0 in Einstein-de Sitter (see tests/growth_setup.py).
"""
import numpy as np
import pytest

from oracle import cosmology as C


@pytest.mark.parametrize("H0", [1.0, 0.37])
def test_einstein_de_sitter_closed_forms(H0):
    for t in (0.01, 0.3, 2.0):
        assert C.a_of_t(1.0, H0, t) == pytest.approx((1.5 * H0 * t) ** (2 / 3), rel=1e-12)
    t0, t1 = 0.05, 0.4
    want = 3 * (1.5 * H0) ** (-4 / 3) * (t0 ** (-1 / 3) - t1 ** (-1 / 3))
    assert C.drift_integral(1.0, H0, t0, t1) == pytest.approx(want, rel=1e-12)


def test_textbook_ages():
    assert C.time_of_a(1.0, 1.0, 1.0) == pytest.approx(2 / 3, rel=1e-13)
    assert C.time_of_a(0.3, 1.0, 1.0) == pytest.approx(0.9641, abs=1e-4)
    assert C.time_of_a(0.3, 2.0, 1.0) == pytest.approx(0.9641 / 2, abs=1e-4)


@pytest.mark.parametrize("om", [0.3, 0.7, 1.0])
def test_friedmann_equation(om):
    H0 = 1.3
    for t in (0.02, 0.2, 0.9):
        h = 1e-5 * t
        dadt = (C.a_of_t(om, H0, t + h) - C.a_of_t(om, H0, t - h)) / (2 * h)
        a = C.a_of_t(om, H0, t)
        assert dadt == pytest.approx(a * C.hubble(om, H0, a), rel=1e-7)


def test_drift_integral_additive_and_short_step():
    om, H0 = 0.31, 1.0
    t0, tm, t1 = 0.1, 0.17, 0.3
    whole = C.drift_integral(om, H0, t0, t1)
    parts = C.drift_integral(om, H0, t0, tm) + C.drift_integral(om, H0, tm, t1)
    assert whole == pytest.approx(parts, rel=1e-12)
    dt = 1e-6
    a = C.a_of_t(om, H0, 0.5 + 0.5 * dt)
    assert C.drift_integral(om, H0, 0.5, 0.5 + dt) / dt == pytest.approx(a ** -2, rel=1e-9)
    a, a2inv = C.steps(om, H0, 0.2, 0.05, 3)
    assert a.shape == (4,) and a2inv.shape == (3,)
    assert np.all(np.diff(a) > 0) and np.all(a2inv < a[:-1] ** -2) and np.all(a2inv > a[1:] ** -2)


def test_growing_mode_follows_the_scale_factor():
    import oracle
    import growth_setup as G

    g = oracle.Grid.make(G.N, G.NU, G.L, G.UMAX)
    f = G.initial_f()
    rho, _, _ = oracle.moments(g, f)
    assert rho.mean() == pytest.approx(1.0, rel=1e-12)
    t0 = C.time_of_a(G.OMEGA_M, G.H0, G.A0)
    dt = (C.time_of_a(G.OMEGA_M, G.H0, G.A1) - t0) / G.NSTEPS
    _, _, rho1, a, _ = C.run_sc(g, f, G.COUPLING_K, G.OMEGA_M, G.H0, t0, dt, G.NSTEPS)
    assert a[-1] == pytest.approx(G.A1, rel=1e-12)
    growth = G.mode_amplitude(rho1) / G.mode_amplitude(rho)
    assert growth == pytest.approx(G.A1 / G.A0, rel=1e-2)
