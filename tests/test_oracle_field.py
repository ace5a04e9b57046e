"""Pins of the oracle's field solve (oracle.field_from_density, Eq. 2).

* a single Fourier mode of the density against the closed form
  g = -c A k sin(k.x + theta) / |k|^2 (any box, any direction);
* the mean of the density has no field; the solve is linear;
* a Nyquist mode along an even axis has no derivative along that axis;
* the field of a density is minus the gradient of a potential whose
  finite-difference Laplacian reproduces the density (spectral accuracy on
  a smooth field).
"""
import numpy as np
import pytest

import oracle


def _centres(g):
    return np.meshgrid(*[(np.arange(g.n[a]) + 0.5) * g.L[a] / g.n[a] for a in range(3)],
                       indexing="ij")


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, -1), (3, 1, 2)])
def test_single_mode_closed_form(m):
    g = oracle.Grid.make((12, 10, 14), (4, 4, 4), (1.0, 2.0, 0.7), (1, 1, 1))
    X = _centres(g)
    k = [2 * np.pi * m[a] / g.L[a] for a in range(3)]
    th = 0.37
    phase = k[0] * X[0] + k[1] * X[1] + k[2] * X[2] + th
    A, c, rho0 = 0.3, 2.5, 1.7
    rho = rho0 + A * np.cos(phase)
    got = oracle.field_from_density(g, rho, c)
    k2 = sum(v * v for v in k)
    for a in range(3):
        want = -c * A * k[a] * np.sin(phase) / k2
        np.testing.assert_allclose(got[a], want, rtol=0, atol=1e-12)


def test_mean_has_no_field_and_linearity():
    g = oracle.Grid.make((8, 6, 10), (4, 4, 4), (1.0, 1.0, 1.0), (1, 1, 1))
    rng = np.random.default_rng(61)
    r1, r2 = rng.uniform(0, 1, (2,) + tuple(g.n))
    np.testing.assert_allclose(oracle.field_from_density(g, np.full(tuple(g.n), 3.0), 1.0), 0.0,
                               atol=1e-14)
    lhs = oracle.field_from_density(g, 2.0 * r1 + r2 + 5.0, 1.3)
    rhs = 2.0 * oracle.field_from_density(g, r1, 1.3) + oracle.field_from_density(g, r2, 1.3)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_nyquist_mode_has_no_derivative_along_its_axis():
    g = oracle.Grid.make((8, 6, 5), (4, 4, 4), (1.0, 1.0, 1.0), (1, 1, 1))
    i = np.arange(8)
    rho = np.broadcast_to(np.cos(np.pi * i)[:, None, None], tuple(g.n)).copy()   # (-1)^i
    got = oracle.field_from_density(g, rho, 1.0)
    np.testing.assert_allclose(got, 0.0, atol=1e-14)


def test_field_is_minus_gradient_of_a_potential_solving_poisson():
    n = (48, 40, 32)
    L = (1.0, 1.3, 0.8)
    g = oracle.Grid.make(n, (4, 4, 4), L, (1, 1, 1))
    X = _centres(g)
    # smooth periodic potential; rho = laplacian / c + const
    c = 0.9
    phi = (np.sin(2 * np.pi * X[0] / L[0]) * np.cos(4 * np.pi * X[1] / L[1])
           + 0.5 * np.cos(2 * np.pi * X[2] / L[2] + 0.3))
    lap = (-(2 * np.pi / L[0]) ** 2 - (4 * np.pi / L[1]) ** 2) * np.sin(2 * np.pi * X[0] / L[0]) \
        * np.cos(4 * np.pi * X[1] / L[1]) - 0.5 * (2 * np.pi / L[2]) ** 2 * np.cos(
            2 * np.pi * X[2] / L[2] + 0.3)
    rho = lap / c + 4.0
    got = oracle.field_from_density(g, rho, c)
    # periodic centred differences of the exact potential: second order
    grad = [(np.roll(phi, -1, axis=a) - np.roll(phi, 1, axis=a)) / (2 * L[a] / n[a])
            for a in range(3)]
    for a in range(3):
        err = np.abs(got[a] + grad[a]).max() / np.abs(grad[a]).max()
        assert err < 0.02, (a, err)


def test_selfconsistent_step_composition():
    """oracle.step_sc with no coupling is the Eq. (5) step with zero fields
    (bit for bit); with periodic velocity faces the kicks keep each cell's
    density, so the density it returns is that of f^{n+1}, and the field it
    returns is the field of that density."""
    from paper_2110_15867_amd import inputs

    w = inputs.scaled(inputs.workload(1), (6, 5, 4), (8, 8, 8))
    g = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    f = inputs.initial_f(w)
    zero = np.zeros((3,) + tuple(g.n), np.float32)
    f1, g1, _ = oracle.step_sc(g, f, zero, 0.0, w.dt)
    np.testing.assert_array_equal(f1, oracle.step(g, f, zero, zero, w.dt))
    assert not g1.any()
    rho0, _, _ = oracle.moments(g, f)
    g0 = oracle.field_from_density(g, rho0, 30.0).astype(np.float32)
    f2, g2, rho2 = oracle.step_sc(g, f, g0, 30.0, w.dt, vbc=1)
    np.testing.assert_allclose(oracle.moments(g, f2)[0], rho2, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(g2, oracle.field_from_density(g, rho2, 30.0).astype(np.float32))
    assert np.abs(g2).max() > 0.0
