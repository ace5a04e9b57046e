"""FP64 oracle of the cosmological background -- TEST INFRASTRUCTURE.

Only the test-suite may import this module; the product path never does.

The Vlasov equation (Eq. 1) drifts comoving positions at u / a(t)^2 and the
Poisson equation (Eq. 2) carries 4 pi G a(t)^2 (rho - mean rho).  This module
takes a(t) from the Friedmann equation of a flat universe of matter and a
cosmological constant (radiation neglected),
    da/dt = a H(a),  H(a) = H0 sqrt(Om a^-3 + 1 - Om),
without using its closed-form solution: t(a) is the integral of
da / (a H(a)) from 0 (scipy quad), a(t) its root (brentq).  Over one step
from t0 to t1 the drift moves a comoving position by u times the integral of
dt / a^2, computed as the integral of da / (a^3 H(a)) over [a(t0), a(t1)];
the step's a2inv argument is that integral over dt.  For comoving f the
density rho = sum f du^3 keeps its mean, and Eq. 2 becomes
nabla^2 phi = (K / a) (rho - mean rho) with K = 4 pi G times the physical
density of one unit of rho at a = 1: the coupling at time t is K / a(t).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize

from . import field_from_density, moments, step_sc


def hubble(om: float, H0: float, a: float) -> float:
    return H0 * np.sqrt(om / a ** 3 + (1.0 - om))


def time_of_a(om: float, H0: float, a: float) -> float:
    v, _ = integrate.quad(lambda x: 1.0 / (x * hubble(om, H0, x)), 0.0, a, epsabs=0.0,
                          epsrel=2e-14, limit=200)
    return v


def a_of_t(om: float, H0: float, t: float) -> float:
    return optimize.brentq(lambda a: time_of_a(om, H0, a) - t, 1e-12, 1e4, xtol=1e-300,
                           rtol=1e-15, maxiter=500)


def drift_integral(om: float, H0: float, t0: float, t1: float) -> float:
    """Integral of dt / a^2 from t0 to t1."""
    a0, a1 = a_of_t(om, H0, t0), a_of_t(om, H0, t1)
    v, _ = integrate.quad(lambda a: 1.0 / (a ** 3 * hubble(om, H0, a)), a0, a1, epsabs=0.0,
                          epsrel=2e-14, limit=200)
    return v


def steps(om: float, H0: float, t0: float, dt: float, nsteps: int):
    """(a[k] = a(t0 + k dt) for k = 0..nsteps, a2inv[n] = drift integral of step n / dt)."""
    t = t0 + dt * np.arange(nsteps + 1)
    a = np.array([a_of_t(om, H0, x) for x in t])
    a2inv = np.array([drift_integral(om, H0, t[n], t[n + 1]) / dt for n in range(nsteps)])
    return a, a2inv


def run_sc(grid, f, K: float, om: float, H0: float, t0: float, dt: float, nsteps: int,
           vbc: int = 0, outflow=None):
    """nsteps self-consistent steps of the comoving system from t0: the field
    of f's density at t0 with coupling K / a(t0), then per step oracle.step_sc
    with the drift's a2inv and the coupling K / a(t_{n+1}) of its new field.
    Returns (f, g, rho, a, a2inv)."""
    a, a2inv = steps(om, H0, t0, dt, nsteps)
    rho, _, _ = moments(grid, f)
    g = field_from_density(grid, rho, K / a[0]).astype(np.float32)
    for n in range(nsteps):
        f, g, rho = step_sc(grid, f, g, K / a[n + 1], dt, float(a2inv[n]), vbc, outflow)
    return f, g, rho, a, a2inv
