"""Kinetic Jeans instability: the linear-theory check of the self-consistent
loop (Eqs. 1, 2, 5) shared by the oracle and device tests.

A Maxwellian of dispersion sigma in u_x with a small density wave
cos(k x) along x, uniform in y and z.  Linearising Eq. (1) about it with the
attractive coupling of Eq. (2) (nabla^2 phi = c (rho - mean rho), omega_J^2 =
c mean rho) gives the kinetic dispersion relation of self-gravitating
systems; for a growing mode exp(gamma t), with y = gamma / (sqrt(2) k sigma),
    (k sigma / omega_J)^2 = 1 - sqrt(pi) y erfcx(y),
(the plasma-dispersion function at an imaginary argument).  It tends to
gamma = omega_J for a cold system and to 0 at the Jeans wavenumber
k = omega_J / sigma.  Above it the mode is damped without oscillating,
exp(-delta t), the same relation continued to a negative imaginary
frequency: with y = delta / (sqrt(2) k sigma),
    (k sigma / omega_J)^2 = 1 + sqrt(pi) y erfcx(-y).
The input holds none of the method's arithmetic.
"""
import numpy as np
from scipy import optimize, special

N = (32, 1, 1)
NU = (64, 2, 2)
L = (1.0, 1.0, 1.0)
UMAX = (0.6, 1.0, 1.0)
SIGMA = 0.1
EPS = 1e-3
K = 2 * np.pi
DT = 0.05


def growth_rate(k_sigma_over_wj: float, k: float = K, sigma: float = SIGMA) -> float:
    r2 = k_sigma_over_wj ** 2
    y = optimize.brentq(lambda y: 1 - np.sqrt(np.pi) * y * special.erfcx(y) - r2, 1e-9, 1e3)
    return np.sqrt(2) * k * sigma * y


def damping_rate(k_sigma_over_wj: float, k: float = K, sigma: float = SIGMA) -> float:
    r2 = k_sigma_over_wj ** 2
    y = optimize.brentq(lambda y: 1 + np.sqrt(np.pi) * y * special.erfcx(-y) - r2, 1e-9, 10.0)
    return np.sqrt(2) * k * sigma * y


def coupling(k_sigma_over_wj: float) -> float:
    """c with omega_J = k sigma / ratio for mean density 1."""
    return (K * SIGMA / k_sigma_over_wj) ** 2


def initial_f():
    du = [2 * UMAX[a] / NU[a] for a in range(3)]
    ux = -UMAX[0] + (np.arange(NU[0]) + 0.5) * du[0]
    m = np.exp(-0.5 * (ux / SIGMA) ** 2)
    m /= m.sum() * du[0]
    x = (np.arange(N[0]) + 0.5) * L[0] / N[0]
    wave = 1 + EPS * np.cos(K * x)
    f = wave[:, None, None, None, None, None] * m[None, None, None, :, None, None]
    return f * np.ones((1, 1, 1, 1, NU[1], NU[2])) / (NU[1] * NU[2] * du[1] * du[2])


def mode_amplitude(rho) -> float:
    r = np.asarray(rho).reshape(N[0])
    return abs(np.fft.fft(r)[1]) / N[0]


def fitted_rate(times, amps, t_lo=3.0) -> float:
    t, a = np.asarray(times), np.asarray(amps)
    m = t >= t_lo
    return float(np.polyfit(t[m], np.log(a[m]), 1)[0])
