"""Linear growth in an expanding background: the check of the comoving loop
(Eqs. 1, 2 with a(t), Eq. 5) shared by the oracle and device tests.

Einstein-de Sitter (Omega_m = 1, H0 = 1): a = (3t/2)^(2/3), and with the
neutrinos as all the matter and mean code density 1 the comoving coupling is
K / a with K = 3/2 H0^2.  A cold component (velocity dispersion well below
the Jeans scale) with a density wave delta = eps cos(k x) and the growing
mode's canonical velocity u = a^2 dx/dt = -eps a0^2 H(a0) sin(k x) / k
(continuity with delta proportional to a) grows as a / a0 in linear theory.
The input holds none of the method's arithmetic.
"""
import numpy as np

N = (32, 1, 1)
NU = (64, 2, 2)
L = (1.0, 1.0, 1.0)
UMAX = (0.02, 1.0, 1.0)
SIGMA = 0.002
EPS = 0.01
K = 2 * np.pi
OMEGA_M, H0, COUPLING_K = 1.0, 1.0, 1.5
A0, A1, NSTEPS = 0.1, 0.4, 100


def initial_f():
    du = [2 * UMAX[a] / NU[a] for a in range(3)]
    ux = -UMAX[0] + (np.arange(NU[0]) + 0.5) * du[0]
    x = (np.arange(N[0]) + 0.5) * L[0] / N[0]
    u0 = -EPS * A0 ** 2 * (H0 * A0 ** -1.5) * np.sin(K * x) / K
    dens = 1 + EPS * np.cos(K * x)
    f = np.zeros(N + NU)
    for i in range(N[0]):
        m = np.exp(-0.5 * ((ux - u0[i]) / SIGMA) ** 2)
        m /= m.sum() * du[0]
        f[i, 0, 0] = dens[i] * m[:, None, None] / (NU[1] * NU[2] * du[1] * du[2])
    return f


def mode_amplitude(rho) -> float:
    r = np.asarray(rho).reshape(N[0])
    return abs(np.fft.fft(r)[1]) / N[0]
