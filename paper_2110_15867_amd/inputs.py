"""Seeded synthetic inputs for the 6D Vlasov sweeps.

This module serves both the HIP path and the FP64 oracle, so it holds none of
the method's arithmetic: it only builds grids, initial distribution functions
and acceleration fields.  The paper's cosmological initial conditions
(N-body CDM, Planck cosmology) are replaced by the recipe below; the grid
shapes follow the paper's N_u and the workload sizes.

Recipe:
  * periodic box [0, L_l) per spatial axis, velocity range [-U, U) with U = 1;
  * f0(x, u) = F(|u|) (1 + delta(x)) at cell centres, F(w) = 1/(exp(w/0.2)+1)
    (an isotropic Fermi-Dirac-like profile);
  * delta = A S / max_grid |S|, S(x) = sum_m cos(2 pi k_m . x / L + theta_m),
    k_m drawn from {-K..K}^3 without 0, theta_m ~ U[0, 2 pi);
  * potential phi(x, t) = sum_m B_m cos(2 pi k'_m . x / L + psi_m + omega_m t)
    with k' in {-2..2}^3 without 0; the field handed to the velocity sweeps
    is g = -grad phi evaluated analytically at cell centres;
  * B_m = beta b_m, b_m ~ U[0.5, 1], beta set so that the velocity half-kick
    shift can never exceed 0.9 cells on any axis;
  * dt = C dx / (U - du/2): C is the largest position shift in cells.
Seeds: initial condition 1000+k, potential 2000+k, target perturbation
3000+k, finite-difference directions 4000+k for workload k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    n: tuple
    nu: tuple
    L: tuple = (1.0, 1.0, 1.0)
    umax: tuple = (1.0, 1.0, 1.0)
    cfl: float = 2.5           # largest position shift (cells) along the axis with the smallest dx
    n_modes: int = 8           # Fourier modes of delta
    kmax: int = 2
    amp: float = 0.05
    drift: bool = False        # potential phase drifts linearly in time
    steps: int = 2
    seed_index: int = 1

    @property
    def shape(self):
        return tuple(self.n) + tuple(self.nu)

    @property
    def cells(self) -> int:
        return int(np.prod(self.n)) * int(np.prod(self.nu))

    def dx(self, a):
        return self.L[a] / self.n[a]

    def du(self, a):
        return 2.0 * self.umax[a] / self.nu[a]

    @property
    def dt(self) -> float:
        # largest |u_j| is U - du/2; the axis with the smallest dx sets the CFL
        a = int(np.argmin([self.dx(k) for k in range(3)]))
        return self.cfl * self.dx(a) / (self.umax[a] - 0.5 * self.du(a))


def workload(k: int) -> Workload:
    """The five workloads: tiny, 32^3x32^3, throughput, precision, adjoint."""
    if k == 1:
        return Workload("tiny 16^3x16^3", (16, 16, 16), (16, 16, 16), cfl=2.5, n_modes=8,
                        kmax=2, amp=0.05, drift=False, steps=2, seed_index=1)
    if k == 2:
        return Workload("32^3x32^3", (32, 32, 32), (32, 32, 32), cfl=2.5, n_modes=32, kmax=3,
                        amp=0.1, drift=True, steps=10, seed_index=2)
    if k == 3:
        return Workload("throughput 64^3x32^3", (64, 64, 64), (32, 32, 32), L=(1.0, 2.0, 10.0),
                        cfl=3.0, n_modes=32, kmax=3, amp=0.1, drift=True, steps=5, seed_index=3)
    if k == 4:
        return Workload("precision 64^3x32^3", (64, 64, 64), (32, 32, 32), L=(1.0, 2.0, 10.0),
                        cfl=3.0, n_modes=32, kmax=3, amp=0.1, drift=True, steps=10, seed_index=4)
    if k == 5:
        return Workload("adjoint 32^3x16^3", (32, 32, 32), (16, 16, 16), cfl=2.5, n_modes=8,
                        kmax=2, amp=0.05, drift=True, steps=8, seed_index=5)
    raise ValueError(f"no workload {k}")


def scaled(w: Workload, n, nu, name=None) -> Workload:
    """Same recipe and seeds on another grid (e.g. a small sub-run)."""
    return dataclasses.replace(w, n=tuple(n), nu=tuple(nu), name=name or f"{w.name} @ {n}x{nu}")


# --- grids ----------------------------------------------------------------------

def cell_centres_x(w: Workload, a: int) -> np.ndarray:
    return (np.arange(w.n[a]) + 0.5) * w.dx(a)


def cell_centres_u(w: Workload, a: int) -> np.ndarray:
    return -w.umax[a] + (np.arange(w.nu[a]) + 0.5) * w.du(a)


def _random_wavevectors(rng, count, kmax):
    out = []
    while len(out) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            out.append(k)
    return np.array(out, dtype=np.int64)


# --- initial condition ------------------------------------------------------------

def density_contrast(w: Workload, seed: int | None = None) -> np.ndarray:
    """delta(x) on the spatial grid (float64 [nx, ny, nz]), max |delta| = amp."""
    rng = np.random.default_rng(1000 + w.seed_index if seed is None else seed)
    ks = _random_wavevectors(rng, w.n_modes, w.kmax)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=w.n_modes)
    x = [cell_centres_x(w, a) / w.L[a] for a in range(3)]
    X, Y, Z = np.meshgrid(x[0], x[1], x[2], indexing="ij")
    S = np.zeros(X.shape)
    for m in range(w.n_modes):
        S += np.cos(2.0 * math.pi * (ks[m, 0] * X + ks[m, 1] * Y + ks[m, 2] * Z) + theta[m])
    return w.amp * S / np.max(np.abs(S))


def velocity_profile(w: Workload, width: float = 0.2) -> np.ndarray:
    """F(|u|) = 1/(exp(|u|/width)+1) on the velocity grid (float64 [nux, nuy, nuz])."""
    u = [cell_centres_u(w, a) for a in range(3)]
    UX, UY, UZ = np.meshgrid(u[0], u[1], u[2], indexing="ij")
    speed = np.sqrt(UX * UX + UY * UY + UZ * UZ)
    return 1.0 / (np.exp(speed / width) + 1.0)


def initial_f(w: Workload, delta=None, profile=None) -> np.ndarray:
    """f0 = F(|u|)(1 + delta(x)) as float64 of shape (nx,ny,nz,nux,nuy,nuz)."""
    delta = density_contrast(w) if delta is None else delta
    profile = velocity_profile(w) if profile is None else profile
    return (1.0 + delta)[:, :, :, None, None, None] * profile[None, None, None, :, :, :]


def initial_f32(w: Workload) -> np.ndarray:
    """The float32 initial condition both paths start from (small grids)."""
    return initial_f(w).astype(np.float32)


def initial_f32_device(w: Workload, device="cuda"):
    """float32 f0 formed on the device from the small factor arrays (large grids)."""
    import torch

    d = torch.from_numpy((1.0 + density_contrast(w)).astype(np.float32)).to(device)
    p = torch.from_numpy(velocity_profile(w).astype(np.float32)).to(device)
    return (d.reshape(-1, 1) * p.reshape(1, -1)).reshape(w.shape).contiguous()


# --- acceleration field ---------------------------------------------------------------

@dataclasses.dataclass
class Potential:
    k: np.ndarray        # [modes, 3] integer wave-vectors
    psi: np.ndarray      # [modes] phases
    omega: np.ndarray    # [modes] phase drift rates
    B: np.ndarray        # [modes] amplitudes


def potential(w: Workload, seed: int | None = None, n_modes: int = 4, cfl_v: float = 0.9,
              perturb: float = 0.0, perturb_seed: int | None = None) -> Potential:
    """Seeded smooth potential whose half-kick shift never exceeds cfl_v cells."""
    rng = np.random.default_rng(2000 + w.seed_index if seed is None else seed)
    ks = _random_wavevectors(rng, n_modes, 2)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    omega = rng.uniform(-math.pi, math.pi, size=n_modes) if w.drift else np.zeros(n_modes)
    b = rng.uniform(0.5, 1.0, size=n_modes)
    worst = 0.0
    for a in range(3):
        bound = np.sum(np.abs(b) * 2.0 * math.pi * np.abs(ks[:, a]) / w.L[a])
        worst = max(worst, bound * (0.5 * w.dt) / w.du(a))
    beta = cfl_v / worst
    B = beta * b
    if perturb:
        prng = np.random.default_rng(3000 + w.seed_index if perturb_seed is None else perturb_seed)
        B = B * (1.0 + perturb * prng.standard_normal(n_modes))
    return Potential(ks, psi, omega, B)


def field_basis(w: Workload, pot: Potential, t: float) -> np.ndarray:
    """d g / d B_m: float64 [modes, 3, nx, ny, nz] (g is linear in the amplitudes)."""
    x = [cell_centres_x(w, a) / w.L[a] for a in range(3)]
    X, Y, Z = np.meshgrid(x[0], x[1], x[2], indexing="ij")
    out = np.zeros((len(pot.B), 3) + X.shape)
    for m in range(len(pot.B)):
        phase = 2.0 * math.pi * (pot.k[m, 0] * X + pot.k[m, 1] * Y + pot.k[m, 2] * Z) \
            + pot.psi[m] + pot.omega[m] * t
        s = np.sin(phase)
        for a in range(3):
            # g_a = -d phi / d x_a = B_m (2 pi k_a / L_a) sin(phase)
            out[m, a] = (2.0 * math.pi * pot.k[m, a] / w.L[a]) * s
    return out


def accel_field(w: Workload, pot: Potential, t: float) -> np.ndarray:
    """g = -grad phi at time t, float32 [3, nx, ny, nz]."""
    basis = field_basis(w, pot, t)
    g = np.tensordot(pot.B, basis, axes=(0, 0))
    return np.ascontiguousarray(g.astype(np.float32))


def uniform_field(w: Workload, value) -> np.ndarray:
    """Spatially constant field, float32 [3, nx, ny, nz]."""
    g = np.zeros((3,) + tuple(w.n), dtype=np.float32)
    for a in range(3):
        g[a] = np.float32(value[a])
    return g


def random_line_data(rng, shape, lo=0.0, hi=1.0) -> np.ndarray:
    """Non-negative random data for invariant and parity tests."""
    return rng.uniform(lo, hi, size=shape)
