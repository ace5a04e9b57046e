"""FP64 CPU oracle for the split SL-MPP5 Vlasov sweeps -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path (the HIP library and its Python
binding) never imports, loads or calls it.

This module is a ctypes shim over ``liboracle_vlasov.so`` (plain C, FP64,
OpenMP over lines).  Arrays are numpy float64 in the layout
``f[ix][iy][iz][jx][jy][jz]`` (jz fastest); fields are float32
``g[3][nx][ny][nz]``.  What each routine computes, and the passage of the
paper it follows, is documented in ``vlasov_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VLASOV_ORACLE_LIB selects another build of the same sources (the sanitizer
# build of the CPU test run)
_LIB_PATH = os.environ.get("VLASOV_ORACLE_LIB", os.path.join(_HERE, "liboracle_vlasov.so"))
_lib = None

c_double_p = ctypes.POINTER(ctypes.c_double)
c_float_p = ctypes.POINTER(ctypes.c_float)


class Grid(ctypes.Structure):
    """Own copy of the grid description (shares nothing with the library)."""

    _fields_ = [("n", ctypes.c_int * 3), ("nu", ctypes.c_int * 3),
                ("L", ctypes.c_double * 3), ("umax", ctypes.c_double * 3)]

    @classmethod
    def make(cls, n, nu, L=(1.0, 1.0, 1.0), umax=(1.0, 1.0, 1.0)):
        g = cls()
        for a in range(3):
            g.n[a] = int(n[a])
            g.nu[a] = int(nu[a])
            g.L[a] = float(L[a])
            g.umax[a] = float(umax[a])
        return g

    @property
    def shape(self):
        return tuple(self.n) + tuple(self.nu)

    def dx(self, a):
        return self.L[a] / self.n[a]

    def du(self, a):
        return 2.0 * self.umax[a] / self.nu[a]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401  (compile on first use)
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.vor_median3.restype = ctypes.c_double
        L.vor_median3.argtypes = [ctypes.c_double] * 3
        L.vor_minmod4.restype = ctypes.c_double
        L.vor_minmod4.argtypes = [ctypes.c_double] * 4
        L.vor_sl5_weights.restype = None
        L.vor_sl5_weights.argtypes = [ctypes.c_double, c_double_p]
        L.vor_mp5_limit.restype = ctypes.c_double
        L.vor_mp5_limit.argtypes = [ctypes.c_double] * 7
        L.vor_mp_alpha.restype = ctypes.c_double
        L.vor_mp_alpha.argtypes = [ctypes.c_double]
        L.vor_split_shift.restype = None
        L.vor_split_shift.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_long), c_double_p]
        L.vor_interface_flux.restype = ctypes.c_double
        L.vor_interface_flux.argtypes = [c_double_p, ctypes.c_long, ctypes.c_long, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int]
        L.vor_sweep_line_opt.restype = None
        L.vor_sweep_line_opt.argtypes = [c_double_p, c_double_p, ctypes.c_long, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, c_double_p]
        L.vor_position_shift.restype = ctypes.c_double
        L.vor_position_shift.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_long,
                                         ctypes.c_double]
        L.vor_velocity_shift.restype = ctypes.c_double
        L.vor_velocity_shift.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_float,
                                         ctypes.c_double]
        L.vor_advect_position.restype = ctypes.c_int
        L.vor_advect_position.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, c_double_p,
                                          c_double_p, ctypes.c_double]
        L.vor_advect_velocity.restype = ctypes.c_int
        L.vor_advect_velocity.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int,
                                          c_double_p, c_double_p, c_float_p, ctypes.c_double,
                                          c_double_p]
        L.vor_step.restype = ctypes.c_int
        L.vor_step.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, c_double_p, c_double_p,
                               c_double_p, c_float_p, c_float_p, ctypes.c_double,
                               ctypes.c_double, c_double_p]
        L.vor_moments.restype = ctypes.c_int
        L.vor_moments.argtypes = [ctypes.POINTER(Grid), c_double_p, c_double_p, c_double_p,
                                  c_double_p]
        L.vor_dispersion.restype = ctypes.c_int
        L.vor_dispersion.argtypes = [ctypes.POINTER(Grid), c_double_p, c_double_p]
        G = ctypes.POINTER(Grid)
        D, I, Lg = ctypes.c_double, ctypes.c_int, ctypes.c_long
        L.vor_sweep_line_jacobian.restype = None
        L.vor_sweep_line_jacobian.argtypes = [c_double_p, Lg, D, I, I, c_double_p, c_double_p]
        L.vor_sweep_line_margin.restype = None
        L.vor_sweep_line_margin.argtypes = [c_double_p, Lg, D, I, c_double_p]
        L.vor_advect_position_margin.restype = I
        L.vor_advect_position_margin.argtypes = [G, I, c_double_p, c_double_p, D]
        L.vor_advect_velocity_margin.restype = I
        L.vor_advect_velocity_margin.argtypes = [G, I, I, c_double_p, c_float_p, D, c_double_p]
        L.vor_advect_position_adj.restype = I
        L.vor_advect_position_adj.argtypes = [G, I, c_double_p, c_double_p, c_double_p, D]
        L.vor_advect_velocity_adj.restype = I
        L.vor_advect_velocity_adj.argtypes = [G, I, I, c_double_p, c_float_p, D, c_double_p,
                                              c_double_p, c_double_p]
        L.vor_advect_velocity_tan.restype = I
        L.vor_advect_velocity_tan.argtypes = [G, I, I, c_double_p, c_float_p, c_double_p, D,
                                              c_double_p, c_double_p]
        L.vor_advect_position_tan.restype = I
        L.vor_advect_position_tan.argtypes = [G, I, c_double_p, c_double_p, c_double_p, D]
        L.vor_step_adj.restype = I
        L.vor_step_adj.argtypes = [G, I, c_double_p, c_float_p, c_float_p, D, D, c_double_p,
                                   c_double_p, c_double_p, c_double_p]
        L.vor_moments_adj.restype = I
        L.vor_moments_adj.argtypes = [G, c_double_p, c_double_p, c_double_p, c_double_p]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(c_double_p) if a is not None else None


def _fp(a):
    return a.ctypes.data_as(c_float_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# --- scalar pieces -------------------------------------------------------------

def median3(x, y, z):
    return lib().vor_median3(x, y, z)


def minmod4(w, x, y, z):
    return lib().vor_minmod4(w, x, y, z)


def sl5_weights(mu: float) -> np.ndarray:
    w = np.zeros(5)
    lib().vor_sl5_weights(mu, _dp(w))
    return w


def mp5_limit(fhat, a, b, c, d, e, alpha) -> float:
    return lib().vor_mp5_limit(fhat, a, b, c, d, e, alpha)


def mp_alpha(mu: float) -> float:
    return lib().vor_mp_alpha(mu)


def split_shift(s: float):
    N = ctypes.c_long()
    nu = ctypes.c_double()
    lib().vor_split_shift(s, ctypes.byref(N), ctypes.byref(nu))
    return N.value, nu.value


def interface_flux(line, j, nu, periodic=True, limiter=True) -> float:
    line = _f64(line)
    return lib().vor_interface_flux(_dp(line), line.size, j, nu, int(periodic), int(limiter))


def sweep_line(line, s, periodic=True, limiter=True):
    """Advance one 1D line by the shift s (cells); returns (new_line, outflow)."""
    line = _f64(line)
    out = np.empty_like(line)
    ofl = ctypes.c_double(0.0)
    lib().vor_sweep_line_opt(_dp(line), _dp(out), line.size, float(s), int(periodic),
                             int(limiter), ctypes.byref(ofl))
    return out, ofl.value


# --- 6D operators -------------------------------------------------------------

def position_shift(grid: Grid, axis: int, j: int, dt_over_a2: float) -> float:
    return lib().vor_position_shift(ctypes.byref(grid), axis, j, dt_over_a2)


def velocity_shift(grid: Grid, axis: int, ga: float, dt: float) -> float:
    return lib().vor_velocity_shift(ctypes.byref(grid), axis, ga, dt)


def advect_position(grid: Grid, axis: int, f, dt_over_a2: float):
    f = _f64(f)
    out = np.empty_like(f)
    _check(lib().vor_advect_position(ctypes.byref(grid), axis, _dp(f), _dp(out), dt_over_a2),
           "advect_position")
    return out


def advect_velocity(grid: Grid, axis: int, f, g, dt: float, vbc: int = 0, outflow=None):
    """Velocity sweep; ``outflow`` (float64 [cells]) is accumulated in place."""
    f = _f64(f)
    g = np.ascontiguousarray(g, dtype=np.float32)
    out = np.empty_like(f)
    _check(lib().vor_advect_velocity(ctypes.byref(grid), axis, vbc, _dp(f), _dp(out), _fp(g),
                                     dt, _dp(outflow)), "advect_velocity")
    return out


def step(grid: Grid, f, g_n, g_np1, dt: float, a2inv: float = 1.0, vbc: int = 0, outflow=None):
    """One Strang-split step (Eq. 5); ``outflow`` is accumulated in place."""
    f = _f64(f)
    out = np.empty_like(f)
    work = np.empty_like(f)
    g_n = np.ascontiguousarray(g_n, dtype=np.float32)
    g_np1 = np.ascontiguousarray(g_np1, dtype=np.float32)
    _check(lib().vor_step(ctypes.byref(grid), vbc, _dp(f), _dp(out), _dp(work), _fp(g_n),
                          _fp(g_np1), dt, a2inv, _dp(outflow)), "step")
    return out


def kick(grid: Grid, f, g, dt: float, vbc: int = 0, outflow=None):
    """The velocity sweeps ux, uy, uz over dt with one field g [3][cells] (each
    of Eq. 5's half kicks, with dt the half step)."""
    for axis in range(3):
        f = advect_velocity(grid, axis, f, g, dt, vbc=vbc, outflow=outflow)
    return f


def steps_merged(grid: Grid, fields, f, dt: float, a2inv=None, vbc: int = 0, outflow=None):
    """len(fields) - 1 steps of Eq. (5) in which the two half kicks that meet
    between consecutive steps -- both with the field at that time -- run as one
    kick over dt:  K(dt/2; g_0), then per step k the drifts z, y, x over
    dt a2inv[k] and K(dt; g_{k+1}), the last kick K(dt/2; g_n).  (A reading of
    the scheme, not a formula of the paper: in exact arithmetic a kick is a
    translation along u with a fixed field, so the merged and the unmerged
    compositions agree; the discrete flux of one kick over dt is not that of
    two over dt/2.)"""
    n = len(fields) - 1
    f = kick(grid, f, fields[0], 0.5 * dt, vbc, outflow)
    for k in range(n):
        dta = dt * (1.0 if a2inv is None else a2inv[k])
        for axis in (2, 1, 0):
            f = advect_position(grid, axis, f, dta)
        f = kick(grid, f, fields[k + 1], dt if k + 1 < n else 0.5 * dt, vbc, outflow)
    return f


def field_from_density(grid: Grid, rho, coupling: float):
    """Eq. (2) on the periodic box, nabla^2 phi = coupling (rho - mean rho),
    solved in Fourier space (the convolution method of section 3, numpy's FFT
    as the transform): phi_k = -coupling rho_k / |k|^2 with phi_0 = 0, and
    g = -grad phi, g_a,k = -i k_a phi_k with k_a = 2 pi m_a / L_a (m_a the
    signed index) and k_a = 0 on the Nyquist plane of an even axis.
    Returns g [3][nx][ny][nz] in FP64."""
    rho = np.asarray(rho, dtype=np.float64).reshape(tuple(grid.n))
    R = np.fft.fftn(rho)
    ks = []
    for a in range(3):
        n = grid.n[a]
        m = np.fft.fftfreq(n, d=1.0 / n)                 # signed indices, Nyquist -n/2
        ks.append(2.0 * np.pi * m / grid.L[a])
    KX, KY, KZ = np.meshgrid(ks[0], ks[1], ks[2], indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    phi = np.zeros_like(R)
    nz = K2 != 0.0
    phi[nz] = -coupling * R[nz] / K2[nz]
    out = np.empty((3,) + tuple(grid.n))
    for a, K in enumerate((KX, KY, KZ)):
        Ka = K.copy()
        if grid.n[a] % 2 == 0:
            sl = [slice(None)] * 3
            sl[a] = grid.n[a] // 2
            Ka[tuple(sl)] = 0.0
        out[a] = np.real(np.fft.ifftn(-1j * Ka * phi))
    return out


def step_sc(grid: Grid, f, g_n, coupling: float, dt: float, a2inv: float = 1.0, vbc: int = 0,
            outflow=None):
    """One self-consistent step: kick(g_n) over dt/2, drifts z, y, x, the field
    of the drifted f's density (Eq. 2, field_from_density), kick over dt/2
    with it.  Returns (f^{n+1}, g^{n+1} rounded to FP32 as the sweeps read
    it, rho^{n+1})."""
    f = kick(grid, f, g_n, 0.5 * dt, vbc, outflow)
    for axis in (2, 1, 0):
        f = advect_position(grid, axis, f, dt * a2inv)
    rho, _, _ = moments(grid, f)
    g = field_from_density(grid, rho, coupling).astype(np.float32)
    f = kick(grid, f, g, 0.5 * dt, vbc, outflow)
    return f, g, rho


def moments(grid: Grid, f):
    """Returns (rho [cells], umean [3, cells], mass)."""
    f = _f64(f)
    nx = grid.n[0] * grid.n[1] * grid.n[2]
    rho = np.empty(nx)
    um = np.empty(3 * nx)
    mass = ctypes.c_double()
    _check(lib().vor_moments(ctypes.byref(grid), _dp(f), _dp(rho), _dp(um), ctypes.byref(mass)),
           "moments")
    return rho.reshape(tuple(grid.n)), um.reshape((3,) + tuple(grid.n)), mass.value


DISPERSION_COMPONENTS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def dispersion(grid: Grid, f):
    """Velocity dispersion tensor [6, cells] (xx, xy, xz, yy, yz, zz): the
    density-weighted covariance of u in each spatial cell (section 5.1.3)."""
    f = _f64(f)
    nx = grid.n[0] * grid.n[1] * grid.n[2]
    sig = np.empty(6 * nx)
    _check(lib().vor_dispersion(ctypes.byref(grid), _dp(f), _dp(sig)), "dispersion")
    return sig.reshape((6,) + tuple(grid.n))


# --- derivatives (frozen limiter selections) ----------------------------------------

def sweep_line_jacobian(line, s, periodic=True, limiter=True):
    """(J, dnu): d out / d f (M x M) and d out / d nu of one line sweep."""
    line = _f64(line)
    M = line.size
    J = np.zeros((M, M))
    dn = np.zeros(M)
    lib().vor_sweep_line_jacobian(_dp(line), M, float(s), int(periodic), int(limiter), _dp(J),
                                  _dp(dn))
    return J, dn


def sweep_line_margin(line, s, periodic=True):
    """Selection margin of every input cell of one line sweep (see vlasov_oracle_adj.c)."""
    line = _f64(line)
    out = np.empty_like(line)
    lib().vor_sweep_line_margin(_dp(line), line.size, float(s), int(periodic), _dp(out))
    return out


def advect_position_margin(grid, axis, f, dt_over_a2):
    """Per cell: the smallest selection margin of the interfaces that read it (position sweep)."""
    f = _f64(f)
    out = np.empty_like(f)
    _check(lib().vor_advect_position_margin(ctypes.byref(grid), axis, _dp(f), _dp(out),
                                            dt_over_a2), "advect_position_margin")
    return out


def advect_velocity_margin(grid, axis, f, g, dt, vbc=0):
    """Per cell: the smallest selection margin of the interfaces that read it (velocity sweep)."""
    f = _f64(f)
    g = np.ascontiguousarray(g, dtype=np.float32)
    out = np.empty_like(f)
    _check(lib().vor_advect_velocity_margin(ctypes.byref(grid), axis, vbc, _dp(f), _fp(g), dt,
                                            _dp(out)), "advect_velocity_margin")
    return out


def advect_position_adj(grid, axis, f, lam_out, dt_over_a2):
    f, lam_out = _f64(f), _f64(lam_out)
    out = np.empty_like(f)
    _check(lib().vor_advect_position_adj(ctypes.byref(grid), axis, _dp(f), _dp(lam_out),
                                         _dp(out), dt_over_a2), "advect_position_adj")
    return out


def advect_position_tan(grid, axis, f, v, dt_over_a2):
    f, v = _f64(f), _f64(v)
    out = np.empty_like(f)
    _check(lib().vor_advect_position_tan(ctypes.byref(grid), axis, _dp(f), _dp(v), _dp(out),
                                         dt_over_a2), "advect_position_tan")
    return out


def advect_velocity_adj(grid, axis, f, g, dt, lam_out, vbc=0, lam_g=None):
    """Returns lam_in; lam_g (float64 [3, cells]) is accumulated in place if given."""
    f, lam_out = _f64(f), _f64(lam_out)
    g = np.ascontiguousarray(g, dtype=np.float32)
    out = np.empty_like(f)
    _check(lib().vor_advect_velocity_adj(ctypes.byref(grid), axis, vbc, _dp(f), _fp(g), dt,
                                         _dp(lam_out), _dp(out), _dp(lam_g)),
           "advect_velocity_adj")
    return out


def advect_velocity_tan(grid, axis, f, g, dt, v, g_dot=None, vbc=0):
    f, v = _f64(f), _f64(v)
    g = np.ascontiguousarray(g, dtype=np.float32)
    gd = None if g_dot is None else _f64(g_dot)
    out = np.empty_like(f)
    _check(lib().vor_advect_velocity_tan(ctypes.byref(grid), axis, vbc, _dp(f), _fp(g), _dp(gd),
                                         dt, _dp(v), _dp(out)), "advect_velocity_tan")
    return out


def step_adj(grid, f, g_n, g_np1, dt, lam_out, a2inv=1.0, vbc=0, lam_g_n=None, lam_g_np1=None):
    """Adjoint of one Strang step; returns lam_in, accumulates lam_g_n / lam_g_np1."""
    f, lam_out = _f64(f), _f64(lam_out)
    cells = grid.n[0] * grid.n[1] * grid.n[2]
    if lam_g_n is None:
        lam_g_n = np.zeros(3 * cells)
    if lam_g_np1 is None:
        lam_g_np1 = np.zeros(3 * cells)
    out = np.empty_like(f)
    _check(lib().vor_step_adj(ctypes.byref(grid), vbc, _dp(f),
                              _fp(np.ascontiguousarray(g_n, np.float32)),
                              _fp(np.ascontiguousarray(g_np1, np.float32)), dt, a2inv,
                              _dp(lam_out), _dp(out), _dp(lam_g_n), _dp(lam_g_np1)), "step_adj")
    return out


def moments_adj(grid, f, lam_rho, lam_umean=None):
    f = _f64(f)
    out = np.zeros_like(f)
    _check(lib().vor_moments_adj(ctypes.byref(grid), _dp(f), _dp(_f64(lam_rho)),
                                 _dp(None if lam_umean is None else _f64(lam_umean)), _dp(out)),
           "moments_adj")
    return out
