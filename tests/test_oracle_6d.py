"""Pins of the FP64 oracle's 6D operators, Strang step and moments.

* axis sweeps against numpy's own axis bookkeeping (an independent indexing);
* the Eq. (5) step against an explicitly built permutation when every shift
  is an integer (the composition order, the half kicks, the field time levels
  and a^-2 all change that permutation);
* conservation of mass with the velocity-boundary outflow tally;
* moments against closed forms (section 5.1.3).
"""
import numpy as np
import pytest

import oracle


def _grid(n, nu, L=(1, 1, 1), U=(1, 1, 1)):
    return oracle.Grid.make(n, nu, L, U)


def _line_sweep_along(f, axis, shift_of, periodic):
    """Apply the 1D oracle line sweep along ``axis`` of a 6D array; shift_of(index)
    gives the shift for the line whose full index tuple (axis entry 0) is given."""
    out = np.empty_like(f)
    moved = np.moveaxis(f, axis, -1)
    res = np.moveaxis(out, axis, -1)
    for idx in np.ndindex(moved.shape[:-1]):
        full = list(idx)
        full.insert(axis, 0)
        s = shift_of(tuple(full))
        res[idx], _ = oracle.sweep_line(moved[idx], s, periodic=periodic)
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_position_sweep_indexing(axis):
    g = _grid((5, 4, 3), (4, 3, 2), L=(1.0, 0.7, 1.3), U=(1.0, 0.8, 1.2))
    rng = np.random.default_rng(21 + axis)
    f = rng.uniform(0, 1, g.shape)
    dt = 0.37
    dx = g.L[axis] / g.n[axis]
    du = 2 * g.umax[axis] / g.nu[axis]

    def shift_of(idx):
        u = -g.umax[axis] + (idx[3 + axis] + 0.5) * du
        return u * (dt / dx)

    want = _line_sweep_along(f, axis, shift_of, periodic=True)
    got = oracle.advect_position(g, axis, f, dt)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_velocity_sweep_indexing_and_outflow(axis):
    g = _grid((3, 2, 4), (5, 4, 6), U=(1.0, 0.9, 1.1))
    rng = np.random.default_rng(31 + axis)
    f = rng.uniform(0, 1, g.shape)
    field = rng.uniform(-3, 3, (3,) + tuple(g.n)).astype(np.float32)
    dt = 0.21
    du = 2 * g.umax[axis] / g.nu[axis]

    def shift_of(idx):
        return float(field[axis][idx[:3]]) * (dt / du)

    want = _line_sweep_along(f, 3 + axis, shift_of, periodic=False)
    outflow = np.zeros(int(np.prod(g.n)))
    got = oracle.advect_velocity(g, axis, f, field, dt, vbc=0, outflow=outflow)
    np.testing.assert_array_equal(got, want)
    du3 = np.prod([2 * g.umax[a] / g.nu[a] for a in range(3)])
    lost = (f.sum(axis=(3, 4, 5)) - got.sum(axis=(3, 4, 5))).reshape(-1) * du3
    np.testing.assert_allclose(outflow, lost, rtol=1e-12, atol=1e-14)
    # periodic velocity boundary: nothing leaves
    per = oracle.advect_velocity(g, axis, f, field, dt, vbc=1)
    np.testing.assert_allclose(per.sum(), f.sum(), rtol=1e-14)


def _shift_fill(a, k, axis):
    """Translate by k cells along axis with zero fill (vacuum)."""
    out = np.zeros_like(a)
    n = a.shape[axis]
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if k >= 0:
        src[axis] = slice(0, max(n - k, 0))
        dst[axis] = slice(min(k, n), n)
    else:
        src[axis] = slice(min(-k, n), n)
        dst[axis] = slice(0, max(n + k, 0))
    out[tuple(dst)] = a[tuple(src)]
    return out


def _integer_step_grid():
    # dx/du = 1/2 on every axis; dt * a^-2 = 1 makes every drift an odd integer
    g = _grid((8, 8, 4), (8, 4, 4), L=(1.0, 2.0, 1.0), U=(1.0, 1.0, 1.0))
    return g


@pytest.mark.parametrize("vbc", [1, 0])
def test_step_is_the_eq5_permutation_at_integer_shifts(vbc):
    g = _integer_step_grid()
    rng = np.random.default_rng(41)
    f = rng.uniform(0, 1, g.shape)
    dt, a2inv = 2.0, 0.5                      # drift shift u_j * dt a^-2 / dx
    du = [2 * g.umax[a] / g.nu[a] for a in range(3)]
    kick_n, kick_np1 = (1, -2, 3), (-1, 1, 2)    # cells per half kick
    # field such that g * (dt/2) / du is the wanted integer
    gn = np.stack([np.full(tuple(g.n), k * du[a] / (0.5 * dt), np.float32)
                   for a, k in enumerate(kick_n)])
    gnp1 = np.stack([np.full(tuple(g.n), k * du[a] / (0.5 * dt), np.float32)
                     for a, k in enumerate(kick_np1)])

    def kick(a, ks):
        for ax in range(3):
            if vbc == 1:
                a = np.roll(a, ks[ax], axis=3 + ax)
            else:
                a = _shift_fill(a, ks[ax], 3 + ax)
        return a

    want = kick(f, kick_n)
    for ax in (2, 1, 0):                      # drift z, y, x
        dx = g.L[ax] / g.n[ax]
        moved = np.empty_like(want)
        for j in range(g.nu[ax]):
            u = -g.umax[ax] + (j + 0.5) * du[ax]
            s = int(round(u * dt * a2inv / dx))
            sl = [slice(None)] * 6
            sl[3 + ax] = slice(j, j + 1)
            moved[tuple(sl)] = np.roll(want[tuple(sl)], s, axis=ax)
        want = moved
    want = kick(want, kick_np1)
    outflow = np.zeros(int(np.prod(g.n)))
    got = oracle.step(g, f, gn, gnp1, dt, a2inv=a2inv, vbc=vbc, outflow=outflow)
    np.testing.assert_array_equal(got, want)
    if vbc == 0:
        du3 = np.prod(du)
        assert outflow.sum() == pytest.approx((f.sum() - got.sum()) * du3, rel=1e-13)


def test_step_mass_plus_outflow_is_conserved():
    from paper_2110_15867_amd import inputs

    w = inputs.scaled(inputs.workload(2), (6, 6, 6), (8, 8, 8))
    g = _grid(w.n, w.nu, w.L, w.umax)
    f = inputs.initial_f(w)
    pot = inputs.potential(w, cfl_v=3.5)      # strong field: real outflow
    _, _, m0 = oracle.moments(g, f)
    outflow = np.zeros(int(np.prod(g.n)))
    dx3 = np.prod([g.L[a] / g.n[a] for a in range(3)])
    for n in range(3):
        gn = inputs.accel_field(w, pot, n * w.dt)
        gnp1 = inputs.accel_field(w, pot, (n + 1) * w.dt)
        f = oracle.step(g, f, gn, gnp1, w.dt, outflow=outflow)
        assert f.min() >= 0.0
    _, _, m = oracle.moments(g, f)
    lost = outflow.sum() * dx3
    assert lost > 1e-4 * m0
    assert m + lost == pytest.approx(m0, rel=1e-13)


def test_moments_closed_forms():
    g = _grid((3, 4, 2), (6, 5, 4), L=(1.0, 2.0, 3.0), U=(1.5, 1.0, 0.5))
    rng = np.random.default_rng(51)
    delta = rng.uniform(-0.3, 0.3, tuple(g.n))
    du = [2 * g.umax[a] / g.nu[a] for a in range(3)]
    u = [-g.umax[a] + (np.arange(g.nu[a]) + 0.5) * du[a] for a in range(3)]
    UX = u[0][:, None, None] * np.ones(tuple(g.nu))
    f = (1 + delta)[..., None, None, None] * (1.0 + UX)[None, None, None]
    rho, um, mass = oracle.moments(g, f)
    vol_u = np.prod([2 * g.umax[a] for a in range(3)])
    np.testing.assert_allclose(rho, (1 + delta) * vol_u, rtol=1e-13)
    # mean of u^2 over cell midpoints of [-U, U): U^2/3 - du^2/12
    want_ux = g.umax[0] ** 2 / 3 - du[0] ** 2 / 12
    np.testing.assert_allclose(um[0], want_ux, rtol=1e-12)
    np.testing.assert_allclose(um[1], 0.0, atol=1e-14)
    np.testing.assert_allclose(um[2], 0.0, atol=1e-14)
    dx3 = np.prod([g.L[a] / g.n[a] for a in range(3)])
    assert mass == pytest.approx(vol_u * (1 + delta).sum() * dx3, rel=1e-13)
    # empty cells have zero mean velocity
    rho0, um0, _ = oracle.moments(g, np.zeros(g.shape))
    assert np.all(rho0 == 0) and np.all(um0 == 0)


def test_free_streaming_converges_in_6d():
    """g = 0: f(x, u, t) = f0(x - u t, u); the split step error shrinks with dx."""
    errs = []
    for n in (8, 16, 32):
        g = _grid((n, 4, 4), (4, 2, 2))
        x = (np.arange(n) + 0.5) / n
        du = 2.0 / 4
        u = -1 + (np.arange(4) + 0.5) * du
        t = 0.3

        def exact(time):
            # cell averages of 1 + 0.5 sin(2 pi (x - u t)) along x
            edges = np.arange(n + 1) / n
            out = np.empty((n, 4))
            for j in range(4):
                e = edges - u[j] * time
                prim = e - 0.5 / (2 * np.pi) * np.cos(2 * np.pi * e)
                out[:, j] = (prim[1:] - prim[:-1]) * n
            return out

        f = np.zeros(g.shape)
        f[:] = exact(0.0)[:, None, None, :, None, None]
        zero = np.zeros((3,) + tuple(g.n), np.float32)
        steps = 4
        for _ in range(steps):
            f = oracle.step(g, f, zero, zero, t / steps)
        errs.append(np.abs(f[:, 0, 0, :, 0, 0] - exact(t)).mean())
    assert errs[0] > errs[1] > errs[2]
    assert np.log2(errs[1] / errs[2]) > 4.0
