"""GPU parity on data built to put the Suresh-Huynh bounds on their ties.

f is a sum of six integer profiles, one per phase-space axis, scaled by
2^-10, so every value, difference and curvature the walks form is exact in
FP32.  Each profile's curvatures D_j run through ratios 4:1 (4 Da - Db = 0:
the curvature minmod's zero by a tie), 3:1 (4 Da - Db = Da), equal
neighbours, sign changes and zeros, and make extrema everywhere, so the
early-out test fails often and the bounds decide.  On such data the
kernels' four-operation minmod equals the four-candidate definition bit for
bit; each sweep and the fused kick are held to the stated bar (L-infinity
within 1e-5 of max f) against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

LINF = 1e-5
N, NU = (8, 6, 8), (16, 16, 32)
PATTERN = np.array([1, 4, 16, 4, 1, 0, -1, -3, -9, -3, -1, 2, 8, 2, 2, 0, -5, -20, -5, 3], float)


def _tie_data(seed, n=N, nu=NU):
    rng = np.random.default_rng(seed)
    og = oracle.Grid.make(n, nu, (1.0, 1.2, 0.9), (1.0, 1.0, 1.0))
    hg = V.make_grid(n, nu, (1.0, 1.2, 0.9), (1.0, 1.0, 1.0))
    f = np.zeros(og.shape)
    for ax, m in enumerate(tuple(n) + tuple(nu)):
        D = np.resize(np.roll(PATTERN, int(rng.integers(len(PATTERN)))), m)
        p = np.cumsum(np.cumsum(D))
        shape = [1] * 6
        shape[ax] = m
        f = f + p.reshape(shape)
    f = (f - f.min()) * 2.0 ** -10
    f32 = f.astype(np.float32)
    assert np.array_equal(f32.astype(np.float64), f)       # exact in FP32
    return og, hg, f32


def _close(got, want, scale):
    err = float(np.max(np.abs(got.astype(np.float64) - want)))
    assert err <= LINF * scale, f"max err {err:.3e} > {LINF:.0e} * {scale:.3e}"


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("dt", [0.19, -0.21, 2.7])
def test_position_sweeps_on_ties(axis, dt):
    og, hg, f32 = _tie_data(axis)
    print("case: ties position", axis, dt, flush=True)
    want = oracle.advect_position(og, axis, f32.astype(np.float64), dt)
    fin = torch.from_numpy(f32).cuda()
    out = torch.empty_like(fin)
    [V.vlasov_advect_x, V.vlasov_advect_y, V.vlasov_advect_z][axis](hg, V.F32, fin, None, out,
                                                                    None, dt)
    torch.cuda.synchronize()
    _close(out.cpu().numpy(), want, float(f32.max()))


def _field(og, axis_shifts, dt, rng):
    cells = int(np.prod(og.n))
    g = np.zeros((3, cells), np.float32)
    for ax in axis_shifts:
        du = 2 * og.umax[ax] / og.nu[ax]
        s = rng.uniform(-3.4, 3.4, cells)
        s[::5] = rng.uniform(-0.9, 0.9, cells)[::5]       # fractions of both kinds
        g[ax] = (s * du / dt).astype(np.float32)
    return g.reshape((3,) + tuple(og.n))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("vbc", [V.VBC_OUTFLOW, V.VBC_PERIODIC])
def test_velocity_sweeps_on_ties(axis, vbc):
    og, hg, f32 = _tie_data(10 + axis)
    print("case: ties velocity", axis, vbc, flush=True)
    dt = 0.1
    g = _field(og, [axis], dt, np.random.default_rng(20 + axis))
    want = oracle.advect_velocity(og, axis, f32.astype(np.float64), g, dt, vbc=vbc)
    fin = torch.from_numpy(f32).cuda()
    out = torch.empty_like(fin)
    fn = [V.vlasov_advect_ux, V.vlasov_advect_uy, V.vlasov_advect_uz][axis]
    fn(hg, V.F32, vbc, fin, None, out, None, torch.from_numpy(g).cuda(), dt, None)
    torch.cuda.synchronize()
    _close(out.cpu().numpy(), want, float(f32.max()))


@pytest.mark.parametrize("vbc", [V.VBC_OUTFLOW, V.VBC_PERIODIC])
def test_kick_on_ties(vbc):
    # a cubic block, so the fused kick runs: 16^3 velocity cells
    og, hg, f32 = _tie_data(30, (4, 3, 4), (16, 16, 16))
    print("case: ties kick", vbc, flush=True)
    dt = 0.1
    g = _field(og, [0, 1, 2], dt, np.random.default_rng(31))
    want = oracle.kick(og, f32.astype(np.float64), g, dt, vbc=vbc)
    got = V.kick(V.State(hg, V.F32, torch.from_numpy(f32).cuda()), torch.from_numpy(g).cuda(),
                 dt, vbc=vbc)
    torch.cuda.synchronize()
    _close(got.f.cpu().numpy(), want, float(f32.max()))
