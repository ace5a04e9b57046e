"""Parity at the throughput workload's full size (64^3 x 32^3 = 8.6e9 cells),
in the launch configuration bench.py times: kick, z, y, x, kick through the
public single-launch calls, FP32 and FP16 storage.

After each launch, sampled outputs that the oracle computes piece by piece:
whole velocity blocks of 32 sampled spatial cells for the kicks (the
oracle's three velocity sweeps on a one-cell grid with that cell's field),
and for the drifts 4 whole spatial lines along the drift axis with every
velocity cell of them (2.1e6 cells each: the oracle's sweep on a grid of
that one line, whose cell width and shifts are the full grid's).  Over
the whole array: positivity, and mass plus the velocity-face outflow kept
(FP64 moments).  FP32 is held to the sweeps' bar (1e-5 of max f per
launch); FP16 to its output codes' rounding plus that bar.
"""
import numpy as np
import pytest

import oracle
from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

HALF_ULP = {V.F32: 0.0, V.F16: 2.0 ** -11}


def _decode_cells(st, idx):
    """FP64 velocity blocks [k][jx][jy][jz] of spatial cells idx (list of (ix, iy, iz))."""
    out = []
    for c in idx:
        blk = st.f[c].double()
        if st.prec != V.F32:
            blk = blk * st.scale[c].double()[..., None]
        out.append(blk.cpu().numpy())
    return np.stack(out)


def _block_scales(st, idx):
    if st.prec == V.F32:
        return None
    return np.stack([st.scale[c].double().cpu().numpy() for c in idx])


def _bundle(st, axis, ix):
    """FP64 values of the spatial line along `axis` through ix (ix[axis]
    ignored) with its whole velocity blocks, shaped as a one-line 6D grid,
    and the scales broadcast to it (None for FP32)."""
    sl = list(ix)
    sl[axis] = slice(None)
    x = st.f[tuple(sl)].double()                     # [n_axis][jx][jy][jz]
    shape = [1, 1, 1]
    shape[axis] = x.shape[0]
    if st.prec == V.F32:
        return x.cpu().numpy().reshape(tuple(shape) + x.shape[1:]), None
    sc = st.scale[tuple(sl)].double()[..., None]     # [n_axis][jx][jy][1]
    return ((x * sc).cpu().numpy().reshape(tuple(shape) + x.shape[1:]),
            sc.expand_as(x).cpu().numpy().reshape(tuple(shape) + x.shape[1:]))


@pytest.mark.parametrize("prec", [V.F32, V.F16])
def test_full_size_step_sampled_against_oracle(prec):
    w = inputs.workload(3)
    print("case: full size", V.PREC_NAME[prec], w.name, flush=True)
    grid = V.make_grid(w.n, w.nu, w.L, w.umax)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    og1 = oracle.Grid.make((1, 1, 1), w.nu, (1.0, 1.0, 1.0), w.umax)
    rng = np.random.default_rng(91)
    f0 = inputs.initial_f32_device(w)
    cur = V.encode(grid, prec, f0)
    del f0
    pot = inputs.potential(w)
    gn = inputs.accel_field(w, pot, 0.0)
    gnp1 = inputs.accel_field(w, pot, w.dt)
    fields = [torch.from_numpy(gn).cuda(), torch.from_numpy(gnp1).cuda()]
    nb = V.vlasov_step_workspace_bytes(grid, prec)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    outflow = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    _, _, mass0 = V.moments(cur)
    mass0 = float(mass0)
    fmax = float(cur.f.float().abs().max()) * (1.0 if prec == V.F32 else float(cur.scale.max()))
    bar = 1e-5 * fmax
    cells = [tuple(int(v) for v in rng.integers(0, w.n[0], 3)) for _ in range(32)]
    for step, name in enumerate(["kick", "z", "y", "x", "kick"]):
        out = V.empty_state(grid, prec, "cuda")
        if name == "kick":
            g = fields[0 if step == 0 else 1]
            V.vlasov_kick(grid, prec, V.VBC_OUTFLOW, cur.f, cur.scale, out.f, out.scale, g,
                          0.5 * w.dt, work, nb, outflow)
            torch.cuda.synchronize()
            xin = _decode_cells(cur, cells)
            got = _decode_cells(out, cells)
            gh = g.cpu().numpy()
            for k, c in enumerate(cells):
                g1 = gh[(slice(None),) + c].reshape(3, 1, 1, 1)
                want = oracle.kick(og1, xin[k][None, None, None], g1, 0.5 * w.dt)[0, 0, 0]
                tol = bar
                if prec != V.F32:
                    tol = bar + 1.01 * HALF_ULP[prec] * _block_scales(out, [c])[0][..., None]
                assert np.all(np.abs(got[k] - want) <= tol), (name, c)
        else:
            axis = "xyz".index(name)
            getattr(V, f"vlasov_advect_{name}")(grid, prec, cur.f, cur.scale, out.f, out.scale,
                                                w.dt)
            torch.cuda.synchronize()
            n1 = [1, 1, 1]
            n1[axis] = w.n[axis]
            L1 = [1.0, 1.0, 1.0]
            L1[axis] = w.L[axis]
            og_line = oracle.Grid.make(tuple(n1), w.nu, tuple(L1), w.umax)
            for _ in range(4):
                ix = tuple(int(v) for v in rng.integers(0, w.n[0], 3))
                b_in, _ = _bundle(cur, axis, ix)
                b_out, sc_out = _bundle(out, axis, ix)
                want = oracle.advect_position(og_line, axis, b_in, w.dt)
                tol = bar if sc_out is None else bar + 1.01 * HALF_ULP[prec] * sc_out
                assert np.all(np.abs(b_out - want) <= tol), (name, ix)
        del cur
        cur = out
    # whole array: positivity; mass plus what left through the velocity faces
    assert float(cur.f.float().min()) >= 0.0
    _, _, mass1 = V.moments(cur)
    dx3 = np.prod([w.L[a] / w.n[a] for a in range(3)])
    lost = float(outflow.sum()) * dx3
    rel = 1e-6 if prec == V.F32 else 2e-3
    assert float(mass1) + lost == pytest.approx(mass0, rel=rel)
