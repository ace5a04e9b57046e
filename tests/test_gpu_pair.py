"""z sweep with the two halves of each uz-line paired in one lane.

With FP16/BF16 storage the z sweep pairs the halves of every uz-line when
all lines of the upper half (u_z > 0) move up and all lines of the lower
half move down, each by less than one cell, on line lengths and uz-line
lengths of 16, 32 or 64; otherwise (a negative time step, a longer step,
other shapes) it walks one line per lane with per-lane stencil selects.

Reversing the u_z index maps a step dt onto a step -dt exactly on these
grids (u_{nu-1-j} = -u_j holds in binary when du is a power of two), so the
paired walk must reproduce the per-lane walk's codes and scales to the bit;
and both must stay within the storage rounding of the FP64 oracle.  The
three grids cover the three lane exchanges (uz-line halves of 4, 8 and 16
lanes) and the three compiled line lengths.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

HALF_ULP = {V.F16: 2.0 ** -11, V.BF16: 2.0 ** -8}

# n, nu, L: dz = 1, so the largest z shift is dt (1 - du/2) < 1 cell
GRIDS = {
    "nuz16_nz16": ((2, 3, 16), (4, 8, 16), (1.0, 1.0, 16.0)),
    "nuz32_nz32": ((3, 2, 32), (4, 4, 32), (1.0, 1.0, 32.0)),
    "nuz64_nz64": ((2, 2, 64), (2, 2, 64), (1.0, 1.0, 64.0)),
}


def _input(name, seed):
    n, nu, L = GRIDS[name]
    og = oracle.Grid.make(n, nu, L, (1.0, 1.0, 1.0))
    hg = V.make_grid(n, nu, L, (1.0, 1.0, 1.0))
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 1.0, og.shape).astype(np.float32) ** 2
    return og, hg, f


@pytest.mark.parametrize("prec", [V.F16, V.BF16, V.F32])
@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("dt", [0.6, 0.05])
def test_paired_walk_equals_per_lane_walk(prec, name, dt):
    og, hg, f = _input(name, 31)
    print("case: pair bits", V.PREC_NAME[prec], name, dt, flush=True)
    ft = torch.from_numpy(f).cuda()
    a = V.advect("z", V.encode(hg, prec, ft), dt)                       # paired (scaled storage)
    b = V.advect("z", V.encode(hg, prec, ft.flip(-1).contiguous()), -dt)  # per-lane walk
    torch.cuda.synchronize()
    assert torch.equal(a.f, b.f.flip(-1))
    if prec != V.F32:
        assert torch.equal(a.scale, b.scale)


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
@pytest.mark.parametrize("name", list(GRIDS))
def test_paired_walk_within_storage_rounding(prec, name):
    og, hg, f = _input(name, 32)
    print("case: pair oracle", V.PREC_NAME[prec], name, flush=True)
    st = V.encode(hg, prec, torch.from_numpy(f).cuda())
    fin = V.decode(st).double().cpu().numpy()
    dt = 0.6
    want = oracle.advect_position(og, 2, fin, dt)
    out = V.advect("z", st, dt)
    torch.cuda.synchronize()
    got = V.decode(out).double().cpu().numpy()
    scale = out.scale.double().cpu().numpy()[..., None]
    np.testing.assert_allclose(np.abs(got).max(axis=-1, keepdims=True), scale,
                               rtol=2 * HALF_ULP[prec])
    bound = 1.01 * HALF_ULP[prec] * scale + 1e-5 * float(fin.max())
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err - bound).max())
    # the content of every periodic z line is kept, up to the output codes' rounding
    drift = np.abs(got.sum(axis=2) - fin.sum(axis=2))
    allowed = (1.01 * HALF_ULP[prec] * scale[..., 0]).sum(axis=2) + 1e-5 * float(fin.max()) * og.n[2]
    assert np.all(drift <= allowed[..., None]), float((drift - allowed[..., None]).max())
