"""FP16 / BF16 storage (one FP32 scale per uz-line, FP32 flux arithmetic).

The FP64 oracle has no storage rounding, so the comparison states an error:
per sweep, each decoded output lies within the code's half-ulp of its line
scale (plus the FP32 bar); after ten Strang steps the density's relative L2
error stays within 2e-3, on the seeded tiny workload and at the precision
form's stated size, 32^3 x 32^3 (reference density from the FP64 oracle,
tests/golden/make_density_32x32.py).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

HALF_ULP = {V.F16: 2.0 ** -11, V.BF16: 2.0 ** -8}


def _grid(name):
    return {
        "g16": ((6, 5, 7), (8, 12, 16), (1.0, 0.8, 1.3), (1.0, 1.2, 0.9)),
        "g32": ((4, 6, 5), (8, 6, 32), (1.0, 2.0, 3.0), (1.0, 1.0, 1.0)),
        "g64": ((3, 4, 20), (4, 2, 64), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
        "c64": ((2, 1, 2), (64, 64, 64), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
    }[name]


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
@pytest.mark.parametrize("name", ["g16", "g32", "g64", "c64"])
@pytest.mark.parametrize("axis", ["x", "y", "z", "ux", "uy", "uz"])
def test_sweep_error_within_storage_rounding(prec, name, axis):
    n, nu, L, U = _grid(name)
    print("case:", V.PREC_NAME[prec], name, axis, flush=True)
    og = oracle.Grid.make(n, nu, L, U)
    hg = V.make_grid(n, nu, L, U)
    rng = np.random.default_rng(17)
    f = torch.from_numpy(rng.uniform(0.0, 1.0, og.shape).astype(np.float32) ** 3).cuda()
    st = V.encode(hg, prec, f)
    fin = V.decode(st).double().cpu().numpy()          # what the kernel reads
    if axis in ("x", "y", "z"):
        a = "xyz".index(axis)
        dt = 0.37
        want = oracle.advect_position(og, a, fin, dt)
        out = V.advect(axis, st, dt)
    else:
        a = "xyz".index(axis[1])
        cells = int(np.prod(n))
        du = 2 * U[a] / nu[a]
        field = np.zeros((3, cells), np.float32)
        field[a] = (rng.uniform(-2.5, 2.5, cells) * du / 0.1).astype(np.float32)
        field = field.reshape((3,) + tuple(n))
        want = oracle.advect_velocity(og, a, fin, field, 0.1)
        out = V.advect(axis, st, 0.1, g=torch.from_numpy(field).cuda())
    torch.cuda.synchronize()
    got = V.decode(out).double().cpu().numpy()
    scale = out.scale.double().cpu().numpy()[..., None]
    # the stored scale is the line maximum of the result it encodes
    line_max = np.abs(got).max(axis=-1, keepdims=True)
    np.testing.assert_allclose(line_max, scale, rtol=2 * HALF_ULP[prec])
    bound = 1.01 * HALF_ULP[prec] * scale + 1e-5 * float(fin.max())
    err = np.abs(got - want)
    assert np.all(err <= bound), float((err - bound).max())
    assert got.min() >= 0.0


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
def test_ten_steps_density_error(prec):
    """Seeded tiny workload, 10 Strang steps: density rel. L2 <= 2e-3 vs the FP64 oracle."""
    w = inputs.workload(1)
    print("case: ten steps", V.PREC_NAME[prec], flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    f32 = inputs.initial_f32(w)
    pot = inputs.potential(w)
    st = V.encode(hg, prec, torch.from_numpy(f32).cuda())
    f_ref = V.decode(st).double().cpu().numpy()
    steps = 10
    for n in range(steps):
        gn = inputs.accel_field(w, pot, n * w.dt)
        gnp1 = inputs.accel_field(w, pot, (n + 1) * w.dt)
        f_ref = oracle.step(og, f_ref, gn, gnp1, w.dt)
        st = V.step(st, torch.from_numpy(gn).cuda(), torch.from_numpy(gnp1).cuda(), w.dt)
    torch.cuda.synchronize()
    rho, _, mass = V.moments(st)
    rho_ref, _, mass_ref = oracle.moments(og, f_ref)
    rho = rho.cpu().numpy()
    rel_l2 = np.linalg.norm(rho - rho_ref) / np.linalg.norm(rho_ref)
    mass_err = abs(float(mass) - mass_ref) / mass_ref
    print(f"{V.PREC_NAME[prec]}: density rel L2 {rel_l2:.3e}, mass rel err {mass_err:.3e}")
    assert rel_l2 <= 2e-3
    assert mass_err <= 2e-3


def test_scaled_storage_rejects_unsupported_lines():
    hg = V.make_grid((2, 2, 2), (4, 4, 6))
    f = torch.zeros(V.grid_shape(hg), dtype=torch.float16, device="cuda")
    s = torch.zeros(V.grid_shape(hg)[:-1], device="cuda")
    with pytest.raises(V.VlasovError) as e:
        V.vlasov_advect_x(hg, V.F16, f, s, torch.empty_like(f), torch.empty_like(s), 0.1)
    assert e.value.code == -2


GOLDEN_32 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "density_32x32_10steps.npz")


@pytest.fixture(scope="module")
def ic_32x32():
    w = inputs.workload(2)
    return w, torch.from_numpy(inputs.initial_f32(w))


@pytest.mark.parametrize("prec", [V.F32, V.F16, V.BF16])
def test_density_error_32x32_ten_steps(prec, ic_32x32):
    """The precision form's stated size: 32^3 x 32^3, 10 steps with the drifting
    field, density against the FP64 oracle's (tests/golden/make_density_32x32.py):
    FP32 storage within 1e-5, FP16/BF16 storage within 2e-3 relative L2; in-domain
    mass plus outflow within 1e-6 (FP32) or 2e-3 of the oracle's."""
    w, f0 = ic_32x32
    print("case: density error 32^3x32^3", V.PREC_NAME[prec], flush=True)
    ref = np.load(GOLDEN_32)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    pot = inputs.potential(w)
    st = V.encode(hg, prec, f0.cuda())
    ofl = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    work = torch.empty(V.vlasov_step_workspace_bytes(hg, prec), dtype=torch.uint8, device="cuda")
    for n in range(10):
        gn = torch.from_numpy(inputs.accel_field(w, pot, n * w.dt)).cuda()
        gnp1 = torch.from_numpy(inputs.accel_field(w, pot, (n + 1) * w.dt)).cuda()
        st = V.step(st, gn, gnp1, w.dt, outflow=ofl, work=work)
    rho, _, mass = V.moments(st)
    torch.cuda.synchronize()
    rho = rho.cpu().numpy()
    rel_l2 = np.linalg.norm(rho - ref["rho"]) / np.linalg.norm(ref["rho"])
    total = float(mass) + float(ofl.sum()) * float(np.prod([w.dx(a) for a in range(3)]))
    total_ref = float(ref["mass"]) + float(ref["outflow"]) * float(np.prod([w.dx(a) for a in range(3)]))
    mass_err = abs(total - total_ref) / total_ref
    print(f"{V.PREC_NAME[prec]}: density rel L2 {rel_l2:.3e}, mass+outflow rel err {mass_err:.3e}")
    tol = 1e-5 if prec == V.F32 else 2e-3
    assert rel_l2 <= tol
    assert mass_err <= (1e-6 if prec == V.F32 else 2e-3)
