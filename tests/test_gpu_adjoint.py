"""GPU tangents and adjoints of the sweeps, the step and the moments.

* duality on the GPU: <T v, w> = <v, A w> (+ <g_dot, lam_g>) within 1e-4 in FP32;
* against the FP64 oracle derivatives on the same input (frozen selections
  agree except at near-ties, absent in these tie-free random inputs);
* the step adjoint on an 8^3 x 8^3 grid, sweep by sweep and element by
  element against the oracle (near-ties excluded by the oracle's margins).
"""
import numpy as np
import pytest

import adjoint_check
import oracle
from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

GRIDS = {
    "ragged": ((5, 4, 6), (6, 5, 7), (1.0, 0.7, 1.3), (1.0, 0.9, 1.1)),
    "cube8": ((6, 5, 4), (8, 8, 8), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
}


def _setup(name, seed):
    n, nu, L, U = GRIDS[name]
    og = oracle.Grid.make(n, nu, L, U)
    hg = V.make_grid(n, nu, L, U)
    rng = np.random.default_rng(seed)
    f = (rng.uniform(0.05, 1.0, og.shape) ** 2).astype(np.float32)
    return og, hg, rng, f


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_position_derivatives(name, axis):
    og, hg, rng, f = _setup(name, 1)
    print("case: position derivative", name, axis, flush=True)
    a = "xyz".index(axis)
    dt = 0.29
    v = rng.standard_normal(og.shape).astype(np.float32)
    w = rng.standard_normal(og.shape).astype(np.float32)
    tv = torch.empty_like(_cuda(f))
    aw = torch.empty_like(tv)
    getattr(V, f"vlasov_advect_{axis}_tan")(hg, _cuda(f), _cuda(v), tv, dt)
    getattr(V, f"vlasov_advect_{axis}_adj")(hg, _cuda(f), _cuda(w), aw, dt)
    torch.cuda.synchronize()
    tv, aw = tv.cpu().numpy().astype(np.float64), aw.cpu().numpy().astype(np.float64)
    lhs, rhs = np.vdot(tv, w), np.vdot(v, aw)
    assert lhs == pytest.approx(rhs, rel=1e-4)
    f64 = f.astype(np.float64)
    tv_ref = oracle.advect_position_tan(og, a, f64, v.astype(np.float64), dt)
    aw_ref = oracle.advect_position_adj(og, a, f64, w.astype(np.float64), dt)
    np.testing.assert_allclose(tv, tv_ref, rtol=0, atol=1e-4 * np.abs(tv_ref).max())
    np.testing.assert_allclose(aw, aw_ref, rtol=0, atol=1e-4 * np.abs(aw_ref).max())


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("axis", ["ux", "uy", "uz"])
@pytest.mark.parametrize("vbc", [0, 1])
def test_velocity_derivatives(name, axis, vbc):
    og, hg, rng, f = _setup(name, 2)
    print("case: velocity derivative", name, axis, vbc, flush=True)
    a = "xyz".index(axis[1])
    cells = int(np.prod(og.n))
    dt = 0.13
    du = 2 * og.umax[a] / og.nu[a]
    field = np.zeros((3, cells), np.float32)
    field[a] = (rng.uniform(-2.7, 2.7, cells) * du / dt).astype(np.float32)
    field = field.reshape((3,) + tuple(og.n))
    gd = rng.standard_normal((3,) + tuple(og.n)).astype(np.float32)
    v = rng.standard_normal(og.shape).astype(np.float32)
    w = rng.standard_normal(og.shape).astype(np.float32)
    tv = torch.empty_like(_cuda(f))
    aw = torch.empty_like(tv)
    lg = torch.zeros((3,) + tuple(og.n), dtype=torch.float32, device="cuda")
    getattr(V, f"vlasov_advect_{axis}_tan")(hg, vbc, _cuda(f), _cuda(field), _cuda(gd), dt,
                                            _cuda(v), tv)
    getattr(V, f"vlasov_advect_{axis}_adj")(hg, vbc, _cuda(f), _cuda(field), dt, _cuda(w), aw, lg)
    torch.cuda.synchronize()
    tv, aw = tv.cpu().numpy().astype(np.float64), aw.cpu().numpy().astype(np.float64)
    lg = lg.cpu().numpy().astype(np.float64)
    lhs = np.vdot(tv, w)
    rhs = np.vdot(v, aw) + np.vdot(gd.astype(np.float64), lg)
    assert lhs == pytest.approx(rhs, rel=1e-4)
    f64 = f.astype(np.float64)
    tv_ref = oracle.advect_velocity_tan(og, a, f64, field, dt, v.astype(np.float64),
                                        g_dot=gd.astype(np.float64), vbc=vbc)
    lg_ref = np.zeros(3 * cells)
    aw_ref = oracle.advect_velocity_adj(og, a, f64, field, dt, w.astype(np.float64), vbc=vbc,
                                        lam_g=lg_ref)
    np.testing.assert_allclose(tv, tv_ref, rtol=0, atol=1e-4 * np.abs(tv_ref).max())
    np.testing.assert_allclose(aw, aw_ref, rtol=0, atol=1e-4 * np.abs(aw_ref).max())
    np.testing.assert_allclose(lg.reshape(-1), lg_ref, rtol=0, atol=1e-4 * np.abs(lg_ref).max())


def test_step_adjoint_against_oracle():
    """8^3 x 8^3 grid of the adjoint workload's recipe: every one of the nine
    transposed sweeps element by element against the oracle's (outputs of
    lines with a selection within 1e-5 of a tie excluded and counted), and
    their chain equal to vlasov_step_adj bit for bit."""
    w = inputs.scaled(inputs.workload(5), (8, 8, 8), (8, 8, 8))
    print("case: step adjoint", w.name, flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    rng = np.random.default_rng(3)
    f = (inputs.initial_f(w) * (1 + 0.01 * rng.uniform(-1, 1, og.shape))).astype(np.float32)
    pot = inputs.potential(w)
    gn, gnp1 = inputs.accel_field(w, pot, 0.0), inputs.accel_field(w, pot, w.dt)
    lam = rng.standard_normal(og.shape).astype(np.float32)
    lam_c, lgn_c, lgnp1_c, excl, total = adjoint_check.check_step_adjoint(
        hg, og, _cuda(f), _cuda(gn), _cuda(gnp1), w.dt, _cuda(lam))
    print(f"step adjoint: {excl} of {total} compared elements excluded as near-ties")
    assert excl <= 0.01 * total
    nbytes = V.vlasov_step_adj_workspace_bytes(hg)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    lam_in = torch.empty_like(_cuda(f))
    lgn = torch.zeros((3,) + tuple(w.n), dtype=torch.float32, device="cuda")
    lgnp1 = torch.zeros_like(lgn)
    V.vlasov_step_adj(hg, 0, _cuda(f), _cuda(gn), _cuda(gnp1), w.dt, 1.0, _cuda(lam), lam_in,
                      lgn, lgnp1, work, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(lam_in, lam_c)
    assert torch.equal(lgn, lgn_c) and torch.equal(lgnp1, lgnp1_c)


def test_moments_adjoint_against_oracle():
    og, hg, rng, f = _setup("ragged", 4)
    cells = int(np.prod(og.n))
    lr = rng.standard_normal(cells)
    lu = rng.standard_normal(3 * cells)
    ref = oracle.moments_adj(og, f.astype(np.float64), lr, lu)
    st = V.State(hg, V.F32, _cuda(f))
    rho, um, _ = V.moments(st)
    lam_f = torch.zeros_like(st.f)
    V.vlasov_moments_adj(hg, rho, um, _cuda(lr), _cuda(lu), lam_f)
    torch.cuda.synchronize()
    np.testing.assert_allclose(lam_f.cpu().numpy(), ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())
