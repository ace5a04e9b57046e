"""64^3 velocity blocks (the paper's velocity resolution).

A 64^3 FP32 block is 1 MiB, more than a work-group's LDS, so the kick is
split: ux as a launch of its own, then uy and uz fused in LDS on slabs of
eight u_x rows (in place on the output for a step's second kick).  Checked
on the 32^3 x 32^3 workload's recipe (32 density modes of amplitude 0.1,
drifting field) on a 4^3 x 64^3 grid against the FP64 oracle: the kick, two
full steps (FP32, to the stated per-step bar) and the density after two
steps with FP16/BF16 storage.
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

LINF = 1e-5


def _workload():
    return inputs.scaled(inputs.workload(2), (4, 4, 4), (64, 64, 64))


def test_kick_against_oracle():
    w = _workload()
    print("case: kick 4^3 x 64^3 f32", flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    f32 = inputs.initial_f32(w)
    g = inputs.accel_field(w, inputs.potential(w), 0.0)
    ofl_ref = np.zeros(int(np.prod(w.n)))
    want = oracle.kick(og, f32.astype(np.float64), g, 0.5 * w.dt, outflow=ofl_ref)
    ofl = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    got = V.kick(V.State(hg, V.F32, torch.from_numpy(f32).cuda()), torch.from_numpy(g).cuda(),
                 0.5 * w.dt, outflow=ofl)
    torch.cuda.synchronize()
    err = float(np.max(np.abs(got.f.cpu().numpy().astype(np.float64) - want)))
    assert err <= LINF * float(want.max()), err
    np.testing.assert_allclose(ofl.cpu().numpy().reshape(-1), ofl_ref, rtol=1e-4, atol=1e-9)


def test_two_steps_against_oracle():
    """Each step from the oracle's previous state (rounded to float32) within
    1e-5 of max f; the free-running pair within n * 1e-5; f >= 0, in-domain
    mass within 1e-6 and mass plus outflow conserved."""
    w = _workload()
    print("case: two steps 4^3 x 64^3 f32", flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    f32 = inputs.initial_f32(w)
    pot = inputs.potential(w)
    f_ref = f32.astype(np.float64)
    st = V.State(hg, V.F32, torch.from_numpy(f32).cuda())
    ofl_ref = np.zeros(int(np.prod(w.n)))
    ofl = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    _, _, m0 = oracle.moments(og, f_ref)
    for n in range(2):
        gn = inputs.accel_field(w, pot, n * w.dt)
        gnp1 = inputs.accel_field(w, pot, (n + 1) * w.dt)
        g0, g1 = torch.from_numpy(gn).cuda(), torch.from_numpy(gnp1).cuda()
        prev32 = f_ref.astype(np.float32)
        one_ref = oracle.step(og, prev32.astype(np.float64), gn, gnp1, w.dt)
        one = V.step(V.State(hg, V.F32, torch.from_numpy(prev32).cuda()), g0, g1, w.dt)
        f_ref = oracle.step(og, f_ref, gn, gnp1, w.dt, outflow=ofl_ref)
        st = V.step(st, g0, g1, w.dt, outflow=ofl)
        torch.cuda.synchronize()
        fmax = float(f_ref.max())
        e_one = float(np.max(np.abs(one.f.cpu().numpy().astype(np.float64) - one_ref))) / fmax
        got = st.f.cpu().numpy()
        e_run = float(np.max(np.abs(got.astype(np.float64) - f_ref))) / fmax
        print(f"step {n + 1}: one-step {e_one:.2e} run {e_run:.2e}", flush=True)
        assert e_one <= LINF
        assert e_run <= (n + 1) * LINF
        assert got.min() >= 0.0
        _, _, mass = V.moments(st)
        _, _, mass_ref = oracle.moments(og, f_ref)
        assert float(mass) == pytest.approx(mass_ref, rel=1e-6)
    dx3 = np.prod([w.L[a] / w.n[a] for a in range(3)])
    _, _, mass = V.moments(st)
    assert float(mass) + float(ofl.sum()) * dx3 == pytest.approx(m0, rel=1e-6)


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
def test_scaled_storage_density(prec):
    """FP16/BF16 storage with 64-value uz-lines: density after two steps
    within 2e-3 (relative L2) of the oracle's, started from the decoded
    initial codes."""
    w = _workload()
    print("case: two steps 4^3 x 64^3", V.PREC_NAME[prec], flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    pot = inputs.potential(w)
    st = V.encode(hg, prec, torch.from_numpy(inputs.initial_f32(w)).cuda())
    f_ref = V.decode(st).double().cpu().numpy()
    for n in range(2):
        gn = inputs.accel_field(w, pot, n * w.dt)
        gnp1 = inputs.accel_field(w, pot, (n + 1) * w.dt)
        f_ref = oracle.step(og, f_ref, gn, gnp1, w.dt)
        st = V.step(st, torch.from_numpy(gn).cuda(), torch.from_numpy(gnp1).cuda(), w.dt)
    torch.cuda.synchronize()
    rho = V.moments(st)[0].cpu().numpy()
    rho_ref = oracle.moments(og, f_ref)[0]
    rel_l2 = float(np.linalg.norm(rho - rho_ref) / np.linalg.norm(rho_ref))
    print(f"density rel L2 {rel_l2:.2e}", flush=True)
    assert rel_l2 <= 2e-3
    assert float(V.decode(st).min()) >= 0.0


@pytest.mark.parametrize("vbc", [V.VBC_OUTFLOW, V.VBC_PERIODIC])
@pytest.mark.parametrize("prec", [V.F32, V.F16])
def test_kick_large_shifts(prec, vbc):
    """The split kick with shifts of up to 2.7 cells on every velocity axis
    (integer parts translated after the update) and both velocity
    boundaries.  FP32: against the oracle's three sweeps.  FP16: the ux
    launch is the public ux sweep (checked on its own elsewhere), so the
    kick's output is held against the oracle's uy and uz sweeps of the
    decoded ux result, to within its own codes' rounding."""
    n, nu = (2, 2, 2), (64, 64, 64)
    print("case: kick large shifts", V.PREC_NAME[prec], vbc, flush=True)
    og = oracle.Grid.make(n, nu, (1.0, 1.0, 1.0), (1.0, 1.0, 1.0))
    hg = V.make_grid(n, nu, (1.0, 1.0, 1.0), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(64 + vbc)
    f32 = rng.uniform(0.0, 1.0, og.shape).astype(np.float32) ** 2
    cells = int(np.prod(n))
    dt = 0.1
    du = 2.0 / 64
    s = rng.uniform(-2.7, 2.7, (3, cells))
    s[:, 0] = [1.0, -2.0, 0.0]                      # whole-cell shifts too
    g = (s * du / dt).astype(np.float32).reshape((3,) + n)
    gt = torch.from_numpy(g).cuda()
    st = V.encode(hg, prec, torch.from_numpy(f32).cuda())
    fin = V.decode(st).double().cpu().numpy()
    ofl_ref = np.zeros(cells)
    if prec == V.F32:
        want = oracle.kick(og, fin, g, dt, vbc=vbc, outflow=ofl_ref)
    else:
        ofl_ux = torch.zeros(n, dtype=torch.float64, device="cuda")
        mid = V.advect("ux", st, dt, g=gt, vbc=vbc, outflow=ofl_ux)
        torch.cuda.synchronize()
        ofl_ref += ofl_ux.cpu().numpy().reshape(-1)
        want = V.decode(mid).double().cpu().numpy()
        for axis in (1, 2):
            want = oracle.advect_velocity(og, axis, want, g, dt, vbc=vbc, outflow=ofl_ref)
    ofl = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = V.kick(st, gt, dt, vbc=vbc, outflow=ofl)
    torch.cuda.synchronize()
    got = V.decode(out).double().cpu().numpy()
    tol = 1e-5 * float(fin.max())
    if prec != V.F32:
        tol = tol + 1.01 * 2.0 ** -11 * out.scale.double().cpu().numpy()[..., None]
    assert np.all(np.abs(got - want) <= tol)
    assert float(got.min()) >= 0.0
    if vbc == V.VBC_OUTFLOW:
        np.testing.assert_allclose(ofl.cpu().numpy().reshape(-1), ofl_ref, rtol=1e-4,
                                   atol=1e-6 * float(fin.max()) * du ** 3 * 64 ** 2)
