"""vlasov_steps: steps of Eq. (5) with the half kicks between steps merged.

* against the oracle's merged composition (oracle.steps_merged, pinned on the
  CPU) on the tiny workload, FP32, at the sweeps' bar;
* one merged step is vlasov_step to the bit; any number of them is the chain
  of single launches kick(dt/2), z, y, x, kick(dt), ..., kick(dt/2) to the
  bit (FP32 and FP16 storage);
* argument errors.
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


def _run_steps(hg, st, fields, nsteps, dt, a2inv=None, outflow=None):
    out = V.empty_state(hg, st.prec, "cuda")
    nb = V.vlasov_steps_workspace_bytes(hg, st.prec)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    V.vlasov_steps(hg, st.prec, V.VBC_OUTFLOW, st.f, st.scale, out.f, out.scale, fields, nsteps,
                   dt, a2inv, work, nb, outflow)
    return out


def test_steps_against_oracle_tiny_workload():
    w = inputs.workload(1)
    print("case: merged steps vs oracle", w.name, flush=True)
    og = oracle.Grid.make(w.n, w.nu, w.L, w.umax)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    f32 = inputs.initial_f32(w)
    pot = inputs.potential(w)
    nsteps = 3
    fl = [inputs.accel_field(w, pot, k * w.dt) for k in range(nsteps + 1)]
    cells = int(np.prod(w.n))
    ofl_ref = np.zeros(cells)
    want = oracle.steps_merged(og, fl, f32.astype(np.float64), w.dt, outflow=ofl_ref)
    fields = torch.from_numpy(np.stack(fl)).cuda()
    ofl = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    out = _run_steps(hg, V.State(hg, V.F32, torch.from_numpy(f32).cuda()), fields, nsteps, w.dt,
                     outflow=ofl)
    torch.cuda.synchronize()
    got = out.f.cpu().numpy().astype(np.float64)
    err = np.abs(got - want).max()
    assert err <= 1e-5 * float(want.max()), err
    assert got.min() >= 0.0
    np.testing.assert_allclose(ofl.cpu().numpy().reshape(-1), ofl_ref, rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("prec", [V.F32, V.F16])
def test_steps_are_the_chain_of_single_launches(prec):
    print("case: merged steps vs launches", V.PREC_NAME[prec], flush=True)
    n, nu = (6, 5, 4), (16, 16, 16)
    hg = V.make_grid(n, nu, (1.0, 1.3, 0.8), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(12)
    f = torch.from_numpy(rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 2).cuda()
    st = V.encode(hg, prec, f)
    dt = 0.19
    nsteps = 3
    fields = torch.from_numpy(rng.uniform(-3, 3, (nsteps + 1, 3) + n).astype(np.float32)).cuda()
    a2 = [1.0, 0.7, 1.3]
    o1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    o2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    got = _run_steps(hg, st, fields, nsteps, dt, a2inv=a2, outflow=o1)
    a = V.kick(st, fields[0], 0.5 * dt, outflow=o2)
    for k in range(nsteps):
        for ax in ("z", "y", "x"):
            a = V.advect(ax, a, dt * a2[k])
        a = V.kick(a, fields[k + 1], dt if k + 1 < nsteps else 0.5 * dt, outflow=o2)
    torch.cuda.synchronize()
    assert torch.equal(got.f, a.f)
    if prec != V.F32:
        assert torch.equal(got.scale, a.scale)
    assert torch.equal(o1, o2)
    # one merged step is vlasov_step
    one = _run_steps(hg, st, fields[:2].contiguous(), 1, dt)
    ref = V.step(st, fields[0], fields[1], dt)
    torch.cuda.synchronize()
    assert torch.equal(one.f, ref.f)


def test_steps_argument_errors():
    n, nu = (3, 2, 2), (16, 16, 16)
    hg = V.make_grid(n, nu)
    f = torch.rand(V.grid_shape(hg), device="cuda")
    out = torch.empty_like(f)
    fields = torch.zeros((3, 3) + n, dtype=torch.float32, device="cuda")
    nb = V.vlasov_steps_workspace_bytes(hg, V.F32)
    assert nb >= 2 * f.numel() * 4
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for bad in (dict(nsteps=0), dict(work_bytes=nb - 1)):
        kw = dict(nsteps=2, work_bytes=nb)
        kw.update(bad)
        with pytest.raises(V.VlasovError):
            V.vlasov_steps(hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, fields, kw["nsteps"],
                           0.1, None, work, kw["work_bytes"], None)
    with pytest.raises(V.VlasovError):       # fields overlapping f_out
        V.vlasov_steps(hg, V.F32, V.VBC_OUTFLOW, f, None, out, None, out, 2, 0.1, None, work, nb,
                       None)
