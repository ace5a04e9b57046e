"""Checkpoint and resume: four steps equal two steps, save, load, two steps,
bit for bit (f, scales and the outflow tally), for FP32 and FP16 storage."""
import numpy as np
import pytest

from paper_2110_15867_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402


@pytest.mark.parametrize("prec", [V.F32, V.F16, V.BF16])
def test_four_steps_equal_two_plus_resume_plus_two(prec, tmp_path):
    w = inputs.workload(1)
    print("case: resume", V.PREC_NAME[prec], flush=True)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    pot = inputs.potential(w)
    fields = [torch.from_numpy(inputs.accel_field(w, pot, n * w.dt)).cuda() for n in range(5)]

    def run(st, n0, n1, ofl):
        for n in range(n0, n1):
            st = V.step(st, fields[n], fields[n + 1], w.dt, outflow=ofl)
        return st

    st0 = V.encode(hg, prec, torch.from_numpy(inputs.initial_f32(w)).cuda())
    ofl_a = torch.zeros(tuple(w.n), dtype=torch.float64, device="cuda")
    a = run(st0, 0, 4, ofl_a)
    ofl_b = torch.zeros_like(ofl_a)
    b = run(st0, 0, 2, ofl_b)
    path = str(tmp_path / "state.npz")
    V.save(path, b, step=2, t=2 * w.dt, outflow=ofl_b)
    del b, ofl_b
    c, step, t, ofl_c = V.load(path)
    assert step == 2 and t == 2 * w.dt and c.prec == prec
    assert tuple(c.grid.n) == tuple(w.n) and tuple(c.grid.nu) == tuple(w.nu)
    c = run(c, step, 4, ofl_c)
    torch.cuda.synchronize()
    assert torch.equal(a.f.view(torch.int16) if prec != V.F32 else a.f,
                       c.f.view(torch.int16) if prec != V.F32 else c.f)
    if prec != V.F32:
        assert torch.equal(a.scale, c.scale)
    assert torch.equal(ofl_a, ofl_c)
