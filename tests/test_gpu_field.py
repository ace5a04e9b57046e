"""vlasov_field: the field of a density on the periodic mesh (Eq. 2).

Against the oracle's solve (numpy FFT, pinned on the CPU against closed
forms) on cubic, mixed odd/even and the throughput workload's meshes, FP64
inside and FP32 out; and the argument errors.
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

MESHES = {
    "16cube": ((16, 16, 16), (1.0, 1.0, 1.0)),
    "mixed": ((12, 9, 14), (1.0, 2.0, 0.7)),
    "throughput": ((64, 64, 64), (1.0, 2.0, 10.0)),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("kind", ["random", "workload"])
def test_field_against_oracle(name, kind):
    n, L = MESHES[name]
    print("case: field", name, kind, flush=True)
    og = oracle.Grid.make(n, (4, 4, 4), L, (1, 1, 1))
    hg = V.make_grid(n, (4, 4, 4), L)
    rng = np.random.default_rng(71)
    if kind == "random":
        rho = rng.uniform(0.5, 1.5, n)
    else:
        w = inputs.Workload("field", n, (4, 4, 4), L=L, n_modes=16, kmax=3, amp=0.2)
        rho = 1.0 + inputs.density_contrast(w, seed=5)
    c = 3.7
    want = oracle.field_from_density(og, rho, c)
    got = V.field(hg, torch.from_numpy(rho).cuda(), c)
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 2e-7 * scale


def test_field_argument_errors():
    hg = V.make_grid((8, 8, 8), (4, 4, 4))
    rho = torch.ones((8, 8, 8), dtype=torch.float64, device="cuda")
    out = torch.empty((3, 8, 8, 8), dtype=torch.float32, device="cuda")
    nb = V.vlasov_field_workspace_bytes(hg)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(V.VlasovError):
        V.vlasov_field(hg, rho, 1.0, out, work, nb - 1)
    with pytest.raises(V.VlasovError):
        V.vlasov_field(hg, None, 1.0, out, work, nb)
    with pytest.raises(V.VlasovError):
        V.vlasov_field(hg, rho, float("nan"), out, work, nb)
    bad = V.make_grid((8, 8, 8), (4, 4, 4), (1.0, 0.0, 1.0))
    with pytest.raises(V.VlasovError):
        V.vlasov_field(bad, rho, 1.0, out, work, nb)
    V.vlasov_field(hg, rho, 1.0, out, work, nb)          # uniform density: no field
    torch.cuda.synchronize()
    assert float(out.abs().max()) <= 1e-12
