"""vlasov_dispersion: rho, umean and the velocity dispersion tensor per
spatial cell, against the FP64 oracle's two-pass definition on the same
(decoded) values.

The library sums f, u f and u_l u_m f about u = 0 in one FP64 pass and
subtracts umean_l umean_m; on these inputs (<u^2> / sigma of order 1) that
keeps about 14 digits, so the bar is 1e-12 of umax_l umax_m.  rho and umean
are the bits vlasov_moments gives (the same sums in the same order).
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

SHAPES = {
    "v4": ((3, 4, 2), (16, 12, 16), (1.0, 1.0, 1.0), (1.0, 0.7, 1.3)),
    "ragged": ((2, 3, 5), (9, 7, 13), (1.0, 2.0, 1.0), (2.0, 1.0, 0.5)),
    "wide": ((2, 2, 2), (32, 32, 32), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
    "nuz4": ((3, 2, 2), (6, 5, 4), (1.0, 1.0, 1.0), (0.8, 1.0, 1.2)),
}
COMP = oracle.DISPERSION_COMPONENTS


def _bar(U):
    return 1e-12 * np.array([U[a] * U[b] for a, b in COMP]).reshape(6, 1, 1, 1)


@pytest.mark.parametrize("prec", [V.F32, V.F16, V.BF16])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_dispersion_against_oracle(prec, shape):
    n, nu, L, U = SHAPES[shape]
    if prec != V.F32 and nu[2] & (nu[2] - 1):
        pytest.skip("FP16/BF16 storage takes a power-of-two nu_z")
    print("case: dispersion", V.PREC_NAME[prec], shape, flush=True)
    hg = V.make_grid(n, nu, L, U)
    og = oracle.Grid.make(n, nu, L, U)
    rng = np.random.default_rng(31)
    f = rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 3
    f[0, 0, 0] = 0.0                                  # an empty cell
    st = V.encode(hg, prec, torch.from_numpy(f).cuda())
    rho, um, sig = V.dispersion(st)
    rho_m, um_m, _ = V.moments(st)
    torch.cuda.synchronize()
    assert torch.equal(rho, rho_m) and torch.equal(um, um_m)
    fd = V.decode(st).double().cpu().numpy()
    want = oracle.dispersion(og, fd)
    got = sig.cpu().numpy()
    assert np.all(got[:, 0, 0, 0] == 0.0)
    err = np.abs(got - want)
    assert np.all(err <= _bar(U)), float((err / _bar(U)).max())


def test_sampled_gaussian_on_the_device():
    """A drifting, correlated Gaussian block stored in FP32: the tensor is its
    covariance to the FP32 rounding of the stored values."""
    nu, U = (32, 32, 32), (3.2, 3.2, 3.2)
    hg = V.make_grid((1, 1, 2), nu, (1.0, 1.0, 1.0), U)
    c = [-U[a] + (np.arange(nu[a]) + 0.5) * 2 * U[a] / nu[a] for a in range(3)]
    Ug = np.stack(np.meshgrid(*c, indexing="ij"), -1)
    S = np.array([[0.25, 0.06, -0.03], [0.06, 0.16, 0.04], [-0.03, 0.04, 0.2]])
    u0 = np.array([0.3, -0.2, 0.1])
    d = Ug - u0
    blk = np.exp(-0.5 * np.einsum("...a,ab,...b->...", d, np.linalg.inv(S), d))
    f = np.stack([blk, 2.0 * blk])[None, None].astype(np.float32)
    rho, um, sig = V.dispersion(V.State(hg, V.F32, torch.from_numpy(f).cuda()))
    torch.cuda.synchronize()
    want = np.array([S[a, b] for a, b in COMP])
    for k in range(2):
        assert np.abs(sig.cpu().numpy()[:, 0, 0, k] - want).max() < 1e-6
        assert np.abs(um.cpu().numpy()[:, 0, 0, k] - u0).max() < 1e-6


@pytest.mark.parametrize("prec", [V.F32, V.F16])
def test_full_size_sampled_cells(prec):
    """The 64^3 x 32^3 workload's initial f (FP32, and encoded to FP16):
    sampled cells against the oracle on a one-cell grid (on the decoded
    values), and the tensor symmetric positive semi-definite in every cell."""
    w = inputs.workload(3)
    print("case: dispersion full size", V.PREC_NAME[prec], w.name, flush=True)
    hg = V.make_grid(w.n, w.nu, w.L, w.umax)
    if prec == V.F32:
        st = V.State(hg, V.F32, inputs.initial_f32_device(w))
    else:
        st = V.encode(hg, prec, inputs.initial_f32_device(w))
    rho, um, sig = V.dispersion(st)
    torch.cuda.synchronize()
    og1 = oracle.Grid.make((1, 1, 1), w.nu, (1.0, 1.0, 1.0), w.umax)
    rng = np.random.default_rng(32)
    for _ in range(8):
        c = tuple(int(v) for v in rng.integers(0, w.n[0], 3))
        blk = st.f[c].float()
        if prec != V.F32:                # the stored value: FP32 product code x scale
            blk = blk * st.scale[c][..., None]
        blk = blk.double().cpu().numpy()[None, None, None]
        want = oracle.dispersion(og1, blk)[:, 0, 0, 0]
        got = sig[(slice(None),) + c].cpu().numpy()
        assert np.all(np.abs(got - want) <= _bar(w.umax).reshape(6)), c
    sh = sig.cpu().numpy()
    t = np.empty(tuple(w.n) + (3, 3))
    for k, (a, b) in enumerate(COMP):
        t[..., a, b] = sh[k]
        t[..., b, a] = sh[k]
    ev = np.linalg.eigvalsh(t.reshape(-1, 3, 3))
    assert ev.min() >= -1e-12 * float(sh[[0, 3, 5]].max())


def test_dispersion_errors():
    hg = V.make_grid((2, 2, 2), (8, 8, 8))
    f = torch.zeros(V.grid_shape(hg), device="cuda")
    rho = torch.empty((2, 2, 2), dtype=torch.float64, device="cuda")
    sig = torch.empty((6, 2, 2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(V.VlasovError) as e:
        V.vlasov_dispersion(hg, V.F32, f, None, sig[0], None, sig)
    assert e.value.code == -4
    with pytest.raises(V.VlasovError) as e:
        V.vlasov_dispersion(hg, V.F16, f, None, rho, None, sig)
    assert e.value.code == -3
    V.vlasov_dispersion(hg, V.F32, f, None, rho, None, sig)     # umean may be NULL
    torch.cuda.synchronize()
    assert float(sig.abs().max()) == 0.0 and float(rho.abs().max()) == 0.0
