"""The storage codec at the boundary (vlasov_encode / vlasov_decode).

* A sweep with FP16/BF16 storage decodes its input, runs FP32 arithmetic and
  encodes its result.  The same sweep with FP32 storage on vlasov_decode's
  values gives that FP32 result, so vlasov_encode of it must reproduce the
  scaled sweep's codes and scales bit for bit (all six sweeps and the kick).
* Scales are the exact line maxima; codes are within one code unit of the
  round-to-nearest quotient (the reciprocal is the hardware's); all-zero
  lines, and lines whose maximum lies below the normal FP32 range, encode to
  zero codes.
* Argument errors.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs an MI355X", allow_module_level=True)

from paper_2110_15867_amd import vlasov as V  # noqa: E402

GRIDS = {
    "cube16": ((4, 5, 6), (16, 16, 16)),
    "nuz32": ((3, 4, 4), (12, 10, 32)),
    "nuz4": ((6, 5, 4), (8, 6, 4)),
}


def _state(name, prec, seed):
    n, nu = GRIDS[name]
    hg = V.make_grid(n, nu, (1.0, 0.8, 1.3), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 1, V.grid_shape(hg)).astype(np.float32) ** 3
    f[0, 0, 0, 1, 2] = 0.0                       # an all-zero uz-line
    return hg, V.encode(hg, prec, torch.from_numpy(f).cuda()), rng


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("axis", ["x", "y", "z", "ux", "uy", "uz", "kick"])
def test_encode_reproduces_the_codes_a_sweep_stores(prec, name, axis):
    hg, st, rng = _state(name, prec, 3)
    print("case: codec vs sweep", V.PREC_NAME[prec], name, axis, flush=True)
    n = tuple(hg.n)
    dt = 0.23
    g = None
    if axis in ("ux", "uy", "uz", "kick"):
        field = np.zeros((3,) + n, np.float32)
        for a in range(3):
            du = 2 * hg.umax[a] / hg.nu[a]
            field[a] = (rng.uniform(-2.6, 2.6, n) * du / dt).astype(np.float32)
        g = torch.from_numpy(field).cuda()
    f32 = V.State(hg, V.F32, V.decode(st))
    if axis == "kick":
        if hg.nu[0] != hg.nu[1] or hg.nu[1] != hg.nu[2]:
            pytest.skip("the fused kick keeps FP32 between its sweeps on cubic blocks only")
        scaled = V.kick(st, g, dt)
        plain = V.kick(f32, g, dt)
    else:
        scaled = V.advect(axis, st, dt, g=g)
        plain = V.advect(axis, f32, dt, g=g)
    enc = V.encode(hg, prec, plain.f)
    torch.cuda.synchronize()
    assert torch.equal(enc.scale, scaled.scale)
    assert torch.equal(enc.f.view(torch.int16), scaled.f.view(torch.int16))


@pytest.mark.parametrize("prec", [V.F16, V.BF16])
def test_codes_and_scales(prec):
    n, nu = GRIDS["nuz32"]
    hg = V.make_grid(n, nu)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2, V.grid_shape(hg)).astype(np.float32)
    x[1, 2, 3, 4, 5] = 0.0                             # all zero
    x[0, 1, 2, 3, 4] *= np.float32(1e-39)              # largest |value| below the normal range
    e = V.encode(hg, prec, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    sc = e.scale.cpu().numpy()
    assert np.array_equal(sc, np.abs(x).max(axis=-1))          # exact line maxima
    codes = e.f.float().cpu().numpy().astype(np.float64)
    assert sc[1, 2, 3, 4, 5] == 0.0 and np.all(codes[1, 2, 3, 4, 5] == 0.0)
    # a sub-normal line maximum has no finite FP32 reciprocal: stored as zeros
    assert np.all(codes[0, 1, 2, 3, 4] == 0.0)
    assert np.all(np.isfinite(codes))
    normal = sc >= np.float32(1.17549435e-38)
    q = np.zeros(x.shape)
    q[normal] = x[normal].astype(np.float64) / sc[normal][..., None].astype(np.float64)
    exact = torch.from_numpy(q).to(V.TORCH_DTYPE[prec]).double().numpy()   # RNE of the quotient
    # one code unit: 2^-10 (FP16) or 2^-7 (BF16) of the value's binade, and
    # FP16's sub-normal spacing 2^-24 below 2^-14
    rel = {V.F16: 2.0 ** -10, V.BF16: 2.0 ** -7}[prec]
    floor = {V.F16: 2.0 ** -14, V.BF16: 2.0 ** -126}[prec]
    assert np.all(np.abs(codes - exact) <= rel * np.maximum(np.abs(exact), floor))
    back = V.decode(e).cpu().numpy()
    assert np.array_equal(back, (e.f.float() * e.scale[..., None]).cpu().numpy())


def test_codec_errors():
    hg = V.make_grid((2, 2, 2), (4, 4, 8))
    f = torch.zeros(V.grid_shape(hg), device="cuda")
    c = torch.zeros(V.grid_shape(hg), dtype=torch.float16, device="cuda")
    s = torch.zeros(V.grid_shape(hg)[:-1], device="cuda")
    for fn, args, code in [
        (V.vlasov_encode, (hg, V.F16, None, c, s), -1),
        (V.vlasov_encode, (hg, V.F16, f, c, None), -3),
        (V.vlasov_encode, (hg, 7, f, c, s), -3),
        (V.vlasov_decode, (hg, V.BF16, c, None, f), -3),
        (V.vlasov_encode, (V.make_grid((2, 2, 2), (4, 4, 6)), V.F16, f, c, s), -2),
        (V.vlasov_encode, (hg, V.F16, f, f, s), -4),
    ]:
        with pytest.raises(V.VlasovError) as e:
            fn(*args)
        assert e.value.code == code
