"""The kernels' operation-saving forms of the Suresh-Huynh bounds (CPU only).

The kernels evaluate two pieces of the bounds (section 5.2) in forms that
differ from their definitions by rounding only; the forms are restated here
in FP32 numpy and held against the definitions in FP64:

* the curvature minmod d^M4 = minmod(4Da - Db, 4Db - Da, Da, Db) as
  med3(m, 5m - (Da + Db), 0), m = minmod(Da, Db) (the candidate 4o - m, o
  the curvature of larger magnitude, never has the least magnitude): the
  same sign and value within one rounding of Da + Db, zero wherever the
  curvatures differ in sign, and symmetric bit for bit in Da and Db (a walk
  carries the minmod of one interface to the next with its arguments
  swapped);
* the median value f^MD = (f_j + f_{j+1} - d^M4) / 2 as
  f_j + (f_{j+1} - f_j) / 2 - d^M4 / 2.
"""
import numpy as np

F32 = np.float32


def med3(a, b, c):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), c))


def fma32(a, b, c):
    """a * b + c with one rounding to FP32 (exact in FP64 for these operands:
    b is a small integer or a half, so a * b has at most 27 significant bits,
    and the sum of it and c is exact as long as their exponents are within
    26 of each other, which the test data keep)."""
    return (np.float64(a) * np.float64(b) + np.float64(c)).astype(F32)


def curv_minmod_form(Da, Db):
    m = med3(Da, Db, F32(0))
    return med3(m, fma32(m, 5.0, -(Da + Db).astype(np.float64)), F32(0))


def curv_minmod_def(Da, Db):
    a, b = Da.astype(np.float64), Db.astype(np.float64)
    c = np.stack([4 * a - b, 4 * b - a, a, b])
    return np.where(np.all(c > 0, 0), c.min(0), np.where(np.all(c < 0, 0), c.max(0), 0.0))


def _pairs(n=400_000, seed=7):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-3, 3, (2, n))
    Da = (rng.standard_normal(n) * mag[0]).astype(F32)
    Db = (rng.standard_normal(n) * mag[1]).astype(F32)
    k = n // 8
    Db[:k] = Da[:k]                                  # equal curvatures
    Db[k:2 * k] = F32(4) * Da[k:2 * k]               # 4Da - Db = 0 exactly
    Db[2 * k:3 * k] = F32(3) * Da[2 * k:3 * k]       # 4Da - Db = Da
    Da[3 * k:4 * k] = 0                               # a zero curvature
    Db[4 * k:5 * k] = -Da[4 * k:5 * k]               # opposite signs
    return Da, Db


def test_curvature_minmod_form_matches_definition():
    Da, Db = _pairs()
    got = curv_minmod_form(Da, Db).astype(np.float64)
    want = curv_minmod_def(Da, Db)
    scale = np.maximum(np.abs(Da), np.abs(Db)).astype(np.float64)
    # within one rounding of Da + Db and one of the fma (|5m - s| <= 6 scale)
    assert np.all(np.abs(got - want) <= 8 * 2.0 ** -24 * scale)
    # exact where the curvature of least magnitude wins (no arithmetic)
    m = med3(Da, Db, F32(0)).astype(np.float64)
    assert np.all(got[want == m] == m[want == m])
    # zero wherever the curvatures do not share a strict sign
    mixed = (Da.astype(np.float64) * Db) <= 0
    assert np.all(got[mixed] == 0)
    # never the wrong sign
    assert np.all(got * want >= 0)


def test_curvature_minmod_form_is_symmetric():
    Da, Db = _pairs(seed=11)
    assert np.array_equal(curv_minmod_form(Da, Db).view(np.uint32),
                          curv_minmod_form(Db, Da).view(np.uint32))


def test_curvature_minmod_form_on_a_parabola_and_a_cubic():
    # equal curvatures (a parabola): d^M4 = D; a cubic with curvatures in the
    # ratio 1:2 gives min(D, 4D - 2D) = D; 1:5 gives 0 (4D - 5D < 0)
    D = np.array([0.25, -3.0, 1e-3], dtype=F32)
    assert np.array_equal(curv_minmod_form(D, D), D)
    assert np.array_equal(curv_minmod_form(D, F32(2) * D), D)
    assert np.all(curv_minmod_form(D, F32(5) * D) == 0)
    assert np.array_equal(curv_minmod_form(F32(3) * D, F32(2) * D), F32(2) * D)


def test_median_value_form():
    rng = np.random.default_rng(5)
    c = rng.uniform(0, 1, 100_000).astype(F32)
    d = rng.uniform(0, 1, 100_000).astype(F32)
    M = (rng.standard_normal(100_000) * 0.1).astype(F32)
    d0 = (d - c).astype(F32)
    got = fma32(M, -0.5, fma32(d0, 0.5, c).astype(np.float64)).astype(np.float64)
    want = 0.5 * (c.astype(np.float64) + d - M)
    assert np.all(np.abs(got - want) <= 3 * 2.0 ** -24 * np.maximum(1.0, np.abs(want)))
