"""Pins of the FP64 oracle's 1D scheme against what mathematics fixes.

The conservative semi-Lagrangian interface value, the Suresh-Huynh bounds and
the 1D update (section 5.2) are checked against an exact rational
construction, textbook values, closed forms, invariants and the measured
order of accuracy -- never against a retyped copy of the oracle's formulas.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- semi-Lagrangian weights ----------------------------------------------------

def _lagrange_primitive_weights(mu: Fraction):
    """Exact rational SL flux weights from first principles.

    The primitive W(x) of the reconstruction is known at the six interfaces
    x = -5/2 .. 5/2 (cell j on [-1/2, 1/2], unit width): W(-5/2) = 0 and each
    step adds one cell average.  The quintic through those points is the
    primitive of the quartic matching the five cell averages; the mass that
    crosses x = 1/2 during a shift by mu is W(1/2) - W(1/2 - mu).
    """
    xs = [Fraction(2 * k - 5, 2) for k in range(6)]

    def lag(x, i):
        p = Fraction(1)
        for k, xk in enumerate(xs):
            if k != i:
                p *= (x - xk) / (xs[i] - xk)
        return p

    out = []
    for cell in range(5):
        def dW(x):
            return sum(lag(x, m) for m in range(cell + 1, 6))
        out.append(dW(Fraction(1, 2)) - dW(Fraction(1, 2) - mu))
    return out


@pytest.mark.parametrize("mu", [Fraction(1, 7), Fraction(3, 10), Fraction(1, 2),
                                Fraction(17, 20), Fraction(99, 100)])
def test_sl5_weights_equal_exact_primitive_construction(mu):
    exact = _lagrange_primitive_weights(mu)
    w = oracle.sl5_weights(float(mu))
    for k in range(5):
        assert w[k] * float(mu) == pytest.approx(float(exact[k]), abs=1e-15)


def test_sl5_weights_small_shift_limit_is_fifth_order_upwind_value():
    with open(os.path.join(GOLDEN, "sl5_upwind_limit.txt")) as fh:
        rows = [l for l in fh if l.strip() and not l.startswith("#")]
    num = np.array([float(v) for v in rows[0].split()])
    np.testing.assert_allclose(oracle.sl5_weights(0.0), num / 60.0, rtol=0, atol=1e-15)


def test_sl5_whole_cell_shift_moves_exactly_the_upwind_cell():
    np.testing.assert_allclose(oracle.sl5_weights(1.0), [0, 0, 1, 0, 0], atol=1e-15)


def test_sl5_weights_partition_of_unity():
    for mu in np.linspace(0, 1, 23):
        assert oracle.sl5_weights(mu).sum() == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_sl5_exact_for_quartic_cell_averages(p):
    """Mean over the departure interval is exact for polynomials of degree <= 4."""
    for mu in (0.11, 0.5, 0.93):
        # cell averages of x^p over [k-1/2, k+1/2], k = -2..2
        avg = [((k + 0.5) ** (p + 1) - (k - 0.5) ** (p + 1)) / (p + 1) for k in range(-2, 3)]
        lo, hi = 0.5 - mu, 0.5
        exact_mean = (hi ** (p + 1) - lo ** (p + 1)) / (p + 1) / mu
        assert oracle.sl5_weights(mu) @ np.array(avg) == pytest.approx(exact_mean, abs=1e-13)


def test_sl5_matches_gauss_quadrature_of_the_reconstruction():
    """Brute force: fit the quartic to random cell averages, integrate with Gauss-Legendre."""
    rng = np.random.default_rng(7)
    xg, wg = np.polynomial.legendre.leggauss(6)
    for _ in range(20):
        avg = rng.uniform(0, 1, 5)
        # cell averages of monomials -> solve for the quartic's coefficients
        A = np.array([[((k + 0.5) ** (p + 1) - (k - 0.5) ** (p + 1)) / (p + 1) for p in range(5)]
                      for k in range(-2, 3)])
        coef = np.linalg.solve(A, avg)
        mu = rng.uniform(0.01, 0.99)
        lo, hi = 0.5 - mu, 0.5
        xq = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        mean = 0.5 * np.sum(wg * np.polyval(coef[::-1], xq))
        assert oracle.sl5_weights(mu) @ avg == pytest.approx(mean, abs=1e-12)


# --- Suresh-Huynh bounds ------------------------------------------------------------

def test_minmod4_and_median_definitions():
    assert oracle.minmod4(3, 1, 2, 5) == 1
    assert oracle.minmod4(-3, -1, -2, -5) == -1
    assert oracle.minmod4(3, -1, 2, 5) == 0
    assert oracle.minmod4(0, 1, 2, 5) == 0
    assert oracle.median3(1, 5, 3) == 3
    assert oracle.median3(5, 1, 3) == 3
    assert oracle.median3(3, 3, 1) == 3


def test_mp5_hand_stencils():
    with open(os.path.join(GOLDEN, "mp5_hand_stencils.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for r in rows:
        fhat, a, b, c, d, e, alpha, want = map(float, r)
        assert oracle.mp5_limit(fhat, a, b, c, d, e, alpha) == pytest.approx(want, abs=1e-15), r


def test_mp_alpha_is_the_single_stage_courant_bound():
    """alpha(mu) = (1-mu)/mu: mu (1 + alpha) = 1 exactly, 4 at mu = 0.2 (the
    Suresh-Huynh constant), 1 at half a cell; capped where the fraction is tiny."""
    assert oracle.mp_alpha(0.2) == pytest.approx(4.0, rel=1e-15)
    assert oracle.mp_alpha(0.5) == 1.0
    for mu in (1e-5, 0.013, 0.11, 0.3, 0.37, 0.49):
        assert mu * (1.0 + oracle.mp_alpha(mu)) == pytest.approx(1.0, rel=1e-14)
    assert oracle.mp_alpha(0.0) == 2.0 ** 20
    assert oracle.mp_alpha(1e-9) == 2.0 ** 20


@pytest.mark.parametrize("s,N", [(0.0, 0), (0.3, 0), (0.5, 1), (0.51, 1), (0.7, 1), (1.49, 1),
                                 (2.5, 3), (-0.3, 0), (-0.5, -1), (-0.7, -1), (-2.5, -3),
                                 (-3.2, -3), (33.1, 33), (0.49999999999999994, 0)])
def test_split_shift_nearest_integer(s, N):
    """Integer part = nearest integer (halves away from zero), fraction = the
    exact remainder, at most half a cell."""
    n, nu = oracle.split_shift(s)
    assert n == N
    assert n + nu == s
    assert abs(nu) <= 0.5


def _sh_early_out(fhat, a, b, c, d, e, alpha=4.0):
    """Suresh-Huynh's own two-stage procedure: keep fhat when it lies between
    f_j and the monotone bound f_MP = f_j + minmod(f_{j+1}-f_j, alpha(f_j-f_{j-1}));
    otherwise fall back to the oracle's bounded median."""
    x, y = d - c, alpha * (c - b)
    mm = 0.0 if x * y <= 0 else (x if abs(x) < abs(y) else y)
    fmp = c + mm
    if (fhat - c) * (fhat - fmp) <= 0:
        return fhat
    return None


@pytest.mark.parametrize("alpha", [1.0, 1.7, 4.0, 9.0])
def test_mp5_median_form_agrees_with_early_out_form(alpha):
    """With epsilon = 0 the early-out of Suresh & Huynh never changes the result:
    the interval [f_j, f_MP] lies inside the bounds (for any alpha >= 0)."""
    rng = np.random.default_rng(11)
    kept = 0
    for _ in range(20000):
        st = rng.uniform(0, 1, 5)
        if rng.random() < 0.5:
            st = np.sort(st) if rng.random() < 0.5 else np.sort(st)[::-1]
        fhat = rng.uniform(-0.2, 1.2)
        early = _sh_early_out(fhat, *st, alpha=alpha)
        lim = oracle.mp5_limit(fhat, *st, alpha)
        if early is not None:
            kept += 1
            assert lim == early
    assert kept > 500


# --- one line -----------------------------------------------------------------------

SHIFTS = [0.0, 0.37, -0.37, 0.9, -0.9, 1.0, -1.0, 2.37, -2.63, 3.0, 7.5, -9.25, 33.1]


@pytest.mark.parametrize("N", [-40, -7, -3, -1, 0, 1, 2, 3, 5, 16, 40])
def test_integer_shift_is_exact_translation(N):
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, 16)
    out, _ = oracle.sweep_line(f, float(N), periodic=True)
    assert np.array_equal(out, np.roll(f, N))
    out, ofl = oracle.sweep_line(f, float(N), periodic=False)
    want = np.zeros_like(f)
    for i in range(16):
        if 0 <= i - N < 16:
            want[i] = f[i - N]
    assert np.array_equal(out, want)
    assert ofl == pytest.approx(f.sum() - want.sum(), abs=1e-14)


@pytest.mark.parametrize("s", SHIFTS)
def test_uniform_line_unchanged_bitwise(s):
    f = np.full(24, 0.731)
    out, _ = oracle.sweep_line(f, s, periodic=True)
    assert np.array_equal(out, f)


@pytest.mark.parametrize("s", SHIFTS)
def test_conservation(s):
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 1, 32)
    out, _ = oracle.sweep_line(f, s, periodic=True)
    assert out.sum() == pytest.approx(f.sum(), rel=1e-14)
    out, ofl = oracle.sweep_line(f, s, periodic=False)
    assert out.sum() + ofl == pytest.approx(f.sum(), rel=1e-14)
    assert ofl >= 0.0


@pytest.mark.parametrize("s", SHIFTS)
def test_positivity(s):
    rng = np.random.default_rng(9)
    for trial in range(20):
        f = rng.uniform(0, 1, 29) ** 4
        f[rng.integers(0, 29, 8)] = 0.0     # zeros and sharp gradients
        for periodic in (True, False):
            out, _ = oracle.sweep_line(f, s, periodic=periodic)
            assert out.min() >= 0.0


@pytest.mark.parametrize("s", [0.31, -0.77, 2.45, -3.2])
def test_linear_data_translated_exactly_in_the_interior(s):
    M = 40
    f = 2.0 + 0.01 * np.arange(M)
    out, _ = oracle.sweep_line(f, s, periodic=False)
    inner = slice(8, M - 8)
    want = 2.0 + 0.01 * (np.arange(M) - s)
    np.testing.assert_allclose(out[inner], want[inner], rtol=0, atol=1e-13)


@pytest.mark.parametrize("s", [0.37, 0.9, 2.37, 5.5])
def test_mirror_symmetry(s):
    """A leftward shift of the mirrored line is the mirror of the rightward shift."""
    rng = np.random.default_rng(13)
    f = rng.uniform(0, 1, 27)
    for periodic in (True, False):
        a, oa = oracle.sweep_line(f, s, periodic=periodic)
        b, ob = oracle.sweep_line(f[::-1].copy(), -s, periodic=periodic)
        np.testing.assert_allclose(a, b[::-1], rtol=0, atol=1e-15)
        assert oa == pytest.approx(ob, abs=1e-14)


MP_SHIFTS = sorted(set([round(x, 4) for x in np.linspace(-3.2, 3.2, 65)]
                       + [0.5, -0.5, 0.499, 0.501, 0.7, 0.9, 0.99, -0.9, 1.5, 2.5, 0.01]))


@pytest.mark.parametrize("s", MP_SHIFTS)
def test_no_new_extrema_at_any_shift(s):
    """Section 5.2 calls SL-MPP5 monotonicity preserving: a square wave swept
    100 times, and monotone ramps between plateaus swept 5 times, gain no new
    maximum or minimum, whatever the shift (fraction and integer part).  (With
    the fixed alpha = 4 and fractions up to a whole cell the square wave gains
    1-3 % of its jump above a fraction of 0.2.)"""
    M = 64
    f = np.where((np.arange(M) > 16) & (np.arange(M) < 40), 1.0, 0.1)
    for _ in range(100):
        f, _ = oracle.sweep_line(f, s, periodic=True)
    assert f.max() <= 1.0 + 1e-14
    assert f.min() >= 0.1 - 1e-14
    rng = np.random.default_rng(21)
    for _ in range(20):
        ramp = np.sort(rng.uniform(0, 1, 20) ** rng.uniform(0.3, 3))
        g = np.concatenate([np.full(12, ramp[0]), ramp, np.full(12, ramp[-1]), ramp[::-1],
                            np.full(12, ramp[0])])
        lo, hi = g.min(), g.max()
        for _ in range(5):
            g, _ = oracle.sweep_line(g, s, periodic=True)
        assert g.max() <= hi + 1e-14 and g.min() >= lo - 1e-14


def _sin_cell_averages(n, shift_cells):
    """Exact cell averages of 1 + 0.5 sin(2 pi x) on [0,1), translated by shift."""
    x = np.arange(n + 1) / n - shift_cells / n
    prim = x - 0.5 / (2 * math.pi) * np.cos(2 * math.pi * x)
    return (prim[1:] - prim[:-1]) * n


@pytest.mark.parametrize("s", [0.37, 2.37, -1.71, 0.5, 0.9, -2.62])
@pytest.mark.parametrize("limiter", [True, False])
def test_fifth_order_convergence(s, limiter):
    """Section 5.1.1 / 5.2: the scheme is fifth-order accurate in space."""
    errs = []
    for n in (32, 64, 128, 256):
        f = _sin_cell_averages(n, 0.0)
        steps = n // 4
        for _ in range(steps):
            f, _ = oracle.sweep_line(f, s, periodic=True, limiter=limiter)
        errs.append(np.abs(f - _sin_cell_averages(n, steps * s)).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders[:2]) > 4.6, (errs, orders)
    assert abs(orders[1] - 5.0) < 0.2, (errs, orders)
