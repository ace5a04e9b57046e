"""Pins of the oracle's velocity dispersion tensor (section 5.1.3) to closed
forms that do not go through the oracle's own formula:

* a sampled correlated Gaussian in velocity: by Poisson summation, the cell-
  centre sums of a Gaussian whose smallest standard deviation spans a few
  cells reproduce its mean and covariance up to exponentially small terms, so
  the tensor equals the covariance matrix (full, with distinct off-diagonal
  entries, so a transposed or mislabelled component fails);
* two occupied velocity cells: sigma = w_a w_b / (w_a + w_b)^2 d d^T with
  d = u_a - u_b;
* translation by whole cells of a compact blob leaves the tensor unchanged,
  scaling f leaves it unchanged, an empty cell gives zero, and the tensor of
  any non-negative block is symmetric positive semi-definite.
"""
import numpy as np
import pytest

import oracle

COMP = oracle.DISPERSION_COMPONENTS


def _tensor(sig6):
    t = np.empty((3, 3))
    for k, (a, b) in enumerate(COMP):
        t[a, b] = t[b, a] = sig6[k]
    return t


def _ucentres(umax, nu):
    return [-umax[a] + (np.arange(nu[a]) + 0.5) * 2 * umax[a] / nu[a] for a in range(3)]


def test_sampled_gaussian_gives_its_covariance():
    nu = (48, 40, 44)
    umax = (4.8, 4.0, 4.4)                      # du = 0.2 on every axis
    g = oracle.Grid.make((2, 1, 2), nu, (1.0, 1.0, 1.0), umax)
    rng = np.random.default_rng(5)
    ux, uy, uz = np.meshgrid(*_ucentres(umax, nu), indexing="ij")
    U = np.stack([ux, uy, uz], -1)
    f = np.zeros((2, 1, 2) + nu)
    want = {}
    for c, sd in [((0, 0, 0), (0.35, 0.45, 0.55)), ((1, 0, 1), (0.5, 0.4, 0.36)),
                  ((0, 0, 1), (0.4, 0.4, 0.4))]:
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        S = q @ np.diag(np.square(sd)) @ q.T
        u0 = rng.uniform(-0.3, 0.3, 3)
        d = U - u0
        e = np.einsum("...a,ab,...b->...", d, np.linalg.inv(S), d)
        f[c] = 3.7 * np.exp(-0.5 * e)
        want[c] = S
    sig = oracle.dispersion(g, f)
    for c, S in want.items():
        got = _tensor(sig[(slice(None),) + c])
        np.testing.assert_allclose(got, S, rtol=0, atol=1e-9)
    S = want[(0, 0, 0)]
    assert abs(S[0, 1] - S[0, 2]) > 1e-3 and abs(S[0, 1] - S[1, 2]) > 1e-3
    # the one empty cell
    assert np.all(sig[:, 1, 0, 0] == 0.0)


def test_two_occupied_cells():
    nu, umax = (6, 5, 7), (1.0, 2.0, 1.5)
    g = oracle.Grid.make((1, 1, 1), nu, (1.0, 1.0, 1.0), umax)
    uc = _ucentres(umax, nu)
    f = np.zeros((1, 1, 1) + nu)
    ja, jb, wa, wb = (1, 4, 2), (5, 0, 6), 0.3, 1.9
    f[(0, 0, 0) + ja] = wa
    f[(0, 0, 0) + jb] = wb
    d = np.array([uc[a][ja[a]] - uc[a][jb[a]] for a in range(3)])
    want = wa * wb / (wa + wb) ** 2 * np.outer(d, d)
    got = _tensor(oracle.dispersion(g, f)[:, 0, 0, 0])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)


def test_translation_scaling_and_psd():
    nu, umax = (16, 12, 20), (2.0, 1.5, 2.5)
    g = oracle.Grid.make((1, 1, 3), nu, (1.0, 1.0, 1.0), umax)
    rng = np.random.default_rng(6)
    blob = rng.uniform(0, 1, (5, 4, 6))
    f = np.zeros((1, 1, 3) + nu)
    f[0, 0, 0, 1:6, 2:6, 3:9] = blob
    f[0, 0, 1, 9:14, 7:11, 12:18] = 4.5 * blob
    f[0, 0, 2] = rng.uniform(0, 1, nu) ** 3
    sig = oracle.dispersion(g, f)
    np.testing.assert_allclose(sig[:, 0, 0, 1], sig[:, 0, 0, 0], rtol=1e-12, atol=1e-15)
    for c in range(3):
        t = _tensor(sig[:, 0, 0, c])
        assert np.linalg.eigvalsh(t).min() > -1e-14
    # a single occupied cell has no spread
    f1 = np.zeros((1, 1, 1) + nu)
    f1[0, 0, 0, 3, 4, 5] = 2.0
    g1 = oracle.Grid.make((1, 1, 1), nu, (1.0, 1.0, 1.0), umax)
    assert np.all(np.abs(oracle.dispersion(g1, f1)) < 1e-15)


def test_planted_mistake_is_caught():
    """A dispersion without the mean subtraction misses the Gaussian pin: the
    pins above would catch that mistake."""
    nu, umax = (32, 32, 32), (3.2, 3.2, 3.2)
    g = oracle.Grid.make((1, 1, 1), nu, (1.0, 1.0, 1.0), umax)
    ux, uy, uz = np.meshgrid(*_ucentres(umax, nu), indexing="ij")
    u0 = np.array([0.4, -0.3, 0.2])
    f = np.exp(-0.5 * ((ux - u0[0]) ** 2 + (uy - u0[1]) ** 2 + (uz - u0[2]) ** 2) / 0.16)
    raw = np.array([np.sum(a * b * f) / f.sum() for a, b in
                    [(ux, ux), (ux, uy), (ux, uz), (uy, uy), (uy, uz), (uz, uz)]])
    sig = oracle.dispersion(g, f[None, None, None])[:, 0, 0, 0]
    want = np.array([0.16, 0, 0, 0.16, 0, 0.16])
    assert np.abs(sig - want).max() < 1e-9
    assert np.abs(raw - want).max() > 1e-2
