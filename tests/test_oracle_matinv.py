"""Pins for the oracle's MatrixInv (Sec. 3.1): Lemma 'mat-inv', Example 1, the Sec. 4.5 conic."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import lf
from oracle.matinv import inv2, interval_matrix, matrix_inv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(7)


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def hull_of_inverse(lo, hi, n=81):
    """Brute-force interval hull of X^-1 over the symmetric interval matrix [lo, hi]."""
    a = np.linspace(lo[0][0], hi[0][0], n)
    b = np.linspace(lo[0][1], hi[0][1], n)
    c = np.linspace(lo[1][1], hi[1][1], n)
    A, Bm, C = np.meshgrid(a, b, c, indexing="ij")
    X = np.stack([np.stack([A, Bm], -1), np.stack([Bm, C], -1)], -2).reshape(-1, 2, 2)
    Xi, _ = inv2(X)
    return Xi.min(axis=0), Xi.max(axis=0)


def test_closed_form_inverse():
    X = RNG.normal(size=(100, 2, 2))
    Xi, det = inv2(X)
    np.testing.assert_allclose(Xi, np.linalg.inv(X), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(det, np.linalg.det(X), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("k", [1, 4, 8])
def test_lemma_encloses_inverse(k):
    """Lemma 'mat-inv': lXinv <= X^-1 <= uXinv for every X of the set, relationally in e."""
    for _ in range(30):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.5 * np.eye(2)
        rad = np.abs(RNG.normal(0, 0.05, (2, 2)))
        rad = 0.5 * (rad + rad.T)
        X = interval_matrix(M - rad, M + rad, symmetric=True)
        conic, ok, _ = matrix_inv(X, k)
        if not ok:
            continue
        for _ in range(50):
            e = RNG.uniform(-1, 1, 3)
            lo, up = conic.eval(e)
            Xe = 0.5 * (X.lo + X.up) @ np.concatenate([e, [1.0]])
            Xi = np.linalg.inv(Xe)
            assert np.all(lo <= Xi + 1e-12) and np.all(Xi <= up + 1e-12)


def test_zero_width_gives_the_inverse():
    for _ in range(20):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.1 * np.eye(2)
        X = lf.const(M, 0)
        conic, ok, info = matrix_inv(X, 8)
        assert ok
        cond = np.linalg.cond(M)
        np.testing.assert_allclose(conic.lo[..., 0], np.linalg.inv(M), atol=1e-12 * cond * np.abs(np.linalg.inv(M)).max())
        np.testing.assert_allclose(conic.up[..., 0], np.linalg.inv(M), atol=1e-12 * cond * np.abs(np.linalg.inv(M)).max())


def test_example1_hull_and_width():
    """Example 'matinv-vs-direct': exact hull width 0.66 (symmetric reading); ours encloses it
    and lies between the exact hull and the paper's adjugate width 1.22."""
    g = _load("example1_matinv.json")
    lo, hi = np.array(g["X_lo"]), np.array(g["X_hi"])
    hlo, hhi = hull_of_inverse(lo, hi)
    exact = np.linalg.norm(hhi - hlo)
    assert exact == pytest.approx(g["width_empirical_paper"], abs=0.005)
    X = interval_matrix(lo, hi, symmetric=True)
    conic, ok, _ = matrix_inv(X, 8)
    assert ok
    clo, chi = conic.bounds()
    assert np.all(clo <= hlo + 1e-12) and np.all(hhi <= chi + 1e-12)
    width = np.linalg.norm(chi - clo)
    assert exact <= width < g["width_adjugate_paper"]
    # soft: within 10 % of the paper's 0.70 (its bound engine is not reproduced)
    assert width == pytest.approx(g["width_matrixinv_paper"], rel=0.10)


def test_example1_printed_bounds_are_not_the_symmetric_hull():
    """The printed X_lo[0][1] = -0.2 with independent entries gives a hull far from 0.66,
    which is why the symmetric reading with -0.02 is taken."""
    g = _load("example1_matinv.json")
    lo, hi = np.array(g["X_lo_printed"]), np.array(g["X_hi_printed"])
    vals = []
    grids = [np.linspace(lo[i][j], hi[i][j], 21) for i in range(2) for j in range(2)]
    for a, b, c, d in itertools.product(*grids):
        vals.append(np.linalg.inv(np.array([[a, b], [c, d]])))
    vals = np.array(vals)
    width = np.linalg.norm(vals.max(axis=0) - vals.min(axis=0))
    assert abs(width - g["width_empirical_paper"]) > 0.1


def test_spiky_conic_encloses_hull():
    """Sec. 4.5 covariance bounds: MatrixInv encloses the exact inverse hull of the box."""
    g = _load("spiky_conic.json")
    lo, hi = np.array(g["cov_lo"]), np.array(g["cov_hi"])
    hlo, hhi = hull_of_inverse(lo, hi, n=61)
    X = interval_matrix(lo, hi, symmetric=True)
    conic, ok, info = matrix_inv(X, 8)
    assert ok and info["nbar"] < 1
    clo, chi = conic.bounds()
    assert np.all(clo <= hlo + 1e-9) and np.all(hhi <= chi + 1e-9)
    # the printed bounds are of the same magnitude (they come from a relational input)
    plo, phi = np.array(g["conic_lo_paper"]), np.array(g["conic_hi_paper"])
    assert np.all(np.sign(plo) == np.sign(clo)) and np.all(np.sign(phi) == np.sign(chi))


def test_assert_failure_reported():
    """A set too wide for the Neumann series (norm bound >= 1) is reported, not bounded."""
    X = interval_matrix(np.array([[0.1, -0.5], [-0.5, 0.1]]), np.array([[2.0, 0.5], [0.5, 2.0]]), symmetric=True)
    conic, ok, info = matrix_inv(X, 8)
    assert not ok and info["nbar"] >= 1
