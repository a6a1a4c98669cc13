"""Pins for the oracle's linear-form algebra (CPU only).

The relaxations are checked against what mathematics fixes: they must enclose the
true function on dense samples of random inputs, collapse to the exact value at zero
width, and match the closed forms of Table "Bounds for operations Exp, Div and Ind".
"""
import numpy as np
import pytest

from oracle import lf

RNG = np.random.default_rng(1234)


def random_lf(shape, P, scale=1.0, slack=0.1, offset=0.0):
    """An LF pair around a random affine function, with a random constant gap."""
    g = RNG.normal(0, scale, shape + (P,))
    h = RNG.normal(offset, scale, shape)
    w = RNG.uniform(0, slack, shape)
    lo = np.concatenate([g, (h - w)[..., None]], axis=-1)
    up = np.concatenate([g, (h + w)[..., None]], axis=-1)
    return lf.LF(lo, up), g, h, w


def true_values(g, h, w, e, t):
    """A true quantity inside the LF pair: affine part plus a point t in [-1,1] of the gap."""
    return g @ e + h + t * w


def check_enclosure(res, f, xs, es):
    for (e, vals) in zip(es, xs):
        lo, up = res.eval(e)
        fv = f(*vals)
        tol = 1e-9 * (1 + np.abs(fv))
        assert np.all(lo <= fv + tol), (lo - fv).max()
        assert np.all(fv <= up + tol), (fv - up).max()


@pytest.mark.parametrize("P", [0, 1, 3, 6])
def test_mul_sqr_exp_enclose(P):
    shape = (400,)
    x, gx, hx, wx = random_lf(shape, P)
    y, gy, hy, wy = random_lf(shape, P, offset=0.5)
    m = lf.mul(x, y)
    s = lf.sqr(x)
    xlo, xhi = x.bounds()
    ex = lf.exp(x, xlo, xhi)
    for _ in range(200):
        e = RNG.uniform(-1, 1, P)
        tx = RNG.uniform(-1, 1, shape)
        ty = RNG.uniform(-1, 1, shape)
        xv = true_values(gx, hx, wx, e, tx)
        yv = true_values(gy, hy, wy, e, ty)
        for res, fv in ((m, xv * yv), (s, xv * xv), (ex, np.exp(xv))):
            lo, up = res.eval(e)
            tol = 1e-9 * (1 + np.abs(fv))
            assert np.all(lo <= fv + tol)
            assert np.all(fv <= up + tol)


def test_zero_width_is_exact():
    x = lf.const(RNG.normal(0, 2, 50), 0)
    y = lf.const(RNG.normal(0, 2, 50), 0)
    xv = x.lo[:, 0]
    yv = y.lo[:, 0]
    np.testing.assert_allclose(lf.mul(x, y).lo[:, 0], xv * yv, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(lf.mul(x, y).up[:, 0], xv * yv, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(lf.sqr(x).lo[:, 0], xv * xv, rtol=1e-15)
    np.testing.assert_allclose(lf.sqr(x).up[:, 0], xv * xv, rtol=1e-15)
    e = lf.exp(x, xv, xv)
    np.testing.assert_allclose(e.lo[:, 0], np.exp(xv), rtol=1e-14)
    np.testing.assert_allclose(e.up[:, 0], np.exp(xv), rtol=1e-14)


def test_exp_matches_table_closed_form():
    """Table 'Bounds for operations Exp, Div and Ind', row Exp, on x = c + r e (P = 1)."""
    c, r = -1.3, 0.7
    x = lf.variable(c, r, 0, 1)
    xlo, xhi = c - r, c + r
    res = lf.exp(x, xlo, xhi)
    for e in np.linspace(-1, 1, 11):
        xv = c + r * e
        lo, up = res.eval([e])
        lo_table = np.exp(xlo) * (xv - xlo) + np.exp(xlo)
        up_table = (np.exp(xhi) - np.exp(xlo)) / (xhi - xlo) * (xv - xlo) + np.exp(xlo)
        assert lo == pytest.approx(lo_table, rel=1e-13)
        assert up == pytest.approx(up_table, rel=1e-13)


def test_mccormick_planes_textbook():
    """Mul of exact forms equals the McCormick planes (x - a)(y - c) >= 0 and (x - a)(d - y) >= 0."""
    x = lf.variable(0.3, 0.5, 0, 2)
    y = lf.variable(-0.2, 0.4, 1, 2)
    a, c, d = 0.3 - 0.5, -0.2 - 0.4, -0.2 + 0.4
    m = lf.mul(x, y)
    for e0 in np.linspace(-1, 1, 5):
        for e1 in np.linspace(-1, 1, 5):
            xv, yv = 0.3 + 0.5 * e0, -0.2 + 0.4 * e1
            lo, up = m.eval([e0, e1])
            assert lo == pytest.approx(c * xv + a * yv - a * c, abs=1e-14)
            assert up == pytest.approx(d * xv + a * yv - a * d, abs=1e-14)


@pytest.mark.parametrize("which,f", [("sin", np.sin), ("cos", np.cos)])
def test_trig_encloses(which, f):
    for c in np.linspace(-3.0, 3.0, 13):
        for r in (1e-4, 0.01, 0.3, 1.0):
            th = lf.variable(c, r, 0, 1)
            res = lf.trig(th, which)
            for e in np.linspace(-1, 1, 41):
                lo, up = res.eval([e])
                v = f(c + r * e)
                assert lo <= v + 1e-15 and v <= up + 1e-15
            # second-order tightness: the gap is M2 r^2 / 2 <= r^2 / 2
            assert (res.up[-1] - res.lo[-1]) <= r * r + 1e-15


def test_mmul_matches_matmul_for_exact_constants():
    a = RNG.normal(size=(3, 3))
    b = RNG.normal(size=(3, 3))
    A = lf.const(a, 2)
    B = lf.const(b, 2)
    np.testing.assert_allclose(lf.mmul(A, B).lo[..., -1], a @ b, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(lf.mmul_const_left(a, B).lo[..., -1], a @ b, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(lf.mmul_const_right(A, b).up[..., -1], a @ b, rtol=1e-14, atol=1e-14)
