"""Linear forms over a normalised pose box, and their relaxations (FP64, NumPy).

Test infrastructure only: nothing in the product path may import this module.

A quantity y that depends on the pose is represented, as in the paper's piecewise
linear relations (Sec. 2.1, definition of a piecewise linear relation), by a pair
of affine forms in the normalised pose variables e in [-1, 1]^P:

    lo[..., :P] . e + lo[..., P]  <=  y(e)  <=  up[..., :P] . e + up[..., P]

Every operation of Table "Operations" that the renderer uses is replaced by a
linear-relational operation (Sec. 3.3, item (2)).  The relaxations used for the
non-linear ones are:

* Mul, McCormick with one fixed plane pair (the paper does not say which planes
  its bound engine picks):  lower = ylo*x + xlo*y - xlo*ylo,
  upper = yhi*x + xlo*y - xlo*yhi.  The left operand of a product is x.
* Sqr, for a product of a quantity with itself: tangent at the point of the
  interval closest to zero (lower), chord (upper).
* Exp, as in Table "Bounds for operations Exp, Div and Ind": tangent at the
  interval's lower end (lower), chord (upper).
* sin / cos of an angle: first-order Taylor polynomial at the centre plus a
  Lagrange remainder (the paper perturbs Euler angles but does not say how the
  rotation entries are bounded).
"""
from __future__ import annotations

import numpy as np


class LF:
    """Lower and upper affine forms, arrays of shape (..., P+1); last entry = constant."""

    __slots__ = ("lo", "up")

    def __init__(self, lo, up):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.up = np.asarray(up, dtype=np.float64)
        assert self.lo.shape == self.up.shape

    # --- structure -----------------------------------------------------------------
    @property
    def P(self) -> int:
        return self.lo.shape[-1] - 1

    @property
    def shape(self):
        return self.lo.shape[:-1]

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        idx = idx + (slice(None),) * (self.lo.ndim - 1 - len(idx)) + (slice(None),)
        return LF(self.lo[idx], self.up[idx])

    def expand(self, axis):
        """Insert a broadcast axis (counted over the quantity axes, not the form axis)."""
        if axis < 0:
            axis = len(self.shape) + 1 + axis
        return LF(np.expand_dims(self.lo, axis), np.expand_dims(self.up, axis))

    def sum(self, axis):
        """Sum of quantities along a quantity axis (exact: forms add)."""
        if axis < 0:
            axis = len(self.shape) + axis
        return LF(self.lo.sum(axis=axis), self.up.sum(axis=axis))

    # --- concretisation over the box e in [-1,1]^P ---------------------------------
    def bounds(self):
        """Interval [min_e lo(e), max_e up(e)] (Sec. 2.1: linear set -> interval)."""
        lo = self.lo[..., -1] - np.abs(self.lo[..., :-1]).sum(axis=-1)
        hi = self.up[..., -1] + np.abs(self.up[..., :-1]).sum(axis=-1)
        return lo, hi

    def eval(self, e):
        """Value of both forms at a point e (shape (P,)) of the box."""
        e1 = np.concatenate([np.asarray(e, dtype=np.float64), [1.0]])
        return self.lo @ e1, self.up @ e1


# --- constructors -----------------------------------------------------------------------
def const(val, P):
    """A pose-independent quantity (a constant relation)."""
    val = np.asarray(val, dtype=np.float64)
    f = np.zeros(val.shape + (P + 1,))
    f[..., -1] = val
    return LF(f, f.copy())


def variable(centre, radius, index, P):
    """The pose parameter centre + radius * e[index]."""
    f = np.zeros(P + 1)
    f[index] = radius
    f[-1] = centre
    return LF(f, f.copy())


def extend(x: LF, extra: int) -> LF:
    """The same forms over extra further variables (zero coefficients), placed after the
    existing ones and before the constant."""
    if extra == 0:
        return x
    z = np.zeros(x.lo.shape[:-1] + (extra,))
    return LF(np.concatenate([x.lo[..., :-1], z, x.lo[..., -1:]], axis=-1),
              np.concatenate([x.up[..., :-1], z, x.up[..., -1:]], axis=-1))


def broadcast(x: LF, shape) -> LF:
    """Broadcast the quantity shape of x to `shape` (copies)."""
    shape = tuple(shape) + (x.lo.shape[-1],)
    return LF(np.broadcast_to(x.lo, shape).copy(), np.broadcast_to(x.up, shape).copy())


def stack(items, axis=0):
    """Stack LFs of equal shape into a new quantity axis."""
    if axis < 0:
        axis = len(items[0].shape) + 1 + axis
    return LF(np.stack([x.lo for x in items], axis=axis), np.stack([x.up for x in items], axis=axis))


# --- exact operations -------------------------------------------------------------------
def add(x: LF, y: LF) -> LF:
    """Add (Table "Operations"): the forms add."""
    return LF(x.lo + y.lo, x.up + y.up)


def neg(x: LF) -> LF:
    return LF(-x.up, -x.lo)


def sub(x: LF, y: LF) -> LF:
    return add(x, neg(y))


def add_const(x: LF, c) -> LF:
    c = np.asarray(c, dtype=np.float64)
    lo = x.lo.copy()
    up = x.up.copy()
    lo[..., -1] = lo[..., -1] + c
    up[..., -1] = up[..., -1] + c
    return LF(lo, up)


def _scale_lower(x: LF, c):
    """Lower form of c*x for a constant c: the lower form if c >= 0, else the upper one."""
    c = np.asarray(c, dtype=np.float64)[..., None]
    return np.where(c >= 0, c * x.lo, c * x.up)


def _scale_upper(x: LF, c):
    c = np.asarray(c, dtype=np.float64)[..., None]
    return np.where(c >= 0, c * x.up, c * x.lo)


def scale(x: LF, c) -> LF:
    """Multiplication by a constant (exact)."""
    return LF(_scale_lower(x, c), _scale_upper(x, c))


# --- relaxations ------------------------------------------------------------------------
def mul(x: LF, y: LF) -> LF:
    """Mul (Table "Operations") by the McCormick planes through (xlo, ylo) and (xlo, yhi).

    For x in [xlo, xhi], y in [ylo, yhi]:
      (x - xlo)(y - ylo) >= 0  gives  x*y >= ylo*x + xlo*y - xlo*ylo
      (x - xlo)(yhi - y) >= 0  gives  x*y <= yhi*x + xlo*y - xlo*yhi
    Each constant factor picks the lower or upper form of the operand it scales.
    """
    xlo, _ = x.bounds()
    ylo, yhi = y.bounds()
    lo = _scale_lower(x, ylo) + _scale_lower(y, xlo)
    up = _scale_upper(x, yhi) + _scale_upper(y, xlo)
    lo[..., -1] -= xlo * ylo
    up[..., -1] -= xlo * yhi
    return LF(lo, up)


def sqr(x: LF) -> LF:
    """x*x for one operand: tangent at clamp(0, xlo, xhi) below, chord above."""
    xlo, xhi = x.bounds()
    xs = np.clip(0.0, xlo, xhi)
    lo = _scale_lower(x, 2.0 * xs)
    up = _scale_upper(x, xlo + xhi)
    lo[..., -1] -= xs * xs
    up[..., -1] -= xlo * xhi
    return LF(lo, up)


def exp_slope(xlo, xhi):
    """Slope (exp(xhi) - exp(xlo)) / (xhi - xlo) of the chord of exp over [xlo, xhi]:
    exp(xlo) expm1(dx) / dx for short intervals (no cancellation), the plain
    difference quotient for long ones (no overflow), exp(xlo) at zero width."""
    xlo = np.asarray(xlo, dtype=np.float64)
    xhi = np.asarray(xhi, dtype=np.float64)
    dx = xhi - xlo
    with np.errstate(invalid="ignore", divide="ignore", over="ignore", under="ignore"):
        safe = np.where(dx > 0, dx, 1.0)
        short = np.exp(xlo) * np.expm1(np.minimum(dx, 1.0)) / np.where(dx > 0, np.minimum(dx, 1.0), 1.0)
        long_ = (np.exp(xhi) - np.exp(xlo)) / safe
        k = np.where(dx <= 0, np.exp(xlo), np.where(dx < 1.0, short, long_))
    return k


def exp(x: LF, xlo, xhi) -> LF:
    """Exp (Table "Bounds for operations Exp, Div and Ind") on an input known to lie in [xlo, xhi].

    lower: exp(xlo) * (x - xlo) + exp(xlo)      (tangent at the lower end)
    upper: k * (x - xlo) + exp(xlo), k = chord slope over [xlo, xhi]
    """
    exlo = np.exp(xlo)
    k = exp_slope(xlo, xhi)
    lo = _scale_lower(x, exlo)
    up = _scale_upper(x, k)
    lo[..., -1] += exlo * (1.0 - xlo)
    up[..., -1] += exlo - k * xlo
    return LF(lo, up)


def recip(x: LF, tangent: str = "lo") -> LF:
    """Div (Table "Bounds for operations Exp, Div and Ind"): 1/x for x in [xlo, xhi], xlo > 0.

    1/x is convex there, so any tangent lies below and the chord above:
      lower: -(x - t)/t^2 + 1/t, tangent at t = xlo as the table prints it (tangent="lo"),
             or at t = xhi (tangent="hi", an alternative the table does not give);
      upper: -(x - xlo)/(xlo xhi) + 1/xlo (the chord).
    Entries with xlo <= 0 are not bounded: their forms are NaN (callers check).
    """
    xlo, xhi = x.bounds()
    with np.errstate(divide="ignore", invalid="ignore"):
        t = xlo if tangent == "lo" else xhi
        ok = xlo > 0
        t = np.where(ok, t, np.nan)
        lo = _scale_lower(x, -1.0 / (t * t))
        up = _scale_upper(x, -1.0 / (np.where(ok, xlo, np.nan) * xhi))
        lo[..., -1] += 2.0 / t
        up[..., -1] += 1.0 / xlo + 1.0 / xhi
    return LF(lo, up)


def trig(theta: LF, which: str) -> LF:
    """sin or cos of an angle theta = c + sum_k r_k e_k that is exactly affine in e.

    f(theta) = f(c) + f'(c)(theta - c) + f''(xi)(theta - c)^2 / 2, and
    |f''| = |f| <= min(1, |f(c)| + rad) on [c - rad, c + rad] (|f'| <= 1).
    """
    assert np.array_equal(theta.lo, theta.up), "angle must be an exact affine form"
    c = theta.lo[..., -1]
    g = theta.lo[..., :-1]
    rad = np.abs(g).sum(axis=-1)
    if which == "sin":
        f0, f1 = np.sin(c), np.cos(c)
    elif which == "cos":
        f0, f1 = np.cos(c), -np.sin(c)
    else:
        raise ValueError(which)
    m2 = np.minimum(1.0, np.abs(f0) + rad)
    rem = 0.5 * m2 * rad * rad
    base = np.concatenate([f1[..., None] * g, f0[..., None]], axis=-1)
    lo = base.copy()
    up = base.copy()
    lo[..., -1] -= rem
    up[..., -1] += rem
    return LF(lo, up)


def mmul(a: LF, b: LF) -> LF:
    """Mmul: (a @ b)_ij = sum_t Mul(a_it, b_tj) over matrices of LFs (last two quantity axes)."""
    prod = mul(a.expand(-1), b.expand(-3))  # (..., i, t, j)
    return prod.sum(axis=-2)


def mmul_const_left(c, b: LF) -> LF:
    """c @ b for a constant matrix c: exact scaling and summation."""
    c = np.asarray(c, dtype=np.float64)
    return scale(b.expand(-3), c[..., :, :, None]).sum(axis=-2)


def mmul_const_right(a: LF, c) -> LF:
    """a @ c for a constant matrix c: exact scaling and summation."""
    c = np.asarray(c, dtype=np.float64)
    return scale(a.expand(-1), c[..., None, :, :]).sum(axis=-2)
