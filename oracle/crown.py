"""Backward (CROWN-style) linear bounds for MatrixInv, FP64 (test infrastructure only).

The paper propagates its linear relations with CROWN (Sec. 2.1 and Sec. 4: linear bound
propagation), which works backward: a bound of an output is built by substituting, from
the output back to the inputs, each relaxed operation's upper or lower plane according
to the sign of the coefficient it carries, so every intermediate keeps its relaxation
symbolic until the end.  The forward mode of lf.py instead commits to one pair of forms
per intermediate.  This module builds Alg. MatrixInv's computation (IXX0 = I - X X0, the
powers IXX0^i by Mmul, Xp = X0 sum_i IXX0^i, then <Xp - Eps, Xp + Eps>) as a graph of
scalar nodes, each a batch of values, and bounds its outputs backward.

* Inputs are the entries of X, given as linear forms over the box e in [-1, 1]^P; X is
  symmetric and its two off-diagonal entries are one quantity (as X = Mp Mp^T in
  AbstractSplat), so there are three inputs.  An input is substituted by its upper
  (positive total coefficient) or lower (negative) form.
* Mul(a, b) is relaxed by the same McCormick planes as lf.mul: upper plane through
  (a_lo, b_hi), lower plane through (a_lo, b_lo), a the left operand.
* The intervals of the operands of every Mul are themselves computed backward before the
  Mul is relaxed (each intermediate is bounded by its own backward pass).
* Eps and the assertion use the interval of IXX0, which is linear in X and so exact.
"""
from __future__ import annotations

import numpy as np

from . import lf
from .matinv import inv2


class Graph:
    """Scalar computation graph over a batch; node ids are in topological order."""

    def __init__(self, P: int, batch):
        self.P = P
        self.batch = tuple(batch)
        self.nodes = []
        self.iv = []

    def _add(self, node, bound: bool):
        self.nodes.append(node)
        i = len(self.nodes) - 1
        self.iv.append(self.interval(i) if bound else None)
        return i

    def inp(self, x: lf.LF) -> int:
        """An input quantity given by its lower / upper forms (batch shape + (P+1,))."""
        return self._add(("in", x.lo, x.up), True)

    def lin(self, terms, const=0.0) -> int:
        """sum_k c_k node_k + const (exact)."""
        return self._add(("lin", terms, np.broadcast_to(np.asarray(const, dtype=np.float64), self.batch)), True)

    def mul(self, a: int, b: int) -> int:
        """Mul(a, b), relaxed by McCormick planes when a bound is substituted through it."""
        return self._add(("mul", a, b), False)

    def backward(self, t: int, sign: float) -> np.ndarray:
        """Linear form over e (batch + (P+1,)) that bounds sign * node_t from above."""
        w = {t: np.full(self.batch, float(sign))}
        form = np.zeros(self.batch + (self.P + 1,))
        for i in range(t, -1, -1):
            wi = w.pop(i, None)
            if wi is None:
                continue
            node = self.nodes[i]
            if node[0] == "in":
                form += np.where(wi[..., None] > 0, wi[..., None] * node[2], wi[..., None] * node[1])
            elif node[0] == "lin":
                for ch, c in node[1]:
                    w[ch] = w.get(ch, 0.0) + wi * c
                form[..., -1] += wi * node[2]
            else:
                a, b = node[1], node[2]
                alo, _ = self.iv[a]
                blo, bhi = self.iv[b]
                pos = wi > 0
                p = np.where(pos, bhi, blo)            # coefficient of a in the plane
                r = np.where(pos, -alo * bhi, -alo * blo)
                w[a] = w.get(a, 0.0) + wi * p
                w[b] = w.get(b, 0.0) + wi * alo
                form[..., -1] += wi * r
        return form

    def forms(self, t: int) -> lf.LF:
        """Lower and upper forms of node t over e."""
        return lf.LF(-self.backward(t, -1.0), self.backward(t, 1.0))

    def interval(self, t: int):
        return self.forms(t).bounds()


def matrix_inv_backward(X: lf.LF, k: int = 8):
    """MatrixInv(X; X0, k) of Sec. 3.1 bounded backward, for X of quantity shape (..., 2, 2).

    X0 is the inverse of the centre of X's interval hull, as in matinv.matrix_inv.  Returns
    (conic LF (..., 2, 2), ok mask, info) in the form of matinv.matrix_inv: ok is False where
    the centre is singular or the assertion ||IXX0|| < 1 fails, and those entries are zero.
    """
    batch = X.shape[:-2]
    P = X.P
    Xlo, Xhi = X.bounds()
    X0, det = inv2(0.5 * (Xlo + Xhi))
    ok = np.isfinite(det) & (det > 0)
    X0 = np.where(ok[..., None, None], X0, 0.0)
    if not (np.array_equal(X.lo[..., 0, 1, :], X.lo[..., 1, 0, :]) and np.array_equal(X.up[..., 0, 1, :],
                                                                                        X.up[..., 1, 0, :])):
        raise ValueError("matrix_inv_backward takes a symmetric X (one off-diagonal quantity)")
    g = Graph(P, batch)
    x00, x01, x11 = g.inp(X[..., 0, 0]), g.inp(X[..., 0, 1]), g.inp(X[..., 1, 1])
    x = [[x00, x01], [x01, x11]]
    # IXX0 = Add(I, -Mmul(X, X0))  (X0 constant: exact)
    E = [[g.lin([(x[i][0], -X0[..., 0, j]), (x[i][1], -X0[..., 1, j])], 1.0 if i == j else 0.0)
          for j in range(2)] for i in range(2)]
    terms = [[[(E[i][j], 1.0)] for j in range(2)] for i in range(2)]
    power = E
    for _ in range(2, k + 1):
        nxt = [[g.lin([(g.mul(power[i][0], E[0][j]), 1.0), (g.mul(power[i][1], E[1][j]), 1.0)])
                for j in range(2)] for i in range(2)]
        power = nxt
        for i in range(2):
            for j in range(2):
                terms[i][j].append((power[i][j], 1.0))
    S = [[g.lin(terms[i][j], 1.0 if i == j else 0.0) for j in range(2)] for i in range(2)]
    # Eps from the norm bound of IXX0 (exact intervals: IXX0 is linear in X)
    Eiv = np.stack([np.stack([np.stack(g.iv[E[i][j]], axis=-1) for j in range(2)], axis=-2) for i in range(2)],
                   axis=-3)
    nbar = np.sqrt(np.maximum(Eiv[..., 0] ** 2, Eiv[..., 1] ** 2).sum(axis=(-2, -1)))
    ok = ok & np.isfinite(nbar) & (nbar < 1.0)
    norm_x0 = np.sqrt((X0 * X0).sum(axis=(-2, -1)))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        eps = np.where(ok, norm_x0 * nbar ** (k + 1) / (1.0 - nbar), np.inf)
    lo = np.zeros(batch + (2, 2, P + 1))
    up = np.zeros(batch + (2, 2, P + 1))
    for i in range(2):
        for j in range(2):
            c = g.forms(g.lin([(S[0][j], X0[..., i, 0]), (S[1][j], X0[..., i, 1])]))
            lo[..., i, j, :] = c.lo
            up[..., i, j, :] = c.up
    lo[..., -1] -= np.where(ok, eps, 0.0)[..., None, None]
    up[..., -1] += np.where(ok, eps, 0.0)[..., None, None]
    lo = np.where(ok[..., None, None, None], lo, 0.0)
    up = np.where(ok[..., None, None, None], up, 0.0)
    return lf.LF(lo, up), ok, {"X0": X0, "nbar": nbar, "eps": eps, "det": det}
