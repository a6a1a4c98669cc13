"""MatrixInv of the paper (Sec. 3.1, Alg. MatrixInv) on 2x2 linear forms, FP64.

Test infrastructure only.

For a set of matrices X and a fixed reference X0 (the inverse of the centre of X's
interval hull, Sec. 3.1 adjustment (1) and the footnote of Sec. 3.3):

    IXX0 = I - X X0                                   (exact: X0 is a constant)
    Xp   = sum_{i=0..k} X0 IXX0^i                     (powers by repeated Mmul)
    Eps  = ||X0|| * n^(k+1) / (1 - n),  n >= ||IXX0|| (Frobenius norm bound)
    <lXinv, uXinv> = <Xp - Eps, Xp + Eps>

The assertion ||IXX0|| < 1 is checked on the norm bound n.  When it fails (or the
centre matrix is not positive definite) the Gaussian is reported as a fallback; the
paper instead splits the input set, which this oracle does not do.
"""
from __future__ import annotations

import numpy as np

from . import lf


def inv2(M):
    """Closed-form inverse of 2x2 matrices (adjugate over determinant); returns (inv, det)."""
    M = np.asarray(M, dtype=np.float64)
    det = M[..., 0, 0] * M[..., 1, 1] - M[..., 0, 1] * M[..., 1, 0]
    adj = np.empty_like(M)
    adj[..., 0, 0] = M[..., 1, 1]
    adj[..., 1, 1] = M[..., 0, 0]
    adj[..., 0, 1] = -M[..., 0, 1]
    adj[..., 1, 0] = -M[..., 1, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = adj / det[..., None, None]
    return inv, det


def matrix_inv(X: lf.LF, k: int = 8):
    """MatrixInv(X; X0, k) for X of quantity shape (..., 2, 2).

    Returns (conic LF, ok mask, info dict with X0, nbar, eps).
    """
    Xlo, Xhi = X.bounds()
    M = 0.5 * (Xlo + Xhi)
    X0, det = inv2(M)
    ok = np.isfinite(det) & (det > 0)
    X0 = np.where(ok[..., None, None], X0, 0.0)
    P = X.P
    eye = np.broadcast_to(np.eye(2), X.shape)
    # IXX0 = Add(I, -Mmul(X, X0))
    E = lf.add_const(lf.neg(lf.mmul_const_right(X, X0)), eye)
    # sum_{i=0..k} IXX0^i, with IXX0^i = Mmul(IXX0^(i-1), IXX0)
    S = lf.add_const(lf.const(np.zeros(X.shape), P), eye)
    power = None
    for i in range(1, k + 1):
        power = E if i == 1 else lf.mmul(power, E)
        S = lf.add(S, power)
    Xp = lf.mmul_const_left(X0, S)
    Elo, Ehi = E.bounds()
    nbar = np.sqrt(np.maximum(Elo * Elo, Ehi * Ehi).sum(axis=(-2, -1)))
    ok = ok & np.isfinite(nbar) & (nbar < 1.0)
    norm_x0 = np.sqrt((X0 * X0).sum(axis=(-2, -1)))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        eps = np.where(ok, norm_x0 * nbar ** (k + 1) / (1.0 - nbar), np.inf)
    lo = Xp.lo.copy()
    up = Xp.up.copy()
    lo[..., -1] -= np.where(ok, eps, 0.0)[..., None, None]
    up[..., -1] += np.where(ok, eps, 0.0)[..., None, None]
    # where the assertion fails the bounds are meaningless; zero them (callers check ok)
    lo = np.where(ok[..., None, None, None], lo, 0.0)
    up = np.where(ok[..., None, None, None], up, 0.0)
    return lf.LF(lo, up), ok, {"X0": X0, "nbar": nbar, "eps": eps, "det": det}


def adjugate_inv(X: lf.LF, tangent: str = "lo"):
    """The direct inverse of a 2x2 set of matrices that Example 'matinv-vs-direct' of
    Sec. 3.1 compares MatrixInv with: adj(X) times Div(det X), every step a
    linear-relational operation (det = Mul(X00, X11) - Mul(X01, X10); Div as in Table
    "Bounds for operations Exp, Div and Ind"; the four entries Mul(adj_ij, 1/det)).

    Returns (LF of quantity shape (..., 2, 2), ok mask): ok is False where the determinant
    is not provably positive (Div needs x > 0), and those entries are zero.
    """
    det = lf.sub(lf.mul(X[..., 0, 0], X[..., 1, 1]), lf.mul(X[..., 0, 1], X[..., 1, 0]))
    rdet = lf.recip(det, tangent)
    dlo, _ = det.bounds()
    ok = dlo > 0
    adj = lf.stack([lf.stack([X[..., 1, 1], lf.neg(X[..., 0, 1])], axis=-1),
                    lf.stack([lf.neg(X[..., 1, 0]), X[..., 0, 0]], axis=-1)], axis=-2)
    r = lf.LF(np.where(ok[..., None], rdet.lo, 0.0), np.where(ok[..., None], rdet.up, 0.0))
    out = lf.mul(adj, lf.broadcast(r.expand(-1).expand(-1), adj.shape))
    okm = ok[..., None, None, None]
    return lf.LF(np.where(okm, out.lo, 0.0), np.where(okm, out.up, 0.0)), ok


def interval_matrix(lo, hi, symmetric=False):
    """A constant interval matrix as linear forms: every free entry is its own variable.

    With symmetric=True the (0,1) and (1,0) entries share one variable (and must
    carry equal bounds).
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    cen = 0.5 * (lo + hi)
    rad = 0.5 * (hi - lo)
    slots = [(0, 0), (0, 1), (1, 1)] if symmetric else [(0, 0), (0, 1), (1, 0), (1, 1)]
    P = len(slots)
    f = np.zeros((2, 2, P + 1))
    f[..., -1] = cen
    for v, (i, j) in enumerate(slots):
        f[i, j, v] = rad[i, j]
        if symmetric and i != j:
            f[j, i, v] = rad[i, j]
    return lf.LF(f, f.copy())
