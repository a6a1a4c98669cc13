"""AbstractSplat in FP64: lower/upper images over a box of camera poses (test infrastructure only).

This is the oracle that the HIP path is checked against.  It follows Sec. 3.3
(AbstractSplat): every input and intermediate of Alg. GaussianSplat becomes a
pair of linear forms over the normalised pose box, every operation becomes its
linear-relational counterpart (lf.py), the Conic inverse of Step 3 becomes MatrixInv
(matinv.py) and the Step 4 blend becomes BlendInd with interval transmittances.

Readings where the paper is silent (each one is also listed in the design notes):
* uc = Mmul(A, Add(uw, -tau)) + beta, see pose.py;
* pixel coordinates are centred on the principal point (render.py);
* products of a quantity with itself (d*d, the diagonal of Mp Mp^T, q q^T) use Sqr;
  the off-diagonal of Mp Mp^T is one quantity Mul(Mp_0m, Mp_1m) used twice;
* the q step (Step 3) is evaluated as v * (Conic * Mp) with v = u d^2 - d up: B = Conic * Mp is
  formed once per Gaussian;
* the a step (Step 3): x = -q q^T / 2 lies in [-s_hi/2, -max(0, s_lo)/2]; a = o * Exp(x) and its
  interval is [o exp(x_lo), o exp(x_hi)];
* Ind(d_i - d_j) (Alg. BlendInd) is decided on two bounds of d_i - d_j: the identity
  d_i - d_j = A_z (uw_i - uw_j) behind the depth d = uc_z (tau and beta cancel), and the literal
  difference of the depth forms with a 1e-10 margin: 1 if a lower bound proves it
  positive, 0 if an upper bound proves it non-positive, unknown otherwise;
* transmittances are interval products (the T step of BlendInd):
      T_hi[i] = prod_{Ind_ij = 1} (1 - a_lo[j]),  T_lo[i] = prod_{Ind_ij != 0} (1 - a_hi[j]);
* colour (the pc step of BlendInd, then item (5) of Sec. 3.3):
      lo = max(min_e sum_i c_i T_lo[i] a_i^lower(e), sum_i c_i T_lo[i] a_lo[i]) - E
      hi = min(max_e sum_i c_i T_hi[i] a_i^upper(e), sum_i c_i T_hi[i] a_hi[i]) + E
  clamped to [0, 1];
* near plane: d_hi <= z_near drops the Gaussian (the concrete renderer gives it
  a = 0); d_lo <= z_near < d_hi gives a in [0, o] at every pixel;
* MatrixInv assertion failure: a in [0, o exp(-dist^2 / (2 lam))] (the footprint bound);
* sets of scenes (Sec. 4.6, see scene_set): colours and opacities given as per-Gaussian
  intervals enter the pc step as c_lo in the lower and c_hi in the upper sums (pc does not
  decrease in any colour, since T and a are non-negative) and the a step as o_lo for the
  lower and o for the upper alpha; means moved along a direction by a scene variable
  become linear forms in that variable, an extra variable after the pose variables;
* per-pixel pruning: Gaussian i is removed from pixel u when o_i exp(-dist(u, mu_box)^2
  / (2 lam_i)) < eps with eps = cull_budget / N, decided in float32 on float32 inputs
  rounded outward; removing Gaussians whose alpha is at most eps moves any concrete
  pixel colour by at most the sum of those alphas, so E = cull_budget (1 + 2^-10).
"""
from __future__ import annotations

import numpy as np

from . import lf
from .crown import matrix_inv_backward
from .matinv import adjugate_inv, matrix_inv
from . import pose
from .pose import pose_forms

DEFAULTS = {"taylor_k": 8, "z_near": 0.01, "cull_budget": 1e-7, "tile": 16,
            # precision baselines of Sec. 3.1 / 3.2 (Examples 'matinv-vs-direct' and '3g-scene'):
            # "inverse": "matrixinv" | "matrixinv_backward" | "adjugate";
            # "blend": "ind" | "ind_interval" | "sort"
            "inverse": "matrixinv", "blend": "ind"}


def _f32_down(x):
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    return np.where(f.astype(np.float64) > x, np.nextafter(f, np.float32(-np.inf)), f).astype(np.float32)


def _f32_up(x):
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    return np.where(f.astype(np.float64) < x, np.nextafter(f, np.float32(np.inf)), f).astype(np.float32)


def options(opts=None):
    o = dict(DEFAULTS)
    if opts:
        o.update({k: v for k, v in opts.items() if v is not None})
    return o


def scene_set(scene):
    """The set of scenes a scene dict stands for (Sec. 4.6, sets of colours, means and opacities).

    Optional keys beside the plain scene's:
      "rgb_hi" (n, 3)      colour upper bounds ("rgb" is then the lower bound);
      "opacity_lo" (n,)    opacity lower bounds ("opacity" is then the upper bound);
      "set_lo", "set_hi"   bounds of the scene variables s_0 .. s_{k-1};
      "mean_var" (n,)      the variable that moves Gaussian i's mean (-1: none) and
      "mean_dir" (n, 3)    its direction: uw_i(s) = uw_i + mean_dir_i s_{mean_var[i]}.
    Returns (rgb_lo, rgb_hi, o_lo, o_hi, nvar, centre, radius, mean_var, mean_dir).
    """
    rgb = np.asarray(scene["rgb"], dtype=np.float64)
    o = np.asarray(scene["opacity"], dtype=np.float64)
    rgb_hi = np.asarray(scene.get("rgb_hi", rgb), dtype=np.float64)
    o_lo = np.asarray(scene.get("opacity_lo", o), dtype=np.float64)
    lo = np.asarray(scene.get("set_lo", []), dtype=np.float64).reshape(-1)
    hi = np.asarray(scene.get("set_hi", []), dtype=np.float64).reshape(-1)
    n = len(o)
    mvar = np.asarray(scene.get("mean_var", np.full(n, -1)), dtype=np.int64)
    mdir = np.asarray(scene.get("mean_dir", np.zeros((n, 3))), dtype=np.float64)
    return rgb, rgb_hi, o_lo, o, len(lo), 0.5 * (lo + hi), 0.5 * (hi - lo), mvar, mdir


def gaussian_forms(scene, intr, box, opts=None):
    """Per-Gaussian part of AbstractSplat (Alg. GaussianSplat, Steps 1-2 and the Conic of Step 3, plus Conic*Mp).

    A set of scenes (scene_set) adds its variables after the pose variables: the forms are
    over e in [-1, 1]^(P_pose + k), and a moved mean uw_i + mean_dir_i s is the linear form
    uw_i + mean_dir_i (centre + radius e_(P_pose + v)) in Step 1 (Sec. 4.6).
    """
    opts = options(opts)
    A, tau, beta, Pp = pose_forms(box)
    uw = np.asarray(scene["mean"], dtype=np.float64)
    Mw = np.asarray(scene["cov_factor"], dtype=np.float64)
    rgb_lo, rgb_hi, o_lo, o, nvar, s_cen, s_rad, mvar, mdir = scene_set(scene)
    N = len(uw)
    fx, fy = float(intr["fx"]), float(intr["fy"])
    P = Pp + nvar
    moving = mvar >= 0

    # Step 1, camera coordinates: uc = Mmul(A, Add(uw, -tau)) + beta
    if nvar == 0:
        y = lf.add_const(lf.neg(lf.broadcast(tau, (N, 3))), uw)
    else:
        A, tau, beta = lf.extend(A, nvar), lf.extend(tau, nvar), lf.extend(beta, nvar)
        uwf = lf.const(uw, P)
        for v in range(nvar):
            rows = mvar == v
            for f in (uwf.lo, uwf.up):
                f[rows, :, Pp + v] = mdir[rows] * s_rad[v]
                f[rows, :, -1] = uw[rows] + mdir[rows] * s_cen[v]
        y = lf.add(uwf, lf.neg(lf.broadcast(tau, (N, 3))))
    uc = lf.mmul(A, y.expand(-1))[:, :, 0]
    uc = lf.add(uc, lf.broadcast(beta, (N, 3)))
    # Step 1, camera covariance factor: Mc = Mmul(A, Mw), Mw constant
    Mc = lf.mmul_const_right(A, Mw)
    x, yy, z = uc[:, 0], uc[:, 1], uc[:, 2]
    # Step 2, projection Jacobian J (zero entries omitted: Mul with a zero constant is exactly zero)
    J00 = lf.scale(z, fx)
    J02 = lf.scale(x, -fx)
    J11 = lf.scale(z, fy)
    J12 = lf.scale(yy, -fy)
    # Step 2, pixel mean up with the principal point removed
    up0 = lf.scale(x, fx)
    up1 = lf.scale(yy, fy)
    # Step 2, pixel covariance factor: Mp = Mmul(J, Mc)
    Mp0 = lf.add(lf.mul(J00.expand(-1), Mc[:, 0, :]), lf.mul(J02.expand(-1), Mc[:, 2, :]))
    Mp1 = lf.add(lf.mul(J11.expand(-1), Mc[:, 1, :]), lf.mul(J12.expand(-1), Mc[:, 2, :]))
    Mp = lf.stack([Mp0, Mp1], axis=1)
    # Step 2, depth d = uc_z
    d = z
    # factors of the q step (Step 3): d*d and d*up
    D2 = lf.sqr(d)
    DUP0 = lf.mul(d, up0)
    DUP1 = lf.mul(d, up1)
    # Step 3, Conic: X = Mmul(Mp, Mp^T), Conic = MatrixInv(X; inverse of centre, k)
    X00 = lf.sqr(Mp0).sum(-1)
    X11 = lf.sqr(Mp1).sum(-1)
    X01 = lf.mul(Mp0, Mp1).sum(-1)
    X = lf.stack([lf.stack([X00, X01], axis=1), lf.stack([X01, X11], axis=1)], axis=1)
    if opts["inverse"] == "adjugate":
        # the direct inverse Example 'matinv-vs-direct' compares with (a failed Div, where the
        # determinant is not provably positive, is treated as a MatrixInv failure)
        conic, inv_ok = adjugate_inv(X)
        inv_info = {}
    elif opts["inverse"] == "matrixinv_backward":
        # MatrixInv with its linear bounds propagated backward (CROWN-style, crown.py)
        conic, inv_ok, inv_info = matrix_inv_backward(X, int(opts["taylor_k"]))
    else:
        conic, inv_ok, inv_info = matrix_inv(X, int(opts["taylor_k"]))
    # B = Mmul(Conic, Mp), hoisted out of the pixel loop
    B = lf.mmul(conic, Mp)

    # near plane
    z_near = float(opts["z_near"])
    dlo, dhi = d.bounds()
    dropped = dhi <= z_near
    straddle = (~dropped) & (dlo <= z_near)

    # footprint bound for pruning: mu = up / d over the box, lam >= lambda_max(X) / d^4
    u0lo, u0hi = up0.bounds()
    u1lo, u1hi = up1.bounds()
    Xlo, Xhi = X.bounds()
    eps_cull = float(opts["cull_budget"]) / max(N, 1)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        dl = np.where(dlo > 0, dlo, np.nan)
        m0lo = np.minimum(u0lo / dl, u0lo / dhi)
        m0hi = np.maximum(u0hi / dl, u0hi / dhi)
        m1lo = np.minimum(u1lo / dl, u1lo / dhi)
        m1hi = np.maximum(u1hi / dl, u1hi / dhi)
        a_lo, a_hi = Xlo[:, 0, 0], Xhi[:, 0, 0]
        c_lo, c_hi = Xlo[:, 1, 1], Xhi[:, 1, 1]
        b_lo, b_hi = Xlo[:, 0, 1], Xhi[:, 0, 1]
        lam_x = 0.5 * (a_hi + c_hi) + np.sqrt(
            0.25 * np.maximum((a_hi - c_lo) ** 2, (c_hi - a_lo) ** 2) + np.maximum(b_lo ** 2, b_hi ** 2))
        lam = lam_x / dl ** 4
        r2 = np.where(o > eps_cull, 2.0 * lam * np.log(o / eps_cull), -1.0)
    geo_ok = np.isfinite(m0lo) & np.isfinite(m0hi) & np.isfinite(m1lo) & np.isfinite(m1hi) \
        & np.isfinite(lam) & np.isfinite(r2) & (lam > 0)
    normal = (~dropped) & (~straddle) & geo_ok
    # anything not dropped whose footprint cannot be bounded is treated like a straddler
    wild = (~dropped) & (~normal)
    fallback = normal & (~inv_ok)
    mu32 = np.stack([_f32_down(np.where(normal, m0lo, 0.0)), _f32_up(np.where(normal, m0hi, 0.0)),
                     _f32_down(np.where(normal, m1lo, 0.0)), _f32_up(np.where(normal, m1hi, 0.0))], axis=1)
    r2_32 = _f32_up(np.where(normal, r2, -1.0))
    mu64 = np.stack([m0lo, m0hi, m1lo, m1hi], axis=1)

    return {
        "P": P, "N": N, "A": A, "uc": uc, "d": d, "Mp": Mp, "X": X, "conic": conic, "B": B,
        "D2": D2, "DUP": lf.stack([DUP0, DUP1], axis=1), "up": lf.stack([up0, up1], axis=1),
        "o": o, "o_lo": o_lo, "rgb": rgb_lo, "rgb_hi": rgb_hi, "uw": uw, "moving": moving,
        "dropped": dropped, "straddle": straddle, "wild": wild, "normal": normal,
        "fallback": fallback, "inv_ok": inv_ok, "inv_info": inv_info,
        "lam": np.where(normal, lam, np.inf), "mu32": mu32, "r2_32": r2_32, "mu64": mu64,
        "eps_cull": eps_cull, "E": float(opts["cull_budget"]) * (1.0 + 2.0 ** -10),
        "opts": opts,
    }


def pixel_coords32(intr, cols, rows):
    """Centred pixel-centre coordinates as float32 (the values both sides use)."""
    ux = (np.asarray(cols, dtype=np.float64) + 0.5 - float(intr["cx"])).astype(np.float32)
    uy = (np.asarray(rows, dtype=np.float64) + 0.5 - float(intr["cy"])).astype(np.float32)
    return ux, uy


def _dist2_f32(mu32, ux, uy):
    """Squared distance from pixel centres to the mean box, in float32 (pruning decision).

    dx = max(max(mu_x_lo - u, 0), u - mu_x_hi) and likewise dy; dist2 = dx*dx + dy*dy,
    every operation rounded to float32 (no fused multiply-add).
    """
    zero = np.float32(0.0)
    dx = np.maximum(np.maximum(mu32[:, None, 0] - ux[None, :], zero), ux[None, :] - mu32[:, None, 1])
    dy = np.maximum(np.maximum(mu32[:, None, 2] - uy[None, :], zero), uy[None, :] - mu32[:, None, 3])
    return (dx * dx + dy * dy).astype(np.float32)


def kept_mask(rec, idx, ux32, uy32):
    """Gaussians idx that are not pruned at pixels (ux32, uy32): bool (len(idx), n_pix)."""
    d2 = _dist2_f32(rec["mu32"][idx], ux32, uy32)
    keep = rec["normal"][idx][:, None] & (d2 <= rec["r2_32"][idx][:, None])
    return keep | rec["wild"][idx][:, None]


def tile_candidates(rec, intr, x0, x1, y0, y1):
    """Gaussians whose pruning test passes somewhere in the pixel rectangle [x0,x1) x [y0,y1).

    The same float32 test on the rectangle of pixel centres; by monotonicity of
    rounding it keeps every Gaussian that any pixel of the rectangle keeps.
    """
    ux32, uy32 = pixel_coords32(intr, [x0, x1 - 1], [y0, y1 - 1])
    mu = rec["mu32"]
    zero = np.float32(0.0)
    dx = np.maximum(np.maximum(mu[:, 0] - ux32[1], zero), ux32[0] - mu[:, 1])
    dy = np.maximum(np.maximum(mu[:, 2] - uy32[1], zero), uy32[0] - mu[:, 3])
    d2 = (dx * dx + dy * dy).astype(np.float32)
    keep = (rec["normal"] & (d2 <= rec["r2_32"])) | rec["wild"]
    return np.nonzero(keep)[0]


def pixel_alpha(rec, idx, ux, uy):
    """Alpha forms at pixels (the q and a steps of Step 3) for Gaussians idx: (LF (n, m), a_lo, a_hi)."""
    D2 = rec["D2"][idx].expand(-1)
    DUP = rec["DUP"][idx]
    B = rec["B"][idx]
    o = rec["o"][idx]
    o_lo = rec["o_lo"][idx]
    ux = np.asarray(ux, dtype=np.float64)[None, :]
    uy = np.asarray(uy, dtype=np.float64)[None, :]
    # v = Add(Mul(d, d, u), -Mul(d, up))
    v0 = lf.sub(lf.scale(D2, ux), DUP[:, 0].expand(-1))
    v1 = lf.sub(lf.scale(D2, uy), DUP[:, 1].expand(-1))
    # q = v (Conic Mp)
    q = [lf.add(lf.mul(v0, B[:, 0, n].expand(-1)), lf.mul(v1, B[:, 1, n].expand(-1))) for n in range(3)]
    # s = q q^T
    s = lf.add(lf.add(lf.sqr(q[0]), lf.sqr(q[1])), lf.sqr(q[2]))
    slo, shi = s.bounds()
    xlo = -0.5 * shi
    xhi = -0.5 * np.maximum(0.0, slo)
    x = lf.scale(s, -0.5)
    # a = o Exp(x); with an opacity interval [o_lo, o] the lower form scales by o_lo
    # (Exp's forms and values are positive where they bound alpha from the right side)
    ex = lf.exp(x, xlo, xhi)
    a = lf.LF(lf.scale(ex, o_lo[:, None]).lo, lf.scale(ex, o[:, None]).up)
    return a, o_lo[:, None] * np.exp(xlo), o[:, None] * np.exp(xhi)


IND_MARGIN = 1e-10


def ind_matrix(rec, idx, block=256):
    """Three-valued Ind(d_i - d_j) for Gaussians idx: 1, 0, or 2 (unknown); plus borderline mask.

    d_i - d_j is bounded two ways, both sound: the identity d_i - d_j = A_z (uw_i - uw_j)
    behind the depth d = uc_z (tau and beta cancel), and the literal Add(d[i], -d[j]) of
    the two depth forms (the V step of Alg. BlendInd).  Ind is 1 if either lower bound proves
    d_i > d_j, 0 if either upper bound proves d_i <= d_j, unknown otherwise.  The
    literal bound is used with a margin IND_MARGIN: its depth forms carry rounding
    noise, and at an exact tie (identity bound exactly 0) that noise must not decide.
    The identity is used only for pairs of Gaussians whose means are fixed: a mean moved
    by a scene variable (Sec. 4.6) is not the constant uw_i of the identity, and the
    literal bound alone decides pairs that involve one.  Rows are evaluated in blocks to
    bound memory.
    """
    A3 = rec["A"][2]                       # z-row of A, quantity shape (3,)
    uw = rec["uw"][idx]
    d = rec["d"][idx]
    mov = rec["moving"][idx]
    n = len(idx)
    ind = np.empty((n, n), np.int8)
    border = np.empty((n, n), bool)
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        duw = uw[b0:b1, None, :] - uw[None, :, :]  # (b, n, 3) constants
        delta = lf.scale(lf.broadcast(A3, duw.shape), duw).sum(-1)
        lo_r, hi_r = delta.bounds()
        lit = lf.sub(d[b0:b1].expand(-1), d.expand(0))
        lo_l, hi_l = lit.bounds()
        fixed = ~(mov[b0:b1, None] | mov[None, :])
        one = ((lo_r > 0) & fixed) | (lo_l > IND_MARGIN)
        zero = ((hi_r <= 0) & fixed) | (hi_l <= -IND_MARGIN)
        ind[b0:b1] = np.where(one, 1, np.where(zero, 0, 2))
        s = 1e-12 * (1.0 + np.abs(duw).sum(axis=-1))
        exact_tie = (lo_r == hi_r) & (lo_r == 0)
        border[b0:b1] = (~exact_tie) & ((np.abs(lo_r) < s) | (np.abs(hi_r) < s)
                                        | (np.abs(lo_l - IND_MARGIN) < s) | (np.abs(hi_l + IND_MARGIN) < s))
    np.fill_diagonal(ind, 0)
    np.fill_diagonal(border, False)
    return ind, border


def blend(al, au, alo_f, aup_f, c, ind, E, c_hi=None):
    """BlendInd (Alg. BlendInd) on interval / linear-form alphas; colour bounds per pixel.

    al, au: (n, m) alpha interval per Gaussian and pixel; alo_f, aup_f: (n, m, P+1)
    lower / upper alpha forms; c: (n, 3) colours; ind: (n, n) in {0, 1, 2 = unknown}.
    V and T steps: V_ij = 1 - a_j Ind_ij is an interval; T_i = prod_j V_ij:
        T_hi[i] = prod_{Ind_ij = 1} (1 - al[j]),   T_lo[i] = prod_{Ind_ij != 0} (1 - au[j]).
    pc step: pc = sum_i T_i a_i c_i, bounded relationally and by intervals.
    Returns lo, hi (m, 3), not clamped.
    """
    n, m = al.shape
    P = alo_f.shape[-1] - 1
    T_hi = np.empty((n, m))
    T_lo = np.empty((n, m))
    one_m_al = 1.0 - al
    one_m_au = 1.0 - au
    for i in range(n):
        T_hi[i] = np.prod(one_m_al[ind[i] == 1], axis=0)
        T_lo[i] = np.prod(one_m_au[ind[i] != 0], axis=0)
    c_hi = c if c_hi is None else c_hi                     # colour interval [c, c_hi] (Sec. 4.6)
    w_lo = T_lo[:, :, None] * c[:, None, :]               # (n, m, 3)
    w_hi = T_hi[:, :, None] * c_hi[:, None, :]
    f_lo = np.einsum("nmc,nmp->mcp", w_lo, alo_f)         # (m, 3, P+1)
    f_hi = np.einsum("nmc,nmp->mcp", w_hi, aup_f)
    rel_lo = f_lo[..., -1] - np.abs(f_lo[..., :P]).sum(axis=-1)
    rel_hi = f_hi[..., -1] + np.abs(f_hi[..., :P]).sum(axis=-1)
    int_lo = np.einsum("nmc,nm->mc", w_lo, al)
    int_hi = np.einsum("nmc,nm->mc", w_hi, au)
    lo = np.maximum(rel_lo, int_lo) - E
    hi = np.minimum(rel_hi, int_hi) + E
    return lo, hi


def blend_interval(al, au, c, ind, E, c_hi=None):
    """BlendInd with the interval colour sum only (the relational sum of blend() left out):
    the T step as in blend(), pc in [sum c T_lo a_lo, sum c T_hi a_hi].  A precision
    baseline for the comparison with the abstract BlendSort."""
    n, m = al.shape
    T_hi = np.empty((n, m))
    T_lo = np.empty((n, m))
    for i in range(n):
        T_hi[i] = np.prod(1.0 - al[ind[i] == 1], axis=0)
        T_lo[i] = np.prod(1.0 - au[ind[i] != 0], axis=0)
    c_hi = c if c_hi is None else c_hi
    lo = np.einsum("nm,nc->mc", T_lo * al, c) - E
    hi = np.einsum("nm,nc->mc", T_hi * au, c_hi) + E
    return lo, hi


def blend_sort_abstract(al, au, c, dlo, dhi, E, c_hi=None):
    """Abstract BlendSort (Alg. BlendSort with an abstract Sort): the precision baseline of
    Sec. 3.2 that BlendInd replaces (Example '3g-scene').

    Sort is not linearly over-approximable (Sec. 2.1); an abstract sort sees each depth as
    the set of its values, the interval [dlo_i, dhi_i], and not the relation between two
    depths that Ind(d_i - d_j) uses.  Gaussian i can then only sit at sorted positions k
    with r_lo[i] <= k <= r_hi[i]: r_lo[i] counts the Gaussians surely strictly in front of
    it (dhi_j < dlo_i), r_hi[i] those that may be sorted before it (dlo_j <= dhi_i, j != i).
    Slot k holds one of its candidates C_k, so its alpha lies in
    [min_{C_k} a_lo, max_{C_k} a_hi].  The Ts step is the interval product over the slots in
    front:
        Gaussian i at slot k:  prod_{j<k} (1 - max a_hi of slot j)
                               <= T_i <=  prod_{j<r_lo[i]} (1 - min a_lo of slot j)
    (the strictly-in-front Gaussians fill the first slots, at least r_lo[i] of them; ties
    share a transmittance, so the upper product stops at r_lo[i], not at k).  pc step:
        lo = sum_k prod_{j<k}(1 - a_hi slot j) * min_{i in C_k} a_lo[i] c_i
        hi = sum_k max_{i in C_k} prod_{j<r_lo[i]}(1 - a_lo slot j) a_hi[i] c_i
    A Gaussian can be counted at several slots, the over-counting Sec. 3.2 attributes to
    index-based accumulation.  al, au: (n, m); c: (n, 3); dlo, dhi: (n,).
    Returns lo, hi (m, 3), widened by E, not clamped.
    """
    n, m = al.shape
    c = np.asarray(c, dtype=np.float64)
    c_hi = c if c_hi is None else np.asarray(c_hi, dtype=np.float64)
    if n == 0:
        return np.zeros((m, 3)) - E, np.zeros((m, 3)) + E
    dlo = np.asarray(dlo, dtype=np.float64)
    dhi = np.asarray(dhi, dtype=np.float64)
    r_lo = (dhi[None, :] < dlo[:, None]).sum(axis=1)
    r_hi = (dlo[None, :] <= dhi[:, None]).sum(axis=1) - 1
    cand = [(r_lo <= k) & (k <= r_hi) for k in range(n)]
    al_slot = np.stack([al[ck].min(axis=0) for ck in cand])      # (n slots, m)
    au_slot = np.stack([au[ck].max(axis=0) for ck in cand])
    T_lo_slot = np.cumprod(np.vstack([np.ones((1, m)), 1.0 - au_slot]), axis=0)[:n]
    T_hi_rank = np.cumprod(np.vstack([np.ones((1, m)), 1.0 - al_slot]), axis=0)   # row r: r slots
    term_hi = T_hi_rank[r_lo][:, :, None] * au[:, :, None] * c_hi[:, None, :]     # (n, m, 3)
    term_lo = al[:, :, None] * c[:, None, :]
    lo = np.zeros((m, 3))
    hi = np.zeros((m, 3))
    for k in range(n):
        lo += T_lo_slot[k][:, None] * term_lo[cand[k]].min(axis=0)
        hi += term_hi[cand[k]].max(axis=0)
    return lo - E, hi + E


def blend_tile(rec, idx, ux, uy, ux32, uy32):
    """BlendInd with interval transmittances and the relational colour sum for one pixel set.

    Returns lo (m, 3), hi (m, 3), kept count (m,), borderline flag (m,).
    """
    n = len(idx)
    m = len(ux)
    P = rec["P"]
    if n == 0:
        z = np.zeros((m, 3))
        return z - rec["E"], z + rec["E"], np.zeros(m, np.int64), np.zeros(m, bool)
    keep = kept_mask(rec, idx, ux32, uy32)
    al = np.empty((n, m))
    au = np.empty((n, m))
    alo_f = np.empty((n, m, P + 1))
    aup_f = np.empty((n, m, P + 1))
    with np.errstate(all="ignore"):
        for s in range(0, n, 128):
            a, al[s:s + 128], au[s:s + 128] = pixel_alpha(rec, idx[s:s + 128], ux, uy)
            alo_f[s:s + 128] = a.lo
            aup_f[s:s + 128] = a.up
    o = rec["o"][idx][:, None]
    # MatrixInv fallback: constant [0, o exp(-dist^2 / (2 lam))]
    fb = rec["fallback"][idx][:, None] & np.ones((1, m), bool)
    if fb.any():
        mu = rec["mu32"][idx].astype(np.float64)
        dx = np.maximum(np.maximum(mu[:, None, 0] - ux[None, :], 0.0), ux[None, :] - mu[:, None, 1])
        dy = np.maximum(np.maximum(mu[:, None, 2] - uy[None, :], 0.0), uy[None, :] - mu[:, None, 3])
        with np.errstate(invalid="ignore"):
            fb_hi = o * np.exp(-0.5 * (dx * dx + dy * dy) / rec["lam"][idx][:, None])
        al = np.where(fb, 0.0, al)
        au = np.where(fb, fb_hi, au)
        alo_f = np.where(fb[..., None], 0.0, alo_f)
        aup_f = np.where(fb[..., None], 0.0, aup_f)
        aup_f[..., -1] = np.where(fb, fb_hi, aup_f[..., -1])
    # straddlers / unbounded footprints: constant [0, o]
    wd = rec["wild"][idx][:, None] & np.ones((1, m), bool)
    if wd.any():
        al = np.where(wd, 0.0, al)
        au = np.where(wd, o, au)
        alo_f = np.where(wd[..., None], 0.0, alo_f)
        aup_f = np.where(wd[..., None], 0.0, aup_f)
        aup_f[..., -1] = np.where(wd, np.broadcast_to(o, wd.shape), aup_f[..., -1])
    # pruned pairs contribute nothing
    al = np.where(keep, al, 0.0)
    au = np.where(keep, au, 0.0)
    alo_f = np.where(keep[..., None], alo_f, 0.0)
    aup_f = np.where(keep[..., None], aup_f, 0.0)

    ind, border = ind_matrix(rec, idx)
    mode = rec["opts"]["blend"]
    c_lo, c_hi = rec["rgb"][idx], rec["rgb_hi"][idx]
    if mode == "sort":
        dlo, dhi = rec["d"][idx].bounds()
        lo, hi = blend_sort_abstract(al, au, c_lo, dlo, dhi, rec["E"], c_hi)
    elif mode == "ind_interval":
        lo, hi = blend_interval(al, au, c_lo, ind, rec["E"], c_hi)
    else:
        lo, hi = blend(al, au, alo_f, aup_f, c_lo, ind, rec["E"], c_hi)
    bflag = np.zeros(m, bool)
    if border.any():
        bi, bj = np.nonzero(border)
        bflag = (keep[bi] & keep[bj]).any(axis=0)
    return lo, hi, keep.sum(axis=0), bflag


def oracle_bounds(scene, intr, box, opts=None, tiles=None, rec=None):
    """Lower/upper images (H, W, 3) in FP64 over the pose box.

    tiles: optional list of (tx, ty) tile indices to evaluate (others are left NaN).
    Returns dict with lo, hi, pairs (kept Gaussians per pixel), border, rec.
    """
    opts = options(opts)
    if rec is None:
        rec = gaussian_forms(scene, intr, box, opts)
    W, H = int(intr["width"]), int(intr["height"])
    TS = int(opts["tile"])
    lo = np.full((H, W, 3), np.nan)
    hi = np.full((H, W, 3), np.nan)
    pairs = np.zeros((H, W), np.int64)
    border = np.zeros((H, W), bool)
    ntx, nty = (W + TS - 1) // TS, (H + TS - 1) // TS
    if tiles is None:
        tiles = [(tx, ty) for ty in range(nty) for tx in range(ntx)]
    for tx, ty in tiles:
        x0, y0 = tx * TS, ty * TS
        x1, y1 = min(x0 + TS, W), min(y0 + TS, H)
        idx = tile_candidates(rec, intr, x0, x1, y0, y1)
        cols, rows = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), indexing="xy")
        cols, rows = cols.ravel(), rows.ravel()
        ux = cols + 0.5 - float(intr["cx"])
        uy = rows + 0.5 - float(intr["cy"])
        ux32, uy32 = pixel_coords32(intr, cols, rows)
        l, h, k, b = blend_tile(rec, idx, ux, uy, ux32, uy32)
        lo[rows, cols] = np.clip(l, 0.0, 1.0)
        hi[rows, cols] = np.clip(h, 0.0, 1.0)
        pairs[rows, cols] = k
        border[rows, cols] = b
    return {"lo": lo, "hi": hi, "pairs": pairs, "border": border, "rec": rec}


def box_rotates(scene, box):
    """Whether the depth order of the scene can change over the box: a rotation axis of a
    CAMERA6 box or the angle of an ORBIT box has positive width, or the scene has set
    variables (a moved mean can change the order under any box).  Otherwise the camera
    only translates, the depth difference of two Gaussians is constant over the box
    (translations cancel in d_i - d_j), and no Ind is ever undecided."""
    lo = np.asarray(box["lo"], dtype=np.float64)
    hi = np.asarray(box["hi"], dtype=np.float64)
    if box.get("model", pose.CAMERA6) == pose.ORBIT:
        rot = bool(hi[0] > lo[0])
    else:
        rot = bool((hi[3:6] > lo[3:6]).any())
    return rot or scene_set(scene)[4] > 0


def ind_uncertain_count(scene, intr, box, opts=None, rec=None):
    """Undecided depth-order tests over a pose cell (Sec. 3.2: Ind(d_i - d_j) is piecewise
    constant, tight on every part of the domain where d_i - d_j keeps its sign, which is
    what partitioning the input aims at): the ordered pairs (i, j), i != j, of Gaussians in
    one tile list (the binning's candidates of the tile) whose three-valued Ind is 2,
    summed over the tile lists; 0 when the box cannot change the depth order.  Also
    returns the number of pairs whose bound sits within rounding of a decision
    threshold (ind_matrix's borderline mask), where an evaluation in another order of
    operations may decide differently.  The tile lists are those of 8x8-pixel tiles (the
    library's) unless opts gives another tile.  Returns (count, borderline)."""
    opts = options({"tile": 8, **(opts or {})})
    if not box_rotates(scene, box):
        return 0, 0
    if rec is None:
        rec = gaussian_forms(scene, intr, box, opts)
    W, H = int(intr["width"]), int(intr["height"])
    TS = int(opts["tile"])
    total = border_total = 0
    for ty in range((H + TS - 1) // TS):
        for tx in range((W + TS - 1) // TS):
            x0, y0 = tx * TS, ty * TS
            idx = tile_candidates(rec, intr, x0, min(x0 + TS, W), y0, min(y0 + TS, H))
            if len(idx) < 2:
                continue
            ind, border = ind_matrix(rec, idx)
            total += int((ind == 2).sum())
            border_total += int(border.sum())
    return total, border_total
