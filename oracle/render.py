"""Concrete Gaussian-splat renderer in FP64 (Alg. GaussianSplat with BlendSort / BlendInd).

Test infrastructure only.

Conventions (the paper leaves them open):
* camera axes x right, y down, z forward; uc = R (uw - t), R world->camera;
* pixel (col, row) has centre u = (col + 1/2, row + 1/2); the principal point is
  subtracted from u and dropped from K, so d^2 u - d up is evaluated as
  d^2 (u - c) - d (fx x, fy y) (the same number, the q step of Alg. GaussianSplat);
* a Gaussian whose depth d is not above the near plane z_near has a = 0;
* Gaussians at equal depth do not occlude one another: the transmittance of
  Gaussian i is the product of (1 - a_j) over the Gaussians strictly in front of
  it.  This is BlendInd's rule (Ind(0) = 0) and coincides with BlendSort whenever
  the depths are distinct (Lemma "BlendSort = BlendInd").
"""
from __future__ import annotations

import numpy as np

from .matinv import inv2
from .pose import concrete_camera


def pixel_grid(intr, rows=None, cols=None):
    """Centred pixel coordinates (u - cx, v - cy) for the given rows/cols (default: whole image)."""
    W, H = int(intr["width"]), int(intr["height"])
    rows = np.arange(H) if rows is None else np.asarray(rows)
    cols = np.arange(W) if cols is None else np.asarray(cols)
    uu, vv = np.meshgrid(cols + 0.5 - intr["cx"], rows + 0.5 - intr["cy"], indexing="xy")
    return uu.ravel(), vv.ravel()


def project(scene, intr, R, t):
    """Steps 1-3a of the algorithm for every Gaussian at one camera (R, t)."""
    uw = np.asarray(scene["mean"], dtype=np.float64)
    Mw = np.asarray(scene["cov_factor"], dtype=np.float64)
    uc = (uw - t) @ R.T                                     # Step 1: uc
    Mc = np.einsum("kl,nlm->nkm", R, Mw)                    # Step 1: Mc
    x, y, z = uc[:, 0], uc[:, 1], uc[:, 2]
    fx, fy = intr["fx"], intr["fy"]
    J = np.zeros((len(uw), 2, 3))                           # Step 2: J
    J[:, 0, 0] = fx * z
    J[:, 0, 2] = -fx * x
    J[:, 1, 1] = fy * z
    J[:, 1, 2] = -fy * y
    upc = np.stack([fx * x, fy * y], axis=1)                # Step 2: up, principal point removed
    Mp = J @ Mc                                             # Step 2: Mp
    d = z                                                   # Step 2: d
    X = Mp @ np.transpose(Mp, (0, 2, 1))
    conic, det = inv2(X)                                    # Step 3: Conic
    return {"d": d, "upc": upc, "Mp": Mp, "conic": conic, "det": det}


def alpha(scene, intr, proj, ux, uy, z_near):
    """Effective opacities a[i, pixel] (the q and a steps of Step 3), shape (N, n_pixels)."""
    d = proj["d"][:, None]
    v0 = d * d * ux[None, :] - d * proj["upc"][:, 0:1]
    v1 = d * d * uy[None, :] - d * proj["upc"][:, 1:2]
    B = proj["conic"] @ proj["Mp"]                          # (N, 2, 3)
    q = v0[:, :, None] * B[:, None, 0, :] + v1[:, :, None] * B[:, None, 1, :]
    s = (q * q).sum(axis=-1)
    o = np.asarray(scene["opacity"], dtype=np.float64)[:, None]
    a = o * np.exp(-0.5 * s)
    valid = (proj["d"] > z_near) & (proj["det"] > 0)
    return np.where(valid[:, None], a, 0.0)


def blend_sort(a, c, d):
    """BlendSort: transmittance as the product over Gaussians strictly in front (ties share it).

    a: (N, n_pix), c: (N, 3), d: (N,) -> pc (n_pix, 3).
    """
    order = np.argsort(d, kind="stable")
    a_s = a[order]
    c_s = np.asarray(c, dtype=np.float64)[order]
    d_s = d[order]
    one_minus = 1.0 - a_s
    # exclusive prefix products along the sorted order
    cum = np.cumprod(np.vstack([np.ones((1, a.shape[1])), one_minus]), axis=0)
    # transmittance of a tie group is the prefix product at the group's first member
    first = np.searchsorted(d_s, d_s, side="left")
    Ts = cum[first]
    return np.einsum("np,nc->pc", Ts * a_s, c_s)


def blend_ind(a, c, d):
    """BlendInd (Alg. BlendInd): T_i = prod_j (1 - a_j Ind(d_i - d_j)); pc = sum_i T_i a_i c_i."""
    N = len(d)
    ind = (d[:, None] - d[None, :]) > 0
    T = np.ones_like(a)
    for i in range(N):
        T[i] = np.prod(1.0 - a * ind[i][:, None], axis=0)
    return np.einsum("np,nc->pc", T * a, np.asarray(c, dtype=np.float64))


def instantiate(scene, s=None, t_rgb=0.0, t_o=1.0):
    """One concrete scene of a set of scenes (Sec. 4.6; keys as splat.scene_set): means moved
    by the scene variables s, colours rgb + t_rgb (rgb_hi - rgb), opacities
    opacity_lo + t_o (opacity - opacity_lo); t_rgb, t_o in [0, 1], scalars or per Gaussian."""
    mean = np.asarray(scene["mean"], dtype=np.float64).copy()
    if s is not None and len(np.atleast_1d(s)):
        mvar = np.asarray(scene["mean_var"])
        mdir = np.asarray(scene["mean_dir"], dtype=np.float64)
        s = np.asarray(s, dtype=np.float64)
        rows = mvar >= 0
        mean[rows] += mdir[rows] * s[mvar[rows]][:, None]
    rgb = np.asarray(scene["rgb"], dtype=np.float64)
    rgb_hi = np.asarray(scene.get("rgb_hi", rgb), dtype=np.float64)
    o = np.asarray(scene["opacity"], dtype=np.float64)
    o_lo = np.asarray(scene.get("opacity_lo", o), dtype=np.float64)
    t_rgb = np.asarray(t_rgb, dtype=np.float64)
    t_o = np.asarray(t_o, dtype=np.float64)
    return {"mean": mean, "cov_factor": scene["cov_factor"],
            "rgb": rgb + (t_rgb[..., None] if t_rgb.ndim else t_rgb) * (rgb_hi - rgb),
            "opacity": o_lo + t_o * (o - o_lo)}


def render(scene, intr, box, p, z_near=0.01, chunk=4096):
    """Concrete image (H, W, 3) at pose p of the box (FP64)."""
    R, t = concrete_camera(box, p)
    proj = project(scene, intr, R, t)
    ux, uy = pixel_grid(intr)
    out = np.empty((len(ux), 3))
    for s in range(0, len(ux), chunk):
        a = alpha(scene, intr, proj, ux[s:s + chunk], uy[s:s + chunk], z_near)
        out[s:s + chunk] = blend_sort(a, scene["rgb"], proj["d"])
    return out.reshape(int(intr["height"]), int(intr["width"]), 3)
