"""Seeded synthetic inputs: Gaussian-splat scenes, intrinsics and camera-pose boxes.

Shared by the tests, the benchmark and the smoke check.  This module only draws
random numbers and builds scene / camera descriptions; it holds none of the
abstract-rendering arithmetic, and neither the oracle nor the HIP path is imported.

The paper's scenes are trained splats that are not available here; these synthetic
scenes stand in for them with the paper's sizes (5.7e4 - 8.8e5 Gaussians, images of
48^2 - 200^2 and beyond) and pose boxes (translation half-widths 0.002 - 10 scene
units, rotation half-widths 0.001 - 0.3 rad).

A scene is a dict of float32 arrays:
  mean (N, 3), cov_factor (N, 3, 3) with Cov = M M^T, opacity (N,), rgb (N, 3).
Intrinsics: dict width, height, fx, fy, cx, cy.
Pose box: dict model (0 = CAMERA6, 1 = ORBIT), R0 (3x3), t0 (3), pivot (3),
  lo (6), hi (6) -- CAMERA6 order (tx, ty, tz, yaw, pitch, roll); ORBIT uses lo[0], hi[0] (phi).
"""
from __future__ import annotations

import numpy as np

CAMERA6 = 0
ORBIT = 1


def _quat_to_rot(q):
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((len(q), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _pack(mean, R, scales, opacity, rgb):
    M = R * scales[:, None, :]                    # M = R diag(s), Cov = M M^T
    return {
        "mean": np.ascontiguousarray(mean, dtype=np.float32),
        "cov_factor": np.ascontiguousarray(M, dtype=np.float32),
        "opacity": np.ascontiguousarray(opacity, dtype=np.float32),
        "rgb": np.ascontiguousarray(rgb, dtype=np.float32),
    }


def random_scene(n, seed=0, depth=4.0):
    """Means uniform in [-1,1]^3 shifted to depth 3-5, log-uniform scales in [0.02, 0.2],
    random unit quaternions, RGB uniform [0,1], opacity uniform [0.1, 0.9]."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, (n, 3)) + np.array([0.0, 0.0, depth])
    scales = np.exp(rng.uniform(np.log(0.02), np.log(0.2), (n, 3)))
    R = _quat_to_rot(rng.standard_normal((n, 4)))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    opacity = rng.uniform(0.1, 0.9, n)
    return _pack(mean, R, scales, opacity, rgb)


def box_surface_scene(n, n_boxes=20, seed=0, scale=1.0):
    """Gaussians on the surfaces of random boxes (object-scale scene).

    Box centres uniform in [-1,1]^2 x [3,5], half-extents uniform [0.1, 0.4], random yaw;
    an equal share of Gaussians per box, uniform by area over its six faces; flat
    Gaussians (tangential scales log-uniform [0.01, 0.05] times `scale`, normal scale
    0.2x the smaller tangential one) aligned with the face; RGB = box colour +
    N(0, 0.05) clipped to [0,1]; opacity ~ Beta(2, 2).
    """
    rng = np.random.default_rng(seed)
    per = np.full(n_boxes, n // n_boxes)
    per[: n - per.sum()] += 1
    means, rots, scs, cols = [], [], [], []
    for b in range(n_boxes):
        c = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 5)])
        h = rng.uniform(0.1, 0.4, 3)
        yaw = rng.uniform(0, 2 * np.pi)
        cy, sy = np.cos(yaw), np.sin(yaw)
        Rb = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
        colour = rng.uniform(0, 1, 3)
        # faces: axis k, sign s; area of face = 4 * h[i] * h[j]
        faces = [(k, s) for k in range(3) for s in (-1.0, 1.0)]
        areas = np.array([4 * np.prod(np.delete(h, k)) for k, _ in faces])
        f_idx = rng.choice(6, size=per[b], p=areas / areas.sum())
        for fi in range(6):
            m = int((f_idx == fi).sum())
            if m == 0:
                continue
            k, s = faces[fi]
            t1, t2 = [a for a in range(3) if a != k]
            local = np.zeros((m, 3))
            local[:, k] = s * h[k]
            local[:, t1] = rng.uniform(-h[t1], h[t1], m)
            local[:, t2] = rng.uniform(-h[t2], h[t2], m)
            means.append(local @ Rb.T + c)
            tang = scale * np.exp(rng.uniform(np.log(0.01), np.log(0.05), (m, 2)))
            sc = np.zeros((m, 3))
            sc[:, t1] = tang[:, 0]
            sc[:, t2] = tang[:, 1]
            sc[:, k] = 0.2 * tang.min(axis=1)
            # in-plane random rotation about the face normal, then the box yaw
            th = rng.uniform(0, 2 * np.pi, m)
            Rl = np.zeros((m, 3, 3))
            Rl[:, k, k] = 1.0
            Rl[:, t1, t1] = np.cos(th)
            Rl[:, t1, t2] = -np.sin(th)
            Rl[:, t2, t1] = np.sin(th)
            Rl[:, t2, t2] = np.cos(th)
            rots.append(np.einsum("ij,njk->nik", Rb, Rl))
            scs.append(sc)
            cols.append(np.clip(colour + rng.normal(0, 0.05, (m, 3)), 0, 1))
    mean = np.concatenate(means)
    R = np.concatenate(rots)
    sc = np.concatenate(scs)
    rgb = np.concatenate(cols)
    perm = rng.permutation(len(mean))
    opacity = rng.beta(2.0, 2.0, len(mean))
    return _pack(mean[perm], R[perm], sc[perm], opacity, rgb[perm])


def intrinsics(side, f=None):
    """Square pinhole camera with fx = fy = side (a 53-degree field of view) by default."""
    f = float(side) if f is None else float(f)
    return {"width": int(side), "height": int(side), "fx": f, "fy": f,
            "cx": side / 2.0, "cy": side / 2.0}


def camera6_box(dt=(0, 0, 0), drot=(0, 0, 0), R0=None, t0=None):
    """CAMERA6 box of half-widths dt (translation) and drot (yaw, pitch, roll, radians)."""
    dt = np.broadcast_to(np.asarray(dt, dtype=np.float64), (3,))
    dr = np.broadcast_to(np.asarray(drot, dtype=np.float64), (3,))
    half = np.concatenate([dt, dr])
    return {"model": CAMERA6, "R0": np.eye(3) if R0 is None else np.asarray(R0, np.float64),
            "t0": np.zeros(3) if t0 is None else np.asarray(t0, np.float64),
            "pivot": np.zeros(3), "lo": -half, "hi": half.copy()}


def orbit_cells(n_cells=256, total_deg=30.0, seed=0, pivot=(0.0, 0.0, 4.0)):
    """A total_deg orbit about the vertical axis through pivot split into cells of uneven
    widths (proportional to U[0.2, 2], renormalised to the total)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 2.0, n_cells)
    w = w / w.sum() * np.deg2rad(total_deg)
    edges = -np.deg2rad(total_deg) / 2 + np.concatenate([[0.0], np.cumsum(w)])
    cells = []
    for i in range(n_cells):
        lo = np.zeros(6)
        hi = np.zeros(6)
        lo[0], hi[0] = edges[i], edges[i + 1]
        cells.append({"model": ORBIT, "R0": np.eye(3), "t0": np.zeros(3),
                      "pivot": np.asarray(pivot, np.float64), "lo": lo, "hi": hi})
    return cells


# --- the five workloads -----------------------------------------------------------------
def config(idx, seed=0):
    """(scene, intrinsics, box or list of boxes, description) for workload idx in 1..4."""
    if idx == 1:
        return (random_scene(64, seed), intrinsics(32), camera6_box(dt=(0.05, 0.0, 0.0)),
                "64 Gaussians, 32x32, translation-x box +-0.05")
    if idx == 2:
        return (random_scene(10_000, seed), intrinsics(128), camera6_box(dt=0.1),
                "10k Gaussians, 128x128, 3-D translation box +-0.1")
    if idx == 3:
        return (box_surface_scene(100_000, seed=seed), intrinsics(400),
                camera6_box(dt=0.05, drot=np.deg2rad(1.0)),
                "100k Gaussians on 20 boxes, 400x400, translation +-0.05 and yaw/pitch/roll +-1 deg")
    if idx == 4:
        return (box_surface_scene(50_000, seed=seed), intrinsics(200), orbit_cells(256, 30.0, seed),
                "50k Gaussians on 20 boxes, 200x200, 30-degree orbit in 256 uneven cells")
    raise ValueError(idx)


def served_scenes(seed=0):
    """Four resident scenes of the serving workload (10k, 100k, 300k, 750k Gaussians).

    Gaussian sizes shrink as the count grows, sqrt(1e5 / n) times those of the 100k
    object scene, so every scene covers its boxes with a similar number of layers (a
    trained splat adapts Gaussian size to detail in the same way)."""
    return [box_surface_scene(n, seed=seed + i, scale=float(np.sqrt(1e5 / n)))
            for i, n in enumerate((10_000, 100_000, 300_000, 750_000))]


def served_queries(n_queries, seed=0):
    """Query stream: (scene index, image side, box); scene and image side (100, 200, 400
    or 800) drawn independently and uniformly, translation full widths U[0.01, 0.1] per
    axis and rotation full widths U[0, 2] degrees per axis."""
    rng = np.random.default_rng(seed)
    sides = (100, 200, 400, 800)
    out = []
    for _ in range(n_queries):
        s = int(rng.integers(0, 4))
        side = sides[int(rng.integers(0, 4))]
        dt = 0.5 * rng.uniform(0.01, 0.1, 3)
        dr = 0.5 * np.deg2rad(rng.uniform(0.0, 2.0, 3))
        out.append((s, side, camera6_box(dt=dt, drot=dr)))
    return out


def perturbed_scene(scene, kinds=("colour",), frac=0.3, shift=0.1, seed=0):
    """A set of scenes around `scene` in the manner of the paper's scene-perturbation
    experiments (Sec. 4.6), applied to a spatially contiguous subset of the Gaussians (the
    fraction `frac` with the smallest x of their means, an object of the scene):
      "colour"  the red channel raised by up to 0.5 (upper bound min(1, r + 0.5));
      "mean"    the subset's means moved along +y by s * shift, s in [0, 1] (one shared
                scene variable);
      "opacity" the opacities scaled by 0.1 and raised by up to 0.1 (interval
                [0.1 o, min(1, 0.1 o + 0.1)]).
    Returns a copy of the scene dict with the set keys (rgb_hi, opacity_lo, set_lo,
    set_hi, mean_var, mean_dir) that apply."""
    out = dict(scene)
    n = len(scene["opacity"])
    order = np.argsort(np.asarray(scene["mean"])[:, 0], kind="stable")
    sub = np.zeros(n, bool)
    sub[order[:max(1, int(round(frac * n)))]] = True
    if "colour" in kinds:
        rgb_hi = np.array(scene["rgb"], dtype=np.float32)
        rgb_hi[sub, 0] = np.minimum(1.0, rgb_hi[sub, 0] + np.float32(0.5))
        out["rgb_hi"] = rgb_hi
    if "opacity" in kinds:
        o = np.array(scene["opacity"], dtype=np.float32)
        lo = o.copy()
        hi = o.copy()
        lo[sub] = np.float32(0.1) * o[sub]
        hi[sub] = np.minimum(np.float32(1.0), np.float32(0.1) * o[sub] + np.float32(0.1))
        out["opacity"] = hi
        out["opacity_lo"] = lo
    if "mean" in kinds:
        out["set_lo"] = np.array([0.0])
        out["set_hi"] = np.array([1.0])
        out["mean_var"] = np.where(sub, 0, -1).astype(np.int32)
        d = np.zeros((n, 3), np.float32)
        d[sub, 1] = np.float32(shift)
        out["mean_dir"] = d
    return out
