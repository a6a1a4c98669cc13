"""Pose stage of the FP64 oracle: the camera set as linear forms (test infrastructure only).

The renderer's first step maps a world point to camera coordinates,
uc = Mmul(R, Add(uw, -t)) (Alg. GaussianSplat, Step 1).  For a set of cameras the
oracle writes every camera model as

    uc = Mmul(A, Add(uw, -tau)) + beta

with A (3x3), tau (3) and beta (3) linear forms over the normalised pose box.

* CAMERA6 -- the box of Sec. 4.2 (position radius eps_t, orientation radius eps_R
  around a nominal camera).  Pose p = (tx, ty, tz, yaw, pitch, roll);
  R(p) = Ry(yaw) Rx(pitch) Rz(roll) R0 (perturbation applied in the camera frame,
  products taken left to right with Mul), t(p) = t0 + (tx, ty, tz).
  A = R(p), tau = t(p), beta = 0: exactly the camera transform of Step 1.
* ORBIT -- camera rig turned by phi about the vertical axis through a pivot c:
  t(phi) = c + Ry(phi)(t0 - c), R(phi) = R0 Ry(phi)^T, hence
  uc = R0 Ry(-phi) (uw - c) + R0 (c - t0): A = R0 Ry(-phi), tau = c, beta = R0(c - t0).

Only axes with a non-zero radius are pose variables; the i-th active axis is e[i].
"""
from __future__ import annotations

import numpy as np

from . import lf

CAMERA6 = 0
ORBIT = 1


def _axes(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if np.any(hi < lo):
        raise ValueError("pose box has lo > hi")
    centre = 0.5 * (lo + hi)
    radius = 0.5 * (hi - lo)
    active = np.nonzero(radius > 0)[0]
    return centre, radius, active


def _param(centre, radius, active, axis, P):
    if axis in active:
        return lf.variable(centre[axis], radius[axis], int(np.nonzero(active == axis)[0][0]), P)
    return lf.const(centre[axis], P)


def _rot(axis: str, ang: lf.LF, P: int) -> lf.LF:
    """Right-handed elementary rotation by an angle given as an exact affine form."""
    c = lf.trig(ang, "cos")
    s = lf.trig(ang, "sin")
    one = lf.const(1.0, P)
    zero = lf.const(0.0, P)
    ns = lf.neg(s)
    if axis == "x":
        rows = [[one, zero, zero], [zero, c, ns], [zero, s, c]]
    elif axis == "y":
        rows = [[c, zero, s], [zero, one, zero], [ns, zero, c]]
    elif axis == "z":
        rows = [[c, ns, zero], [s, c, zero], [zero, zero, one]]
    else:
        raise ValueError(axis)
    return lf.stack([lf.stack(r, axis=0) for r in rows], axis=0)


def camera6(R0, t0, lo, hi):
    """Linear forms (A, tau, beta, P) of the CAMERA6 box lo <= p <= hi, p = (tx,ty,tz,yaw,pitch,roll)."""
    R0 = np.asarray(R0, dtype=np.float64).reshape(3, 3)
    t0 = np.asarray(t0, dtype=np.float64).reshape(3)
    centre, radius, active = _axes(lo, hi)
    P = len(active)
    t = lf.stack([lf.add_const(_param(centre, radius, active, k, P), t0[k]) for k in range(3)])
    yaw = _param(centre, radius, active, 3, P)
    pitch = _param(centre, radius, active, 4, P)
    roll = _param(centre, radius, active, 5, P)
    R = lf.mmul(_rot("y", yaw, P), _rot("x", pitch, P))
    R = lf.mmul(R, _rot("z", roll, P))
    R = lf.mmul(R, lf.const(R0, P))
    beta = lf.const(np.zeros(3), P)
    return R, t, beta, P


def orbit(R0, t0, pivot, phi_lo, phi_hi):
    """Linear forms (A, tau, beta, P) of the ORBIT cell phi in [phi_lo, phi_hi]."""
    R0 = np.asarray(R0, dtype=np.float64).reshape(3, 3)
    t0 = np.asarray(t0, dtype=np.float64).reshape(3)
    pivot = np.asarray(pivot, dtype=np.float64).reshape(3)
    centre, radius, active = _axes([phi_lo], [phi_hi])
    P = len(active)
    phi = _param(centre, radius, active, 0, P)
    A = lf.mmul(lf.const(R0, P), _rot("y", lf.neg(phi), P))
    tau = lf.const(pivot, P)
    beta = lf.const(R0 @ (pivot - t0), P)
    return A, tau, beta, P


def pose_forms(box):
    """Dispatch on a pose-box dict {"model", "R0", "t0", "pivot", "lo", "hi"}."""
    model = box.get("model", CAMERA6)
    if model == CAMERA6:
        return camera6(box["R0"], box["t0"], box["lo"], box["hi"])
    if model == ORBIT:
        return orbit(box["R0"], box["t0"], box["pivot"], box["lo"][0], box["hi"][0])
    raise ValueError(f"unknown pose model {model}")


# --- concrete cameras (used by the concrete renderer) --------------------------------------
def _rot_np(axis, a):
    c, s = np.cos(a), np.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def concrete_camera(box, p):
    """World->camera rotation R and camera centre t at a concrete pose p in the box."""
    model = box.get("model", CAMERA6)
    R0 = np.asarray(box["R0"], dtype=np.float64).reshape(3, 3)
    t0 = np.asarray(box["t0"], dtype=np.float64).reshape(3)
    p = np.asarray(p, dtype=np.float64)
    if model == CAMERA6:
        R = _rot_np("y", p[3]) @ _rot_np("x", p[4]) @ _rot_np("z", p[5]) @ R0
        t = t0 + p[:3]
        return R, t
    if model == ORBIT:
        c = np.asarray(box["pivot"], dtype=np.float64).reshape(3)
        Q = _rot_np("y", p[0])
        return R0 @ Q.T, c + Q @ (t0 - c)
    raise ValueError(model)


def sample_poses(box, n, rng, include_vertices=True):
    """Poses from the box: its centre, (up to 64) vertices, then n uniform samples."""
    lo = np.asarray(box["lo"], dtype=np.float64)
    hi = np.asarray(box["hi"], dtype=np.float64)
    out = [0.5 * (lo + hi)]
    active = np.nonzero(hi > lo)[0]
    if include_vertices and len(active) > 0:
        m = len(active)
        for bits in range(min(1 << m, 64)):
            v = out[0].copy()
            for j, ax in enumerate(active):
                v[ax] = hi[ax] if (bits >> j) & 1 else lo[ax]
            out.append(v)
    for _ in range(n):
        out.append(lo + (hi - lo) * rng.random(lo.shape))
    return out
