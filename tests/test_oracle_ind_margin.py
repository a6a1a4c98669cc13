"""Pin of the literal depth-difference bound's margin (splat.IND_MARGIN = 1e-10).

Ind decides on the literal bound Add(d[i], -d[j]) of two depth forms (Alg. BlendInd's
difference step) only beyond a margin, so that rounding noise in the forms cannot decide
an exact tie (Ind(0) = 0).  The margin must exceed the rounding of that bound's own
evaluation by orders of magnitude at the workloads' scales.  Checked here:

* the literal bounds of every pair of a rotating box's Gaussians, evaluated in FP64 as
  ind_matrix does and in extended precision from the same forms, differ by less than
  1e-4 of the margin (so the margin is not a tuning knob of the decisions it separates);
* two Gaussians whose depths are equal at every pose of a yaw box (they differ only
  along the rotation axis) are never ordered, in either direction: Ind = 0 both ways
  (Ind(0) = 0), and the pair is not borderline (an exact tie).
"""
import numpy as np

from oracle import lf, splat
from paper_2503_00308_amd import synth


def test_margin_is_far_above_the_literal_bounds_rounding():
    scene = synth.box_surface_scene(400, n_boxes=5, seed=14)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=0.02, drot=np.deg2rad(0.8))
    rec = splat.gaussian_forms(scene, intr, box)
    idx = np.arange(min(300, rec["N"]))
    d = rec["d"][idx]
    lit = lf.sub(d.expand(-1), d.expand(0))
    lo64, hi64 = lit.bounds()
    L = np.asarray(d.lo, np.longdouble)
    U = np.asarray(d.up, np.longdouble)
    llo = L[:, None, :] - U[None, :, :]
    lup = U[:, None, :] - L[None, :, :]
    lo_x = llo[..., -1] - np.abs(llo[..., :-1]).sum(-1)
    hi_x = lup[..., -1] + np.abs(lup[..., :-1]).sum(-1)
    err = max(float(np.abs(lo64 - lo_x).max()), float(np.abs(hi64 - hi_x).max()))
    scale = float(np.abs(np.asarray(d.up)[:, -1]).max())
    print(f"literal bound rounding {err:.3e} at depths up to {scale:.1f}; margin {splat.IND_MARGIN:.0e}")
    assert 0.0 < scale and err < 1e-4 * splat.IND_MARGIN


def test_exact_depth_tie_is_never_ordered():
    # two Gaussians one above the other: the same depth at every yaw
    mean = np.array([[0.3, -0.4, 5.0], [0.3, 0.4, 5.0]])
    scene = synth._pack(mean, np.stack([np.eye(3)] * 2), np.full((2, 3), 0.5), np.array([0.7, 0.7]),
                        np.array([[1.0, 0.3, 0.3], [0.3, 0.3, 1.0]]))
    intr = synth.intrinsics(16)
    box = synth.camera6_box()
    box["lo"][3], box["hi"][3] = np.deg2rad(-2.0), np.deg2rad(2.0)
    rec = splat.gaussian_forms(scene, intr, box)
    ind, border = splat.ind_matrix(rec, np.arange(2))
    assert ind[0, 1] == 0 and ind[1, 0] == 0
    assert not border.any()
