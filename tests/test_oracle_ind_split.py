"""Pins of the oracle's count of undecided depth-order tests (splat.ind_uncertain_count),
the quantity that drives refinement where Ind is uncertain (Sec. 3.2: Ind(d_i - d_j) is
piecewise constant, so it is tight on every part of the pose domain where d_i - d_j
keeps its sign).

* A box that only translates the camera leaves every Ind decided: translations cancel in
  d_i - d_j (checked on the Ind matrix itself, not through the function's early return).
* Two Gaussians mirrored across the optical axis swap their depth order exactly at yaw 0:
  a yaw box that contains 0 counts both orders, boxes on either side count none.
* Every pair sharing a tile list whose concrete depth order differs between two sampled
  poses of the box is counted.
"""
import numpy as np

from oracle import pose, splat
from paper_2503_00308_amd import synth


def _tile_lists(scene, intr, box, tile=8):
    rec = splat.gaussian_forms(scene, intr, box, {"tile": tile})
    W, H = intr["width"], intr["height"]
    out = []
    for ty in range((H + tile - 1) // tile):
        for tx in range((W + tile - 1) // tile):
            x0, y0 = tx * tile, ty * tile
            out.append(splat.tile_candidates(rec, intr, x0, min(x0 + tile, W), y0, min(y0 + tile, H)))
    return rec, out


def test_translation_box_leaves_every_ind_decided():
    scene = synth.random_scene(150, seed=4)
    intr = synth.intrinsics(24)
    box = synth.camera6_box(dt=(0.05, 0.03, 0.04))
    rec, lists = _tile_lists(scene, intr, box)
    undecided = sum(int((splat.ind_matrix(rec, idx)[0] == 2).sum()) for idx in lists if len(idx) > 1)
    assert undecided == 0
    assert sum(len(i) for i in lists) > 300          # the lists are not trivially empty
    assert splat.ind_uncertain_count(scene, intr, box) == (0, 0)


def _mirrored_pair():
    mean = np.array([[0.5, 0.0, 5.0], [-0.5, 0.0, 5.0]])
    R = np.stack([np.eye(3), np.eye(3)])
    scales = np.full((2, 3), 0.6)
    return synth._pack(mean, R, scales, np.array([0.6, 0.6]), np.array([[1.0, 0.2, 0.2], [0.2, 0.2, 1.0]]))


def test_mirrored_pair_is_undecided_exactly_where_its_order_swaps():
    scene = _mirrored_pair()
    intr = synth.intrinsics(8)
    deg = np.deg2rad

    def yaw_box(lo, hi):
        b = synth.camera6_box()
        b["lo"][3], b["hi"][3] = deg(lo), deg(hi)
        return b

    # one tile holding both Gaussians
    rec, lists = _tile_lists(scene, intr, yaw_box(-1.0, 1.0))
    assert len(lists) == 1 and len(lists[0]) == 2
    assert splat.ind_uncertain_count(scene, intr, yaw_box(-1.0, 1.0))[0] == 2
    assert splat.ind_uncertain_count(scene, intr, yaw_box(0.2, 1.0))[0] == 0
    assert splat.ind_uncertain_count(scene, intr, yaw_box(-1.0, -0.2))[0] == 0
    # the concrete depths do swap at yaw 0 (depth = -sin(yaw) x + cos(yaw) z)
    for y, sign in ((deg(0.5), -1.0), (deg(-0.5), 1.0)):
        R, t = pose.concrete_camera(yaw_box(-1.0, 1.0), [0, 0, 0, y, 0, 0])
        d = ((np.asarray(scene["mean"], np.float64) - t) @ R.T)[:, 2]
        assert np.sign(d[0] - d[1]) == sign


def test_every_order_flip_at_sampled_poses_is_counted():
    scene = synth.box_surface_scene(200, n_boxes=4, seed=6)
    intr = synth.intrinsics(24)
    box = synth.camera6_box(dt=0.02, drot=(np.deg2rad(1.5), np.deg2rad(1.0), 0.0))
    rec, lists = _tile_lists(scene, intr, box)
    uw = np.asarray(scene["mean"], dtype=np.float64)
    rng = np.random.default_rng(11)
    depths = []
    for p in pose.sample_poses(box, 40, rng):
        R, t = pose.concrete_camera(box, p)
        depths.append(((uw - t) @ R.T)[:, 2])
    depths = np.array(depths)                          # (poses, n)
    flips = 0
    for idx in lists:
        if len(idx) < 2:
            continue
        diff = depths[:, idx, None] - depths[:, None, idx]
        flip = (diff > 0).any(axis=0) & (diff < 0).any(axis=0)
        ind = splat.ind_matrix(rec, idx)[0]
        assert np.all(ind[flip] == 2)
        flips += int(flip.sum())
    count, border = splat.ind_uncertain_count(scene, intr, box)
    assert flips > 0 and count >= flips
    assert border <= count // 10 + 2                  # borderline pairs are rare
