"""Pins for the oracle's adaptive refinement of a pose box (Sec. 3.1: divide the input
range where MatrixInv's convergence assertion fails; Sec. 4.2: bounds of subsets of the
cameras, united).

The leaves must tile the box, a box with nothing flagged must be its own leaf, the cell
budget must hold, refinement must remove the failures when the budget allows, and the
united bounds must enclose concrete renders sampled from the box (the soundness theorem).
"""
import numpy as np

from oracle import pose, refine, render, splat
from paper_2503_00308_amd import synth

SCENE = synth.box_surface_scene(200, n_boxes=4, seed=3)
INTR = synth.intrinsics(32)


def orbit_box(deg):
    a = np.deg2rad(deg)
    return {"model": pose.ORBIT, "R0": np.eye(3), "t0": np.zeros(3), "pivot": np.array([0.0, 0.0, 4.0]),
            "lo": np.array([-a, 0, 0, 0, 0, 0], np.float64), "hi": np.array([a, 0, 0, 0, 0, 0], np.float64)}


def _inside(box, p):
    return bool(np.all(p >= box["lo"]) and np.all(p <= box["hi"]))


def _strictly_inside(box, p, axes):
    return all(box["lo"][a] < p[a] < box["hi"][a] for a in axes)


def test_leaves_tile_the_box():
    """Leaves lie in the box, their volumes add up to the box's, and every sampled pose
    lies in at least one leaf and strictly inside at most one."""
    box = synth.camera6_box(dt=(0.05, 0.0, 0.05), drot=(np.deg2rad(2), np.deg2rad(2), 0.0))
    leaves = refine.refine(SCENE, INTR, box, 16)
    assert 1 < len(leaves) <= 16
    axes = refine.active_axes(box)
    assert axes == [0, 2, 3, 4]
    vol = lambda b: float(np.prod([b["hi"][a] - b["lo"][a] for a in axes]))
    assert abs(sum(vol(c) for c in leaves) - vol(box)) <= 1e-12 * vol(box)
    for c in leaves:
        assert np.all(c["lo"] >= box["lo"]) and np.all(c["hi"] <= box["hi"])
    rng = np.random.default_rng(7)
    for p in pose.sample_poses(box, 300, rng):
        assert sum(_inside(c, p) for c in leaves) >= 1
        assert sum(_strictly_inside(c, p, axes) for c in leaves) <= 1


def test_one_axis_leaves_chain_and_cuts_are_midpoints():
    """On a one-axis box the leaves are intervals that chain from lo to hi, and each
    leaf's width is the box width over a power of two (bisection at midpoints)."""
    box = orbit_box(3.0)
    leaves = refine.refine(SCENE, INTR, box, 16)
    iv = sorted((float(c["lo"][0]), float(c["hi"][0])) for c in leaves)
    assert iv[0][0] == box["lo"][0] and iv[-1][1] == box["hi"][0]
    for (a0, b0), (a1, b1) in zip(iv, iv[1:]):
        assert b0 == a1
    W = float(box["hi"][0] - box["lo"][0])
    for a, b in iv:
        k = np.log2(W / (b - a))
        assert abs(k - round(k)) < 1e-9


def test_nothing_flagged_gives_the_box_itself():
    """A translation box over round Gaussians has no MatrixInv failure: one leaf, the box."""
    scene = synth.random_scene(60, seed=11)
    box = synth.camera6_box(dt=(0.02, 0.0, 0.0))
    fb, wild = refine.flagged_counts(scene, INTR, box)
    assert fb == 0 and wild == 0
    leaves = refine.refine(scene, INTR, box, 64)
    assert len(leaves) == 1
    assert np.array_equal(leaves[0]["lo"], box["lo"]) and np.array_equal(leaves[0]["hi"], box["hi"])


def test_budget_caps_the_cells():
    box = orbit_box(3.0)
    assert refine.flagged_counts(SCENE, INTR, box)[0] > 0
    assert len(refine.refine(SCENE, INTR, box, 1)) == 1
    two = refine.refine(SCENE, INTR, box, 2)
    assert len(two) == 2
    assert two[0]["hi"][0] == two[1]["lo"][0] == 0.0
    assert len(refine.refine(SCENE, INTR, box, 4)) == 4


def test_refinement_removes_the_failures():
    """With room enough, every leaf passes MatrixInv's assertion for every Gaussian kept
    in the image, and the whole box does not."""
    box = orbit_box(3.0)
    assert refine.flagged_counts(SCENE, INTR, box)[0] > 0
    leaves = refine.refine(SCENE, INTR, box, 64)
    assert 1 < len(leaves) < 64
    assert all(refine.flagged_counts(SCENE, INTR, c)[0] == 0 for c in leaves)
    # the near-plane criterion changes nothing where no Gaussian straddles it
    assert [c["lo"][0] for c in refine.refine(SCENE, INTR, box, 64, near=True)] == [c["lo"][0] for c in leaves]


def test_refined_bounds_enclose_concrete_renders_and_tighten():
    """Soundness (Theorem in Sec. 3.3) of the united bounds at sampled poses, and the
    refined bounds no wider on average than the whole box's."""
    box = orbit_box(3.0)
    lo, hi, leaves = refine.refined_bounds(SCENE, INTR, box, 16)
    whole = splat.oracle_bounds(SCENE, INTR, box)
    rng = np.random.default_rng(3)
    worst = -np.inf
    for p in pose.sample_poses(box, 12, rng):
        img = render.render(SCENE, INTR, box, p)
        worst = max(worst, (lo - img).max(), (img - hi).max())
    assert worst <= 1e-9
    assert (hi - lo).mean() <= (whole["hi"] - whole["lo"]).mean()


def near_scene():
    """40 random Gaussians at depth 3-5 and one whose mean sits at depth 0.02."""
    s = synth.random_scene(40, seed=5)
    t = synth.random_scene(1, seed=6)
    t["mean"][0] = (0.05, -0.03, 0.02)
    return {k: np.concatenate([s[k], t[k]]) for k in s}


def test_near_plane_criterion_isolates_the_crossing():
    """With the camera moving along z by tz in [-0.04, 0.04], the near Gaussian's depth is
    m - tz (m its stored depth, float32 0.02): over a cell [lo, hi] of tz it straddles
    z_near = 0.01 exactly when lo < m - 0.01 <= hi.  Refining on the near-plane criterion
    alone bisects toward that point, so exactly one leaf holds it; the MatrixInv
    criterion alone leaves the box whole."""
    scene = near_scene()
    box = synth.camera6_box(dt=(0.0, 0.0, 0.04))
    assert refine.flagged_counts(scene, INTR, box) == (0, 1)
    assert len(refine.refine(scene, INTR, box, 6)) == 1
    leaves = refine.refine(scene, INTR, box, 6, near=True, matinv=False)
    assert len(leaves) == 6
    t_cross = float(np.float32(0.02)) - 0.01
    hits = 0
    for c in leaves:
        lo, hi = float(c["lo"][2]), float(c["hi"][2])
        straddles = refine.flagged_counts(scene, INTR, c)[1] == 1
        assert straddles == (lo < t_cross <= hi), (lo, hi)
        hits += straddles
    assert hits == 1


def test_ind_criterion_cuts_only_cells_that_hold_the_order_swap():
    """Two Gaussians mirrored across the optical axis swap their depth order at yaw 0
    (depth -sin(yaw) x + cos(yaw) z).  Refining a yaw box [-1, 3] degrees on the Ind
    criterion alone cuts only cells whose closure holds yaw 0 (there the pair's Ind is
    undecided, elsewhere decided; a cut lands within rounding of 0, where the depth
    difference is far too small to decide), so the leaves around 0 shrink and the others
    are not cut again; MatrixInv alone leaves the box whole."""
    mean = np.array([[0.5, 0.0, 5.0], [-0.5, 0.0, 5.0]])
    scene = synth._pack(mean, np.stack([np.eye(3)] * 2), np.full((2, 3), 0.6), np.array([0.6, 0.6]),
                        np.array([[1.0, 0.2, 0.2], [0.2, 0.2, 1.0]]))
    intr = synth.intrinsics(8)
    box = synth.camera6_box()
    box["lo"][3], box["hi"][3] = np.deg2rad(-1.0), np.deg2rad(3.0)
    assert len(refine.refine(scene, intr, box, 8)) == 1
    leaves = refine.refine(scene, intr, box, 8, matinv=False, ind=True)
    assert len(leaves) == 8
    for c in leaves:
        lo, hi = float(c["lo"][3]), float(c["hi"][3])
        holds_swap = lo <= 1e-12 and hi >= -1e-12   # the midpoints land within rounding of 0
        assert (splat.ind_uncertain_count(scene, intr, c)[0] > 0) == holds_swap, (lo, hi)
        if holds_swap:
            assert hi - lo <= np.deg2rad(4.0) / 8
    m1 = 0.5 * (float(box["lo"][3]) + float(box["hi"][3]))   # the first cut
    assert any(float(c["lo"][3]) == m1 and float(c["hi"][3]) == float(box["hi"][3]) for c in leaves)
