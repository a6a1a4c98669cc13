"""Pins for the oracle's sets of scenes (Sec. 4.6: colour, mean and opacity perturbations).

* a set of zero width (no moved mean, colour and opacity intervals of zero width, a
  scene variable with no Gaussian on it) gives exactly the plain scene's bounds;
* a camera fixed and only colours uncertain: the bounds are the concrete renders with
  the lower and the upper colours (pc is linear in every colour with non-negative
  weights: a closed form);
* one Gaussian, camera fixed, only its opacity uncertain: the bounds are the renders at
  the two ends of the opacity interval (pc = o a' c, monotone in o);
* Theorem 'all' over scenes: concrete renders at sampled (pose, scene) points, the
  vertices of the scene box and of the colour / opacity intervals included, lie inside;
* first order: one Gaussian moved along an axis by s in [-r, r], tiny r: the width per
  unit radius tends to |d pc / d s| by finite differences;
* Ind with moved means: every decided entry equals the concrete depth order at sampled
  scene variables (the identity bound is not used for moved Gaussians).
"""
import numpy as np
import pytest

from oracle import pose, render, splat
from paper_2503_00308_amd import synth

E2 = 2 * 1e-7 * (1 + 2.0 ** -10) + 1e-9


def _renders(scene, intr, box, n, rng, vertices=True):
    """Concrete renders at sampled poses and scenes of the set."""
    out = []
    lo = np.asarray(scene.get("set_lo", []), dtype=np.float64)
    hi = np.asarray(scene.get("set_hi", []), dtype=np.float64)
    poses = pose.sample_poses(box, n, rng, include_vertices=vertices)
    for k, p in enumerate(poses):
        if len(lo):
            s = lo + (hi - lo) * (rng.random(len(lo)) if k % 3 else (k // 3) % 2)
        else:
            s = None
        ng = len(scene["opacity"])
        if k % 4 == 0:
            t_rgb, t_o = 0.0, 0.0
        elif k % 4 == 1:
            t_rgb, t_o = 1.0, 1.0
        else:
            t_rgb, t_o = rng.random(ng), rng.random(ng)
        out.append(render.render(render.instantiate(scene, s, t_rgb, t_o), synth.intrinsics(intr["width"]), box, p))
    return out


def test_zero_width_set_equals_plain_scene():
    sc = synth.random_scene(40, seed=3)
    intr = synth.intrinsics(24)
    box = synth.camera6_box(dt=0.05, drot=(0.0, 0.01, 0.0))
    s = dict(sc)
    s["rgb_hi"] = sc["rgb"].copy()
    s["opacity_lo"] = sc["opacity"].copy()
    s["set_lo"], s["set_hi"] = np.array([0.0]), np.array([0.5])
    s["mean_var"] = np.full(40, -1, np.int32)
    s["mean_dir"] = np.zeros((40, 3), np.float32)
    a = splat.oracle_bounds(s, intr, box)
    b = splat.oracle_bounds(sc, intr, box)
    assert a["rec"]["P"] == b["rec"]["P"] + 1
    np.testing.assert_array_equal(a["lo"], b["lo"])
    np.testing.assert_array_equal(a["hi"], b["hi"])


def test_colour_set_fixed_camera_is_exact():
    sc = synth.perturbed_scene(synth.random_scene(50, seed=4), ("colour",), frac=0.5)
    intr = synth.intrinsics(24)
    box = synth.camera6_box()
    res = splat.oracle_bounds(sc, intr, box)
    lo_img = render.render(render.instantiate(sc, None, 0.0), intr, box, np.zeros(6))
    hi_img = render.render(render.instantiate(sc, None, 1.0), intr, box, np.zeros(6))
    assert np.abs(hi_img - lo_img).max() > 0.05
    assert np.abs(res["lo"] - lo_img).max() <= E2
    assert np.abs(res["hi"] - np.minimum(hi_img, 1.0)).max() <= E2


def test_opacity_set_single_gaussian_is_exact():
    sc = {"mean": np.array([[0.1, -0.05, 3.0]], np.float32),
          "cov_factor": np.array([[[0.3, 0.02, 0.0], [0.01, 0.25, 0.03], [0.0, 0.02, 0.2]]], np.float32),
          "opacity": np.array([0.7], np.float32), "rgb": np.array([[1.0, 0.5, 0.25]], np.float32),
          "opacity_lo": np.array([0.2], np.float32)}
    intr = synth.intrinsics(24)
    box = synth.camera6_box()
    res = splat.oracle_bounds(sc, intr, box)
    lo_img = render.render(render.instantiate(sc, None, 0.0, 0.0), intr, box, np.zeros(6))
    hi_img = render.render(render.instantiate(sc, None, 0.0, 1.0), intr, box, np.zeros(6))
    assert np.abs(res["lo"] - lo_img).max() <= E2
    assert np.abs(res["hi"] - hi_img).max() <= E2


@pytest.mark.parametrize("kinds,box", [
    (("colour",), synth.camera6_box(dt=0.03)),
    (("opacity",), synth.camera6_box(dt=0.03)),
    (("mean",), synth.camera6_box()),
    (("mean",), synth.camera6_box(dt=0.02, drot=np.deg2rad(0.5))),
    (("colour", "mean", "opacity"), synth.camera6_box(dt=(0.02, 0.0, 0.02))),
])
def test_sound_over_scenes_and_poses(kinds, box):
    base = synth.box_surface_scene(160, n_boxes=3, seed=5)
    sc = synth.perturbed_scene(base, kinds, frac=0.4, shift=0.15)
    intr = synth.intrinsics(28)
    res = splat.oracle_bounds(sc, intr, box)
    rng = np.random.default_rng(7)
    worst = -np.inf
    for img in _renders(sc, intr, box, 24, rng):
        worst = max(worst, (res["lo"] - img).max(), (img - res["hi"]).max())
    assert worst <= 1e-9, worst
    # a set that contains the plain scene (colours raised, means moved from s = 0) has
    # wider bounds than the plain scene; the opacity set (0.1 o + [0, 0.1]) does not
    # contain it
    if "opacity" not in kinds:
        plain = splat.oracle_bounds(base, intr, box)
        assert (res["hi"] - res["lo"]).mean() > (plain["hi"] - plain["lo"]).mean()


@pytest.mark.parametrize("axis", range(3))
def test_first_order_width_of_a_moved_mean(axis):
    r = 1e-6
    direction = np.zeros(3, np.float32)
    direction[axis] = 1.0
    sc = {"mean": np.array([[0.15, -0.1, 3.5]], np.float32),
          "cov_factor": np.array([[[0.12, 0.02, 0.0], [0.01, 0.09, 0.03], [0.0, 0.02, 0.1]]], np.float32),
          "opacity": np.array([0.8], np.float32), "rgb": np.array([[1.0, 0.5, 0.25]], np.float32),
          "set_lo": np.array([-r]), "set_hi": np.array([r]), "mean_var": np.array([0], np.int32),
          "mean_dir": direction[None, :]}
    intr = synth.intrinsics(32)
    box = synth.camera6_box()
    res = splat.oracle_bounds(sc, intr, box, {"cull_budget": 1e-30})
    h = 1e-5
    plus = render.render(render.instantiate(sc, [h]), intr, box, np.zeros(6))
    minus = render.render(render.instantiate(sc, [-h]), intr, box, np.zeros(6))
    deriv = (plus - minus) / (2 * h)
    width = (res["hi"] - res["lo"]) / (2 * r)
    sel = np.abs(deriv) > 1e-3
    assert sel.sum() > 20
    np.testing.assert_allclose(width[sel], np.abs(deriv[sel]), rtol=2e-3, atol=1e-4)


def test_ind_with_moved_means_agrees_with_concrete_order():
    base = synth.random_scene(80, seed=6)
    sc = synth.perturbed_scene(base, ("mean",), frac=0.5, shift=0.6)
    # move along the depth axis so that the order really changes
    sc["mean_dir"] = np.where(sc["mean_var"][:, None] >= 0, np.array([[0.0, 0.0, 1.0]], np.float32), 0.0)
    box = synth.camera6_box(drot=(0.0, 0.004, 0.0))
    rec = splat.gaussian_forms(sc, synth.intrinsics(16), box)
    idx = np.arange(80)
    ind, _ = splat.ind_matrix(rec, idx)
    assert (ind == 2).any() and (ind != 2).mean() > 0.5
    rng = np.random.default_rng(2)
    for k, p in enumerate(pose.sample_poses(box, 30, rng)):
        s = np.array([rng.random() if k % 3 else float(k % 2)])
        R, t = pose.concrete_camera(box, p)
        uw = render.instantiate(sc, s)["mean"]
        d = ((uw - t) @ R.T)[:, 2]
        concrete = (d[:, None] - d[None, :]) > 0
        np.fill_diagonal(concrete, False)
        assert np.all(concrete[ind == 1]) and not np.any(concrete[ind == 0])
