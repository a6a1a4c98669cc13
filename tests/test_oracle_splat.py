"""Pins for the oracle's AbstractSplat (Sec. 3.3).

* zero-width box: the bounds collapse to the concrete render (exact special case);
* Theorem 'all': every concrete render at sampled poses (box centre, vertices,
  random points) lies inside the bounds;
* first order: for one Gaussian and a tiny box on one axis, (hi - lo) / (2 r) tends to
  |d pc / d p| measured by finite differences of the concrete renderer;
* BlendInd with interval transmittances encloses brute force over all depth orders
  consistent with Ind and all vertices of the alpha box (tiny N);
* pruning removes only Gaussians whose concrete alpha is below eps at every pose;
* the result does not depend on the tile size.
"""
import itertools

import numpy as np
import pytest

from oracle import pose, render, splat
from paper_2503_00308_amd import synth

RNG = np.random.default_rng(2024)


def _sound(sc, intr, box, res, n_samples, tol=1e-9):
    assert np.all(np.isfinite(res["lo"])) and np.all(np.isfinite(res["hi"]))
    rng = np.random.default_rng(5)
    worst = -np.inf
    for p in pose.sample_poses(box, n_samples, rng):
        img = render.render(sc, intr, box, p)
        worst = max(worst, (res["lo"] - img).max(), (img - res["hi"]).max())
    assert worst <= tol, worst
    return worst


def test_zero_width_collapses_to_concrete_render():
    sc, intr, _, _ = synth.config(1)
    box = synth.camera6_box()
    res = splat.oracle_bounds(sc, intr, box)
    img = render.render(sc, intr, box, np.zeros(6))
    # lo = pc' - E and hi = pc' + E, pc' the render without pruned Gaussians, |pc - pc'| <= E
    E = res["rec"]["E"]
    assert np.abs(res["lo"] - img).max() <= 2 * E + 1e-9
    assert np.abs(res["hi"] - img).max() <= 2 * E + 1e-9


def test_zero_width_rotated_camera_collapses():
    sc = synth.random_scene(30, seed=4)
    intr = synth.intrinsics(24)
    R0 = pose._rot_np("y", 0.1) @ pose._rot_np("x", -0.05)
    box = synth.camera6_box(R0=R0, t0=(0.05, -0.02, 0.1))
    res = splat.oracle_bounds(sc, intr, box)
    img = render.render(sc, intr, box, np.zeros(6))
    assert np.abs(res["lo"] - img).max() <= 2 * res["rec"]["E"] + 1e-9
    assert np.abs(res["hi"] - img).max() <= 2 * res["rec"]["E"] + 1e-9


def test_sound_config1_translation():
    sc, intr, box, _ = synth.config(1)
    res = splat.oracle_bounds(sc, intr, box)
    _sound(sc, intr, box, res, 64)


def test_sound_translation_3d_small():
    sc = synth.random_scene(48, seed=11)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=0.1)
    res = splat.oracle_bounds(sc, intr, box)
    _sound(sc, intr, box, res, 48)


@pytest.mark.parametrize("seed", [0, 1])
def test_sound_rotation_6dof_small(seed):
    sc = synth.box_surface_scene(200, n_boxes=3, seed=seed)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=0.03, drot=np.deg2rad(0.7))
    res = splat.oracle_bounds(sc, intr, box)
    _sound(sc, intr, box, res, 40)


def test_sound_orbit_cell():
    sc = synth.box_surface_scene(150, n_boxes=3, seed=2)
    intr = synth.intrinsics(32)
    cells = synth.orbit_cells(8, 30.0, seed=1)
    for cell in cells[:2]:
        res = splat.oracle_bounds(sc, intr, cell)
        _sound(sc, intr, cell, res, 24)


@pytest.mark.parametrize("axis", range(6))
def test_first_order_width_matches_derivative(axis):
    """N = 1, T = 1: pc = c a(p); the bound width per unit radius tends to |c da/dp|."""
    sc = {"mean": np.array([[0.15, -0.1, 3.5]], np.float32),
          "cov_factor": np.array([[[0.12, 0.02, 0.0], [0.01, 0.09, 0.03], [0.0, 0.02, 0.1]]], np.float32),
          "opacity": np.array([0.8], np.float32), "rgb": np.array([[1.0, 0.5, 0.25]], np.float32)}
    intr = synth.intrinsics(32)
    r = 1e-6
    half = np.zeros(6)
    half[axis] = r
    box = {"model": 0, "R0": np.eye(3), "t0": np.zeros(3), "pivot": np.zeros(3), "lo": -half, "hi": half.copy()}
    res = splat.oracle_bounds(sc, intr, box, {"cull_budget": 1e-30})
    h = 1e-5
    pp = np.zeros(6)
    pm = np.zeros(6)
    pp[axis] = h
    pm[axis] = -h
    deriv = (render.render(sc, intr, box, pp) - render.render(sc, intr, box, pm)) / (2 * h)
    width = (res["hi"] - res["lo"]) / (2 * r)
    sel = np.abs(deriv) > 1e-3
    assert sel.sum() > 20
    np.testing.assert_allclose(width[sel], np.abs(deriv[sel]), rtol=2e-3, atol=1e-4)


def _brute_force_blend(al, au, c, ind):
    """min / max of BlendSort over total orders consistent with ind and alpha-box vertices."""
    n = len(al)
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for perm in itertools.permutations(range(n)):
        pos = np.empty(n, int)
        pos[list(perm)] = np.arange(n)
        # j may be in front of i only if Ind_ij is 1 or unknown; it must be if Ind_ij is 1
        ok = True
        for i in range(n):
            for j in range(n):
                if i != j and ind[i, j] == 1 and not pos[j] < pos[i]:
                    ok = False
                if i != j and ind[i, j] == 0 and pos[j] < pos[i]:
                    ok = False
        if not ok:
            continue
        for bits in range(1 << n):
            a = np.where([(bits >> k) & 1 for k in range(n)], au, al)
            T = 1.0
            pc = np.zeros(3)
            for k in perm:
                pc += T * a[k] * c[k]
                T *= 1 - a[k]
            lo = np.minimum(lo, pc)
            hi = np.maximum(hi, pc)
    return lo, hi


def test_blendind_interval_encloses_brute_force_orders():
    for trial in range(40):
        n = int(RNG.integers(2, 6))
        al = RNG.uniform(0, 0.6, n)
        au = np.minimum(1.0, al + RNG.uniform(0, 0.4, n))
        c = RNG.uniform(0, 1, (n, 3))
        # a random consistent three-valued Ind: depth intervals on a line
        dc = RNG.uniform(0, 3, n)
        dr = RNG.uniform(0, 0.6, n)
        ind = np.zeros((n, n), np.int8)
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                lo_ = (dc[i] - dr[i]) - (dc[j] + dr[j])
                hi_ = (dc[i] + dr[i]) - (dc[j] - dr[j])
                ind[i, j] = 1 if lo_ > 0 else (0 if hi_ <= 0 else 2)
        P = 0
        alo_f = al[:, None, None] * np.ones((n, 1, 1))
        aup_f = au[:, None, None] * np.ones((n, 1, 1))
        lo, hi = splat.blend(al[:, None], au[:, None], alo_f, aup_f, c, ind, 0.0)
        blo, bhi = _brute_force_blend(al, au, c, ind)
        assert np.all(lo[0] <= blo + 1e-12), (lo, blo)
        assert np.all(bhi <= hi[0] + 1e-12), (hi, bhi)


def test_pruned_gaussians_are_below_eps_at_all_poses():
    sc = synth.random_scene(80, seed=8)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=0.08, drot=np.deg2rad(0.5))
    rec = splat.gaussian_forms(sc, intr, box, {"cull_budget": 1e-3})
    cols, rows = np.meshgrid(np.arange(32), np.arange(32), indexing="xy")
    ux32, uy32 = splat.pixel_coords32(intr, cols.ravel(), rows.ravel())
    keep = splat.kept_mask(rec, np.arange(80), ux32, uy32)
    assert (~keep).sum() > 1000
    rng = np.random.default_rng(3)
    for p in pose.sample_poses(box, 20, rng):
        R, t = pose.concrete_camera(box, p)
        proj = render.project(sc, intr, R, t)
        ux, uy = render.pixel_grid(intr)
        a = render.alpha(sc, intr, proj, ux, uy, 0.01)
        assert np.all(a[~keep] <= rec["eps_cull"] * (1 + 2.0 ** -10))


def test_tile_size_does_not_change_result():
    sc = synth.random_scene(60, seed=9)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=(0.05, 0.02, 0.0), drot=(0.0, 0.01, 0.0))
    ref = splat.oracle_bounds(sc, intr, box, {"tile": 16})
    for ts in (8, 32):
        r = splat.oracle_bounds(sc, intr, box, {"tile": ts})
        np.testing.assert_allclose(r["lo"], ref["lo"], atol=1e-12)
        np.testing.assert_allclose(r["hi"], ref["hi"], atol=1e-12)
        assert np.array_equal(r["pairs"], ref["pairs"])


def test_translation_only_ind_is_exact():
    """Without rotation A_z is constant, so every Ind entry is decided (no unknowns)."""
    sc = synth.random_scene(50, seed=12)
    intr = synth.intrinsics(16)
    rec = splat.gaussian_forms(sc, intr, synth.camera6_box(dt=0.1))
    ind, border = splat.ind_matrix(rec, np.arange(50))
    assert not np.any(ind == 2) and not border.any()
    d = sc["mean"][:, 2].astype(np.float64)
    assert np.array_equal(ind == 1, d[:, None] > d[None, :])


def test_exp_chord_slope_wide_intervals_finite():
    """The chord slope stays finite for very wide exponent intervals (regression)."""
    from oracle import lf
    xlo = np.array([-2000.0, -800.0, -50.0, -1e-9, -3.0])
    xhi = np.array([0.0, -700.0, -49.0, 0.0, -3.0])
    k = lf.exp_slope(xlo, xhi)
    assert np.all(np.isfinite(k))
    dx = xhi - xlo
    quotient = (np.exp(xhi) - np.exp(xlo)) / np.where(dx > 0, dx, 1.0)
    taylor = np.exp(xlo) * (1 + dx / 2 + dx * dx / 6)        # for tiny dx, no cancellation
    ref = np.where(dx == 0, np.exp(xlo), np.where(dx < 1e-3, taylor, quotient))
    np.testing.assert_allclose(k, ref, rtol=1e-9, atol=1e-300)
