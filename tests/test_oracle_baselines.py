"""Pins for the oracle's precision baselines (Sec. 3.1 Example 'matinv-vs-direct', Sec. 3.2
Example '3g-scene') and for three details of the oracle's AbstractSplat.

* Div (Table "Bounds for operations Exp, Div and Ind"): the printed tangent / chord
  planes, sound on dense samples, exact at zero width;
* the adjugate inverse: exact at zero width (closed form), encloses the inverse of every
  matrix of random interval sets, encloses the exact hull of Example 1 and is wider than
  MatrixInv there (the paper's ranking: adjugate 1.22 against MatrixInv 0.70);
* the abstract BlendSort: equal to the concrete BlendSort when the depth order and the
  alphas are fixed; encloses brute force over sampled depths (ties included) and all
  alpha vertices on tiny inputs; on a three-Gaussian scene under a translation box (an
  analogue of Example '3g-scene', whose scene the paper does not give) it is sound and
  wider than BlendInd, which is the paper's claim;
* Ind under rotation: every decided entry of the oracle's Ind matrix equals the concrete
  depth order at sampled poses of six-axis and orbit boxes;
* pruning: the float32 keep decision keeps every pair whose FP64 footprint bound exceeds
  eps (1 + 2^-10), the per-pair share of the widening E;
* MatrixInv bounded backward (CROWN-style, the paper's bound engine): encloses the inverse
  relationally, exact at zero width, and on Example 1 lies between the exact hull and the
  forward-mode width, within 0.01 of the paper's 0.70; sound in the whole pipeline.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import lf, pose, render, splat
from oracle.matinv import adjugate_inv, inv2, interval_matrix, matrix_inv
from paper_2503_00308_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(99)


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --- Div ---------------------------------------------------------------------------------
@pytest.mark.parametrize("tangent", ["lo", "hi"])
def test_recip_planes_sound_and_exact(tangent):
    for _ in range(200):
        a = RNG.uniform(0.05, 3.0)
        b = a + RNG.uniform(0.0, 3.0)
        x = lf.variable(0.5 * (a + b), 0.5 * (b - a), 0, 1)
        r = lf.recip(x, tangent)
        xs = np.linspace(a, b, 101)
        es = (xs - 0.5 * (a + b)) / max(0.5 * (b - a), 1e-300)
        for xv, ev in zip(xs, es):
            lo, up = r.eval([ev])
            assert lo <= 1.0 / xv + 1e-12 and 1.0 / xv <= up + 1e-12
        # the table's planes at the ends: the chord meets 1/x at both ends, the tangent at t
        t = a if tangent == "lo" else b
        lo_t, _ = r.eval([(t - 0.5 * (a + b)) / max(0.5 * (b - a), 1e-300)])
        assert lo_t == pytest.approx(1.0 / t, rel=1e-12)
        _, up_a = r.eval([-1.0])
        _, up_b = r.eval([1.0])
        if b > a:
            assert up_a == pytest.approx(1.0 / a, rel=1e-12) and up_b == pytest.approx(1.0 / b, rel=1e-12)
    z = lf.const(2.5, 0)
    r = lf.recip(z)
    assert r.lo[-1] == pytest.approx(0.4, rel=1e-15) and r.up[-1] == pytest.approx(0.4, rel=1e-15)


# --- adjugate inverse ----------------------------------------------------------------------
def test_adjugate_zero_width_is_the_inverse():
    for _ in range(20):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.2 * np.eye(2)
        A, ok = adjugate_inv(lf.const(M, 0))
        assert ok
        np.testing.assert_allclose(A.lo[..., 0], np.linalg.inv(M), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(A.up[..., 0], np.linalg.inv(M), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("tangent", ["lo", "hi"])
def test_adjugate_encloses_inverse(tangent):
    for _ in range(30):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.5 * np.eye(2)
        rad = np.abs(RNG.normal(0, 0.05, (2, 2)))
        rad = 0.5 * (rad + rad.T)
        X = interval_matrix(M - rad, M + rad, symmetric=True)
        A, ok = adjugate_inv(X, tangent)
        if not ok:
            continue
        for _ in range(50):
            e = RNG.uniform(-1, 1, 3)
            lo, up = A.eval(e)
            Xe = 0.5 * (X.lo + X.up) @ np.concatenate([e, [1.0]])
            Xi = np.linalg.inv(Xe)
            assert np.all(lo <= Xi + 1e-12) and np.all(Xi <= up + 1e-12)


def test_adjugate_not_provably_positive_determinant_reported():
    X = interval_matrix(np.array([[0.1, -0.5], [-0.5, 0.1]]), np.array([[2.0, 0.5], [0.5, 2.0]]), symmetric=True)
    _, ok = adjugate_inv(X)
    assert not ok


def test_example1_adjugate_wider_than_matrixinv():
    """Example 'matinv-vs-direct': the adjugate bounds enclose the exact hull (0.66) and are
    wider than MatrixInv's, with either tangent of the Div relaxation."""
    g = _load("example1_matinv.json")
    lo, hi = np.array(g["X_lo"]), np.array(g["X_hi"])
    X = interval_matrix(lo, hi, symmetric=True)
    conic, ok, _ = matrix_inv(X, 8)
    assert ok
    clo, chi = conic.bounds()
    w_matinv = np.linalg.norm(chi - clo)
    # exact hull of the inverse by brute force over the box
    grid = [np.linspace(lo[i][j], hi[i][j], 61) for i, j in ((0, 0), (0, 1), (1, 1))]
    Am, Bm, Cm = np.meshgrid(*grid, indexing="ij")
    Xs = np.stack([np.stack([Am, Bm], -1), np.stack([Bm, Cm], -1)], -2).reshape(-1, 2, 2)
    Xi, _ = inv2(Xs)
    hlo, hhi = Xi.min(axis=0), Xi.max(axis=0)
    for tangent in ("lo", "hi"):
        A, ok = adjugate_inv(X, tangent)
        assert ok
        alo, ahi = A.bounds()
        assert np.all(alo <= hlo + 1e-12) and np.all(hhi <= ahi + 1e-12)
        w_adj = np.linalg.norm(ahi - alo)
        assert w_adj > w_matinv > np.linalg.norm(hhi - hlo)
    # the paper's ranking of its own numbers
    assert g["width_adjugate_paper"] > g["width_matrixinv_paper"] > g["width_empirical_paper"]


def test_adjugate_scene_sound():
    """The adjugate inverse in the whole pipeline: sound at sampled poses.  On this
    translation case it is no tighter on average than MatrixInv; on relational inputs in
    general it can be (Example 'matinv-vs-direct' ranks them on a constant interval
    matrix), so that comparison is this case's, not a law."""
    sc = synth.random_scene(24, seed=3)
    intr = synth.intrinsics(24)
    box = synth.camera6_box(dt=0.04)
    r_adj = splat.oracle_bounds(sc, intr, box, {"inverse": "adjugate"})
    r_mi = splat.oracle_bounds(sc, intr, box)
    rng = np.random.default_rng(1)
    for p in pose.sample_poses(box, 24, rng):
        img = render.render(sc, intr, box, p)
        assert (r_adj["lo"] - img).max() <= 1e-9 and (img - r_adj["hi"]).max() <= 1e-9
    assert (r_adj["hi"] - r_adj["lo"]).mean() >= (r_mi["hi"] - r_mi["lo"]).mean() - 1e-12


# --- abstract BlendSort --------------------------------------------------------------------
def test_blend_sort_fixed_order_is_concrete():
    for _ in range(20):
        n, m = int(RNG.integers(1, 7)), 5
        a = RNG.uniform(0, 0.95, (n, m))
        c = RNG.uniform(0, 1, (n, 3))
        d = RNG.permutation(n).astype(np.float64) + 3.0
        lo, hi = splat.blend_sort_abstract(a, a, c, d, d, 0.0)
        ref = render.blend_sort(a, c, d)
        np.testing.assert_allclose(lo, ref, atol=1e-13)
        np.testing.assert_allclose(hi, ref, atol=1e-13)


def test_blend_sort_encloses_brute_force():
    """Every concrete BlendSort over depths drawn from the intervals (their ends and ties
    included) and every vertex of the alpha box lies inside the abstract BlendSort."""
    for trial in range(40):
        n, m = int(RNG.integers(2, 6)), 3
        centre = RNG.uniform(3, 4, n)
        rad = RNG.uniform(0, 0.3, n)
        if trial % 4 == 0:
            centre[1] = centre[0]          # equal depth intervals (ties possible)
            rad[1] = rad[0]
        dlo, dhi = centre - rad, centre + rad
        al = RNG.uniform(0, 0.6, (n, m))
        au = np.minimum(al + RNG.uniform(0, 0.3, (n, m)), 0.99)
        c = RNG.uniform(0, 1, (n, 3))
        lo, hi = splat.blend_sort_abstract(al, au, c, dlo, dhi, 0.0)
        depths = [dlo, dhi, centre] + [RNG.uniform(dlo, dhi) for _ in range(6)]
        for d in depths:
            for bits in itertools.product((0, 1), repeat=n):
                a = np.where(np.array(bits)[:, None] == 1, au, al)
                pc = render.blend_sort(a, c, d)
                assert np.all(lo <= pc + 1e-12) and np.all(pc <= hi + 1e-12)


def test_example2_analogue_sort_wider_than_ind():
    """Example '3g-scene' analogue: three Gaussians (red, green, blue) in front of the camera,
    translation box +-0.3 on each axis, 20x20 image.  BlendSort's abstract sort sees only
    the depth intervals (they overlap), BlendInd the exact depth differences (fixed under a
    translation box): both enclose sampled renders, and BlendSort's bounds are wider."""
    g = _load("example2_analogue.json")
    scene = {"mean": np.array(g["mean"]), "cov_factor": np.stack([np.eye(3) * s for s in g["scale"]]),
             "opacity": np.array(g["opacity"]), "rgb": np.array(g["rgb"])}
    intr = synth.intrinsics(g["side"])
    box = synth.camera6_box(dt=g["half_width"])
    res = {m: splat.oracle_bounds(scene, intr, box, {"blend": m, "cull_budget": 1e-9})
           for m in ("ind", "ind_interval", "sort")}
    rng = np.random.default_rng(0)
    emp_lo = np.full((g["side"], g["side"], 3), np.inf)
    emp_hi = np.full((g["side"], g["side"], 3), -np.inf)
    for p in pose.sample_poses(box, 120, rng):
        img = render.render(scene, intr, box, p)
        emp_lo = np.minimum(emp_lo, img)
        emp_hi = np.maximum(emp_hi, img)
    for r in res.values():
        assert (r["lo"] - emp_lo).max() <= 1e-9 and (emp_hi - r["hi"]).max() <= 1e-9
    w = {m: (r["hi"] - r["lo"]).mean() for m, r in res.items()}
    assert w["sort"] > w["ind_interval"] >= w["ind"] - 1e-12
    # the same alpha intervals, blended two ways: BlendSort's upper bound is never below
    # the interval BlendInd's here, and strictly above it at the paper's pixel (row 2, col 10)
    assert (res["sort"]["hi"] - res["ind_interval"]["hi"]).min() >= -1e-12
    r, c = g["pixel_row_col"]
    assert np.all(res["sort"]["hi"][r, c] > res["ind"]["hi"][r, c])


# --- Ind under rotation ------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["camera6", "orbit"])
def test_ind_matrix_agrees_with_concrete_depth_order(kind):
    sc = synth.box_surface_scene(120, n_boxes=3, seed=8)
    if kind == "camera6":
        box = synth.camera6_box(dt=0.03, drot=np.deg2rad(1.0))
    else:
        box = synth.orbit_cells(1, 4.0, seed=0)[0]
    rec = splat.gaussian_forms(sc, synth.intrinsics(32), box)
    idx = np.arange(len(sc["opacity"]))
    ind, _ = splat.ind_matrix(rec, idx)
    decided = ind != 2
    assert decided.mean() > 0.5 and (ind == 2).any()
    uw = np.asarray(sc["mean"], dtype=np.float64)
    rng = np.random.default_rng(3)
    for p in pose.sample_poses(box, 60, rng):
        R, t = pose.concrete_camera(box, p)
        d = ((uw - t) @ R.T)[:, 2]
        concrete = (d[:, None] - d[None, :]) > 0
        np.fill_diagonal(concrete, False)
        assert np.all(concrete[ind == 1]) and not np.any(concrete[ind == 0])


# --- pruning -------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_float32_keep_contains_fp64_keep(seed):
    sc = synth.random_scene(300, seed=seed)
    intr = synth.intrinsics(48)
    box = synth.camera6_box(dt=0.05, drot=np.deg2rad(0.5) if seed == 2 else 0.0)
    rec = splat.gaussian_forms(sc, intr, box, {"cull_budget": 1e-4})
    cols, rows = np.meshgrid(np.arange(48), np.arange(48), indexing="xy")
    ux32, uy32 = splat.pixel_coords32(intr, cols.ravel(), rows.ravel())
    ux = cols.ravel() + 0.5 - intr["cx"]
    uy = rows.ravel() + 0.5 - intr["cy"]
    idx = np.nonzero(rec["normal"])[0]
    keep32 = splat.kept_mask(rec, idx, ux32, uy32)
    mu = rec["mu64"][idx]
    dx = np.maximum(np.maximum(mu[:, None, 0] - ux[None, :], 0.0), ux[None, :] - mu[:, None, 1])
    dy = np.maximum(np.maximum(mu[:, None, 2] - uy[None, :], 0.0), uy[None, :] - mu[:, None, 3])
    a64 = rec["o"][idx][:, None] * np.exp(-0.5 * (dx * dx + dy * dy) / rec["lam"][idx][:, None])
    must = a64 > rec["eps_cull"] * (1.0 + 2.0 ** -10)
    assert must.any() and not must.all()
    assert np.all(keep32[must])


# --- backward (CROWN-style) MatrixInv ------------------------------------------------------
@pytest.mark.parametrize("k", [2, 8])
def test_backward_matrixinv_encloses_inverse(k):
    from oracle.crown import matrix_inv_backward
    for _ in range(20):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.5 * np.eye(2)
        rad = np.abs(RNG.normal(0, 0.05, (2, 2)))
        rad = 0.5 * (rad + rad.T)
        X = interval_matrix(M - rad, M + rad, symmetric=True)
        conic, ok, _ = matrix_inv_backward(X, k)
        if not ok:
            continue
        for _ in range(50):
            e = RNG.uniform(-1, 1, 3)
            lo, up = conic.eval(e)
            Xe = 0.5 * (X.lo + X.up) @ np.concatenate([e, [1.0]])
            Xi = np.linalg.inv(Xe)
            assert np.all(lo <= Xi + 1e-12) and np.all(Xi <= up + 1e-12)


def test_backward_matrixinv_zero_width_is_the_inverse():
    from oracle.crown import matrix_inv_backward
    for _ in range(10):
        L = RNG.normal(size=(2, 2))
        M = L @ L.T + 0.2 * np.eye(2)
        conic, ok, _ = matrix_inv_backward(lf.const(M, 0), 8)
        assert ok
        tol = 1e-12 * np.linalg.cond(M) * np.abs(np.linalg.inv(M)).max()
        np.testing.assert_allclose(conic.lo[..., 0], np.linalg.inv(M), atol=tol)
        np.testing.assert_allclose(conic.up[..., 0], np.linalg.inv(M), atol=tol)


def test_example1_backward_matrixinv_reaches_the_papers_width():
    """Example 'matinv-vs-direct': bounded backward, as the paper's bound engine does,
    MatrixInv encloses the exact hull (0.66) and is tighter than forward mode (0.737),
    within 0.01 of the paper's 0.70."""
    from oracle.crown import matrix_inv_backward
    g = _load("example1_matinv.json")
    lo, hi = np.array(g["X_lo"]), np.array(g["X_hi"])
    X = interval_matrix(lo, hi, symmetric=True)
    grid = [np.linspace(lo[i][j], hi[i][j], 61) for i, j in ((0, 0), (0, 1), (1, 1))]
    Am, Bm, Cm = np.meshgrid(*grid, indexing="ij")
    Xs = np.stack([np.stack([Am, Bm], -1), np.stack([Bm, Cm], -1)], -2).reshape(-1, 2, 2)
    Xi, _ = inv2(Xs)
    hlo, hhi = Xi.min(axis=0), Xi.max(axis=0)
    back, ok, _ = matrix_inv_backward(X, 8)
    fwd, ok2, _ = matrix_inv(X, 8)
    assert ok and ok2
    blo, bhi = back.bounds()
    flo, fhi = fwd.bounds()
    assert np.all(blo <= hlo + 1e-12) and np.all(hhi <= bhi + 1e-12)
    w_back, w_fwd = np.linalg.norm(bhi - blo), np.linalg.norm(fhi - flo)
    assert np.linalg.norm(hhi - hlo) < w_back < w_fwd
    assert abs(w_back - g["width_matrixinv_paper"]) < 0.01


def test_backward_matrixinv_scene_sound_and_not_wider():
    sc = synth.random_scene(30, seed=5)
    intr = synth.intrinsics(24)
    box = synth.camera6_box(dt=0.05, drot=np.deg2rad(0.4))
    r_b = splat.oracle_bounds(sc, intr, box, {"inverse": "matrixinv_backward"})
    r_f = splat.oracle_bounds(sc, intr, box)
    rng = np.random.default_rng(4)
    for p in pose.sample_poses(box, 24, rng):
        img = render.render(sc, intr, box, p)
        assert (r_b["lo"] - img).max() <= 1e-9 and (img - r_b["hi"]).max() <= 1e-9
    assert (r_b["hi"] - r_b["lo"]).mean() <= (r_f["hi"] - r_f["lo"]).mean() + 1e-9
