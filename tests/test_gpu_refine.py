"""Adaptive refinement of a pose box through the C ABI (Sec. 3.1: the input range is
divided where MatrixInv's convergence assertion fails; Sec. 4.2: bounds of subsets of
the cameras, united).

The per-cell counts must equal the oracle's, the leaves must be the oracle's (bit for
bit, same order), the united bounds must equal the union of the leaves rendered one by
one (bit for bit with a fixed segment length), match the oracle's united bounds within
1e-5, and enclose sampled concrete renders.
"""
import numpy as np
import pytest

from paper_2503_00308_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
SCENE = synth.box_surface_scene(200, n_boxes=4, seed=3)
INTR = synth.intrinsics(32)


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_00308_amd import api
    api.load()
    return api


def orbit_box(deg):
    a = np.deg2rad(deg)
    return {"model": 1, "R0": np.eye(3), "t0": np.zeros(3), "pivot": np.array([0.0, 0.0, 4.0]),
            "lo": np.array([-a, 0, 0, 0, 0, 0], np.float64), "hi": np.array([a, 0, 0, 0, 0, 0], np.float64)}


def near_scene():
    """40 random Gaussians at depth 3-5 and one whose mean sits at depth 0.02."""
    s = synth.random_scene(40, seed=5)
    t = synth.random_scene(1, seed=6)
    t["mean"][0] = (0.05, -0.03, 0.02)
    return {k: np.concatenate([s[k], t[k]]) for k in s}


MATINV, NEAR = 1, 2
NEAR_SCENE = near_scene()
# name: (scene, box, max_cells, criteria)
CASES = {
    "orbit3": (SCENE, orbit_box(3.0), 16, MATINV),
    "orbit3_budget4": (SCENE, orbit_box(3.0), 4, MATINV),
    "camera4": (SCENE, synth.camera6_box(dt=(0.05, 0.0, 0.05), drot=(np.deg2rad(2), np.deg2rad(2), 0.0)), 16, MATINV),
    "near_only": (NEAR_SCENE, synth.camera6_box(dt=(0.0, 0.0, 0.04)), 6, NEAR),
    "near_and_matinv": (NEAR_SCENE, synth.camera6_box(dt=(0.0, 0.0, 0.04)), 6, MATINV | NEAR),
}


@pytest.mark.parametrize("name", list(CASES))
def test_counts_and_leaves_equal_the_oracle(name):
    from oracle import refine
    api = _api()
    scene, box, max_cells, crit = CASES[name]
    sc = api.Scene(scene)
    lo, hi, leaves, st = api.render_refined(sc, INTR, box, max_cells, criteria=crit, opts={"chunk": 32})
    ref = refine.refine(scene, INTR, box, max_cells, near=bool(crit & NEAR), matinv=bool(crit & MATINV))
    print(f"[refine {name}] {len(leaves)} leaves (oracle {len(ref)}), stats {st}", flush=True)
    assert len(leaves) == len(ref)
    for a, b in zip(leaves, ref):
        assert a["model"] == b.get("model", 0)
        assert np.array_equal(a["lo"], np.asarray(b["lo"], np.float64))
        assert np.array_equal(a["hi"], np.asarray(b["hi"], np.float64))
    counts = api.classify_cells(sc, INTR, [box] + leaves)
    sc.close()
    want = np.array([refine.flagged_counts(scene, INTR, c) for c in [box] + ref], np.int64)
    print(f"[refine {name}] counts {counts.tolist()}", flush=True)
    assert np.array_equal(counts, want)


@pytest.mark.parametrize("name", ["orbit3", "camera4"])
def test_refined_bounds_union_parity_and_soundness(name):
    from oracle import pose, refine, render
    api = _api()
    scene, box, max_cells, _ = CASES[name]
    assert scene is SCENE
    sc = api.Scene(SCENE)
    opts = {"chunk": 32}
    rlo, rhi, leaves, _ = api.render_refined(sc, INTR, box, max_cells, opts=opts)
    rlo, rhi = rlo.cpu().numpy(), rhi.cpu().numpy()
    ulo = np.full(rlo.shape, np.inf, np.float32)
    uhi = np.full(rhi.shape, -np.inf, np.float32)
    for c in leaves:
        lo, hi, _ = api.render_bounds(sc, INTR, c, opts)
        ulo = np.minimum(ulo, lo.cpu().numpy())
        uhi = np.maximum(uhi, hi.cpu().numpy())
    wlo, whi, _ = api.render_bounds(sc, INTR, box, opts)
    sc.close()
    assert np.array_equal(rlo, ulo) and np.array_equal(rhi, uhi)
    # oracle: the union of its leaves' bounds (pixels with a borderline decision excluded)
    from oracle import splat
    olo = np.full(rlo.shape, np.inf)
    ohi = np.full(rhi.shape, -np.inf)
    border = np.zeros(rlo.shape[:2], bool)
    for c in refine.refine(SCENE, INTR, box, max_cells):
        r = splat.oracle_bounds(SCENE, INTR, c)
        olo = np.minimum(olo, r["lo"])
        ohi = np.maximum(ohi, r["hi"])
        border |= r["border"]
    ok = np.broadcast_to(~border[..., None], rlo.shape)
    dlo = np.abs(rlo.astype(np.float64) - olo)[ok].max()
    dhi = np.abs(rhi.astype(np.float64) - ohi)[ok].max()
    print(f"[refine {name}] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}, border pixels {int(border.sum())}", flush=True)
    assert dlo <= TOL and dhi <= TOL
    rng = np.random.default_rng(9)
    worst = -np.inf
    for p in pose.sample_poses(box, 16, rng):
        img = render.render(SCENE, INTR, box, p)
        worst = max(worst, (rlo - img).max(), (img - rhi).max())
    print(f"[refine {name}] soundness worst {worst:.3e}; mean width {float((rhi - rlo).mean()):.4f} "
          f"against {float((whi.cpu().numpy() - wlo.cpu().numpy()).mean()):.4f} for the whole box", flush=True)
    assert worst <= 1e-7


def test_refine_without_failures_is_the_plain_render():
    api = _api()
    scene = synth.random_scene(60, seed=11)
    box = synth.camera6_box(dt=(0.02, 0.0, 0.0))
    sc = api.Scene(scene)
    opts = {"chunk": 32}
    rlo, rhi, leaves, _ = api.render_refined(sc, INTR, box, 64, opts=opts)
    lo, hi, _ = api.render_bounds(sc, INTR, box, opts)
    sc.close()
    assert len(leaves) == 1
    assert np.array_equal(rlo.cpu().numpy(), lo.cpu().numpy()) and np.array_equal(rhi.cpu().numpy(), hi.cpu().numpy())


def test_refine_rejects_bad_arguments():
    api = _api()
    sc = api.Scene(synth.random_scene(50, seed=43))
    box = synth.camera6_box(dt=0.01)
    with pytest.raises(api.ARError):
        api.render_refined(sc, synth.intrinsics(16), box, 0)
    with pytest.raises(api.ARError):
        api.render_refined(sc, synth.intrinsics(16), box, 70000)
    with pytest.raises(api.ARError):
        api.render_refined(sc, synth.intrinsics(16), box, 8, criteria=8)
    sc.close()
