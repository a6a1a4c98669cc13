"""Batched rendering of pose cells (one launch per stage for many cells), through the C ABI.

The batched pipeline must give, cell by cell, exactly the bounds of a single-cell call
(same records, same per-cell depth order, same lists and runs; the translation path with
a fixed segment length), and the single-cell calls are pinned to the oracle elsewhere;
a few cells are also compared with the oracle directly.
"""
import numpy as np
import pytest

from paper_2503_00308_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_00308_amd import api
    api.load()
    return api


def _single(api, sc, intr, cells, opts=None):
    out_lo, out_hi = [], []
    for c in cells:
        lo, hi, _ = api.render_bounds(sc, intr, c, opts)
        out_lo.append(lo.cpu().numpy())
        out_hi.append(hi.cpu().numpy())
    return np.stack(out_lo), np.stack(out_hi)


def _batch(api, sc, intr, cells, opts=None):
    lo, hi, st = api.render_batch(sc, intr, cells, opts)
    return lo.cpu().numpy(), hi.cpu().numpy(), st


def test_batch_orbit_cells_equal_single_cells():
    api = _api()
    scene = synth.box_surface_scene(800, n_boxes=6, seed=11)
    intr = synth.intrinsics(48)
    cells = synth.orbit_cells(12, 30.0, seed=5)
    sc = api.Scene(scene)
    slo, shi = _single(api, sc, intr, cells)
    blo, bhi, st = _batch(api, sc, intr, cells)
    print("orbit batch stats", st, flush=True)
    assert np.array_equal(blo, slo) and np.array_equal(bhi, shi)
    # several launches of 5 cells give the same result
    clo, chi, _ = _batch(api, sc, intr, cells, {"cells_per_launch": 5})
    assert np.array_equal(clo, slo) and np.array_equal(chi, shi)
    sc.close()


def test_batch_translation_cells_equal_single_cells():
    api = _api()
    scene = synth.random_scene(400, seed=12)
    intr = synth.intrinsics(40)
    rng = np.random.default_rng(3)
    cells = []
    for _ in range(7):
        b = synth.camera6_box(dt=0.05)
        shift = rng.uniform(-0.3, 0.3, 3)
        b["lo"][:3] += shift
        b["hi"][:3] += shift
        cells.append(b)
    sc = api.Scene(scene)
    opts = {"chunk": 32}        # the same segment length in both calls
    slo, shi = _single(api, sc, intr, cells, opts)
    blo, bhi, _ = _batch(api, sc, intr, cells, opts)
    assert np.array_equal(blo, slo) and np.array_equal(bhi, shi)
    # automatic segment lengths differ between the calls: equal up to rounding
    alo, ahi, _ = _batch(api, sc, intr, cells)
    assert np.abs(alo - slo).max() <= 1e-12 and np.abs(ahi - shi).max() <= 1e-12
    sc.close()


def test_batch_mixed_pose_variables():
    """Consecutive cells with different numbers of pose variables (and rotating or not)
    go to separate launches; every cell still equals its single-cell render."""
    api = _api()
    scene = synth.box_surface_scene(500, n_boxes=5, seed=13)
    intr = synth.intrinsics(32)
    cells = [synth.camera6_box(dt=(0.05, 0.0, 0.0)), synth.camera6_box(dt=(0.02, 0.0, 0.0)),
             synth.camera6_box(dt=(0.03, 0.03, 0.0)), synth.camera6_box(dt=0.02, drot=np.deg2rad(0.5)),
             synth.camera6_box(dt=0.01, drot=np.deg2rad(0.3)), synth.camera6_box()]
    sc = api.Scene(scene)
    opts = {"chunk": 32}
    slo, shi = _single(api, sc, intr, cells, opts)
    blo, bhi, _ = _batch(api, sc, intr, cells, opts)
    assert np.array_equal(blo, slo) and np.array_equal(bhi, shi)
    sc.close()


def test_batch_orbit_cells_parity_with_oracle():
    from oracle import splat
    api = _api()
    scene = synth.box_surface_scene(250, n_boxes=4, seed=3)
    intr = synth.intrinsics(40)
    cells = synth.orbit_cells(16, 30.0, seed=2)
    sc = api.Scene(scene)
    blo, bhi, _ = _batch(api, sc, intr, cells)
    sc.close()
    for k in (0, 7, 15):
        ref = splat.oracle_bounds(scene, intr, cells[k])
        ok = ~ref["border"][..., None]
        dlo = np.abs(blo[k] - ref["lo"])[np.broadcast_to(ok, ref["lo"].shape)].max()
        dhi = np.abs(bhi[k] - ref["hi"])[np.broadcast_to(ok, ref["hi"].shape)].max()
        print(f"[orbit cell {k}] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
        assert dlo <= TOL and dhi <= TOL


def test_batch_full_size_orbit_sampled_tiles():
    """The batched workload (50k Gaussians on boxes, 200x200, 256 orbit cells of uneven
    widths) in its launch configuration; two cells compared with the oracle on sampled
    8x8 tiles, every cell finite and ordered."""
    from oracle import splat
    api = _api()
    scene, intr, cells, _ = synth.config(4)
    sc = api.Scene(scene)
    blo, bhi, st = _batch(api, sc, intr, cells)
    sc.close()
    print("cfg4 batch stats", st, flush=True)
    assert np.all(np.isfinite(blo)) and np.all(np.isfinite(bhi)) and np.all(blo <= bhi)
    tiles = [(12, 12), (9, 14)]
    for k in (0, 200):
        ref = splat.oracle_bounds(scene, intr, cells[k], opts={"tile": 8}, tiles=tiles)
        mask = np.zeros(blo.shape[1:3], bool)
        for tx, ty in tiles:
            mask[ty * 8:(ty + 1) * 8, tx * 8:(tx + 1) * 8] = True
        ok = (mask & ~ref["border"])[..., None]
        dlo = np.abs(blo[k] - ref["lo"])[np.broadcast_to(ok, ref["lo"].shape)].max()
        dhi = np.abs(bhi[k] - ref["hi"])[np.broadcast_to(ok, ref["hi"].shape)].max()
        print(f"[cfg4 cell {k}] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
        assert dlo <= TOL and dhi <= TOL


def test_autotune_segment_length():
    """Autotuning returns a candidate segment length; the bounds it leaves are those of a
    render with the tuned options, bit for bit, and agree with the default render up to
    rounding and the early-stop allowance (t_min = 1e-7 on the upper bound)."""
    api = _api()
    scene = synth.random_scene(2000, seed=31)
    intr = synth.intrinsics(64)
    box = synth.camera6_box(dt=0.08)
    sc = api.Scene(scene)
    tuned, lo, hi, st = api.autotune(sc, intr, box)
    print("translation tuned", tuned["chunk"], st, flush=True)
    assert tuned["chunk"] % 8 == 0 and 8 <= tuned["chunk"] <= 4096
    assert st["segment_length"] == tuned["chunk"]
    l2, h2, _ = api.render_bounds(sc, intr, box, tuned)
    assert np.array_equal(lo[0].cpu().numpy(), l2.cpu().numpy()) and np.array_equal(hi[0].cpu().numpy(),
                                                                                      h2.cpu().numpy())
    l0, h0, _ = api.render_bounds(sc, intr, box)
    # another segment length sums in another order: FP64 rounding, then directed rounding to
    # float32 (one float32 ulp of a small lower bound)
    assert np.abs(l0.cpu().numpy() - l2.cpu().numpy()).max() <= 1e-9
    assert np.abs(h0.cpu().numpy() - h2.cpu().numpy()).max() <= 2e-7
    sc.close()
    scene = synth.box_surface_scene(1500, n_boxes=8, seed=32)
    cells = synth.orbit_cells(6, 10.0, seed=3)
    sc = api.Scene(scene)
    tuned, lo, hi, st = api.autotune(sc, intr, cells, reps=1)
    print("rotation tuned", tuned["chunk"], "cells per launch", tuned["cells_per_launch"], flush=True)
    assert tuned["chunk"] in (32, 48, 64, 96, 128)
    assert 0 <= tuned["cells_per_launch"] <= len(cells)
    l3, h3, _ = _batch(api, sc, intr, cells, tuned)
    assert np.array_equal(lo.cpu().numpy(), l3) and np.array_equal(hi.cpu().numpy(), h3)
    # every cells-per-launch count gives the same images (rotation cells: bit for bit)
    for cpl in (1, 2, 4):
        l4, h4, _ = _batch(api, sc, intr, cells, dict(tuned, cells_per_launch=cpl))
        assert np.array_equal(l3, l4) and np.array_equal(h3, h4), cpl
    sc.close()
