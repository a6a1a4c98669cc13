"""Batches whose cells render different scenes (ar_render_batch_scenes), through the C ABI.

The partition of a set of poses (Sec. 4.2) rendered for several scenes at once: cells of
scenes of different sizes share one launch per stage, each cell's Gaussians being its own
range of the launch's items.

Bar: every cell's images equal, bit for bit, those of rendering that cell alone with its
own scene (rotation boxes; translation boxes with a fixed segment length), with the cells
in one launch or split over several, and the accumulated pair count is the sum of the
cells' own; one cell is also checked against the oracle at 1e-5; sets of scenes among
other scenes and NULL scenes are rejected.
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


def _scenes():
    return [synth.random_scene(150, seed=21), synth.box_surface_scene(700, n_boxes=5, seed=22),
            synth.random_scene(420, seed=23)]


def _cells():
    deg = np.deg2rad
    rot = [synth.camera6_box(dt=0.01, drot=deg(0.2)),
           synth.camera6_box(dt=(0.02, 0.0, 0.01), drot=(deg(0.4), 0.0, deg(0.1))),
           synth.camera6_box(dt=0.005, drot=deg(0.3)),
           synth.camera6_box(dt=0.01, drot=deg(0.1))]
    trans = [synth.camera6_box(dt=0.05), synth.camera6_box(dt=(0.02, 0.08, 0.01)), synth.camera6_box(dt=0.03)]
    # (scene index, box): runs of rotation and translation cells, scenes interleaved
    return [(0, rot[0]), (1, rot[1]), (2, rot[2]), (1, rot[3]), (0, trans[0]), (2, trans[1]), (1, trans[2])]


@pytest.mark.parametrize("per_launch", [0, 2])
def test_cells_of_several_scenes_equal_their_own_renders(per_launch):
    import torch
    api = _api()
    scenes = [api.Scene(s) for s in _scenes()]
    intr = synth.intrinsics(40)
    plan = _cells()
    opts = {"chunk": 48, "cells_per_launch": per_launch}
    lo, hi, st = api.render_batch_scenes([scenes[k] for k, _ in plan], intr, [b for _, b in plan], opts)
    torch.cuda.synchronize()
    lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
    pairs = 0
    for c, (k, box) in enumerate(plan):
        l1, h1, s1 = api.render_bounds(scenes[k], intr, box, {"chunk": 48})
        torch.cuda.synchronize()
        same = np.array_equal(lo[c], l1.cpu().numpy()) and np.array_equal(hi[c], h1.cpu().numpy())
        if not same:
            print(f"cell {c} (scene {k}, P {s1['P']}): max diff lo {np.abs(lo[c] - l1.cpu().numpy()).max():.3e} "
                  f"hi {np.abs(hi[c] - h1.cpu().numpy()).max():.3e}", flush=True)
        assert same, c
        pairs += s1["pairs"]
    print(f"[per launch {per_launch}] pairs {st['pairs']} (cells alone {pairs}), runs {st['runs']}", flush=True)
    assert st["pairs"] == pairs
    for sc in scenes:
        sc.close()


def test_mixed_batch_cell_against_the_oracle():
    import torch
    from oracle import splat
    api = _api()
    raw = _scenes()
    scenes = [api.Scene(s) for s in raw]
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=0.01, drot=np.deg2rad(0.2))
    lo, hi, _ = api.render_batch_scenes([scenes[2], scenes[0], scenes[1]], intr, [box, box, box])
    torch.cuda.synchronize()
    for c, k in enumerate((2, 0, 1)):
        ref = splat.oracle_bounds(raw[k], intr, box)
        ok = np.broadcast_to(~ref["border"][..., None], ref["lo"].shape)
        dlo = np.abs(lo[c].cpu().numpy() - ref["lo"])[ok].max()
        dhi = np.abs(hi[c].cpu().numpy() - ref["hi"])[ok].max()
        print(f"cell {c} scene {k}: max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
        assert dlo <= TOL and dhi <= TOL
    for sc in scenes:
        sc.close()


def test_batch_scenes_rejections():
    api = _api()
    plain = api.Scene(synth.random_scene(40, seed=3))
    varied = api.Scene(synth.perturbed_scene(synth.random_scene(40, seed=4), kinds=("mean",)))
    intr = synth.intrinsics(16)
    box = synth.camera6_box(dt=0.01)
    with pytest.raises(api.ARError) as ei:
        api.render_batch_scenes([plain, varied], intr, [box, box])
    assert ei.value.code == api.AR_E_UNSUPPORTED
    # one scene for every cell is an ordinary batch, sets of scenes included
    lo, hi, _ = api.render_batch_scenes([varied, varied], intr, [box, box])
    l1, h1, _ = api.render_batch(varied, intr, [box, box])
    assert np.array_equal(lo.cpu().numpy(), l1.cpu().numpy()) and np.array_equal(hi.cpu().numpy(), h1.cpu().numpy())
    with pytest.raises(ValueError):
        api.render_batch_scenes([plain], intr, [box, box])
    plain.close()
    varied.close()


def test_orbit_cells_of_several_scenes_and_host_outputs():
    """Orbit cells (one angle) of two scenes in one call, into device and into host
    memory: the same images, each equal to its scene's own batch of that cell."""
    import torch
    api = _api()
    raw = _scenes()[:2]
    scenes = [api.Scene(s) for s in raw]
    intr = synth.intrinsics(32)
    cells = synth.orbit_cells(4, 8.0, seed=4)
    owner = [0, 1, 1, 0]
    lo, hi, st = api.render_batch_scenes([scenes[k] for k in owner], intr, cells)
    torch.cuda.synchronize()
    hlo = torch.empty((4, 32, 32, 3), dtype=torch.float32, pin_memory=True)
    hhi = torch.empty_like(hlo)
    api.render_batch_scenes([scenes[k] for k in owner], intr, cells, out=(hlo, hhi))
    assert np.array_equal(lo.cpu().numpy(), hlo.numpy()) and np.array_equal(hi.cpu().numpy(), hhi.numpy())
    for c, k in enumerate(owner):
        l1, h1, _ = api.render_batch(scenes[k], intr, [cells[c]])
        torch.cuda.synchronize()
        assert np.array_equal(lo[c].cpu().numpy(), l1[0].cpu().numpy()), c
        assert np.array_equal(hi[c].cpu().numpy(), h1[0].cpu().numpy()), c
    assert st["P"] == 1
    for sc in scenes:
        sc.close()
