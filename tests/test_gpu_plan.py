"""Planned batched renders (ar_plan_*): the batch's whole launch sequence captured once in a
HIP graph and replayed, through the C ABI.

The captured sequence keeps every count on the device, so it must give, cell by cell,
exactly the images of ar_render_batch (rotation boxes always; translation boxes with a
fixed segment length), after creation and after every replay, with other work on the
device between replays; new cells set into the plan give their own batch's images; cells
that outgrow the plan are rendered again (replanned) and still exact; one cell is also
checked against the oracle.
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


def _batch(api, sc, intr, cells, opts=None):
    import torch
    lo, hi, st = api.render_batch(sc, intr, cells, opts)
    torch.cuda.synchronize()
    return lo.cpu().numpy(), hi.cpu().numpy(), st


def _plan_images(plan):
    import torch
    torch.cuda.synchronize()
    return plan.lo.cpu().numpy(), plan.hi.cpu().numpy()


def test_plan_orbit_cells_replays_equal_the_batch():
    import torch
    from oracle import splat
    api = _api()
    scene = synth.box_surface_scene(800, n_boxes=6, seed=11)
    intr = synth.intrinsics(48)
    cells = synth.orbit_cells(12, 30.0, seed=5)
    sc = api.Scene(scene)
    opts = {"cells_per_launch": 5}
    blo, bhi, bst = _batch(api, sc, intr, cells, opts)
    plan = api.Plan(sc, intr, cells, opts)
    plo, phi = _plan_images(plan)
    assert np.array_equal(plo, blo) and np.array_equal(phi, bhi)
    for rep in range(3):
        plan.lo.fill_(float("nan"))
        plan.hi.fill_(float("nan"))
        # other work on the device between replays
        _ = torch.ones(1 << 20, device="cuda").sum().item()
        st, replanned = plan.launch()
        plo, phi = _plan_images(plan)
        print(f"replay {rep}: pairs {st['pairs']} (batch {bst['pairs']}), runs {st['runs']}, "
              f"graph {st['total_ms']:.2f} ms, replanned {replanned}", flush=True)
        assert not replanned
        assert np.array_equal(plo, blo) and np.array_equal(phi, bhi)
        assert st["pairs"] == bst["pairs"] and st["tile_pairs"] == bst["tile_pairs"]
    # one cell against the oracle
    ref = splat.oracle_bounds(scene, intr, cells[3])
    assert np.abs(plo[3] - ref["lo"]).max() <= TOL and np.abs(phi[3] - ref["hi"]).max() <= TOL
    # other cells of the same kind, within the plan's room or not
    other = synth.orbit_cells(12, 24.0, seed=9)
    plan.set_cells(other)
    st, _ = plan.launch()
    olo, ohi, _ = _batch(api, sc, intr, other, opts)
    plo, phi = _plan_images(plan)
    assert np.array_equal(plo, olo) and np.array_equal(phi, ohi)
    plan.close()
    sc.close()


def test_plan_outgrown_cells_are_replanned():
    api = _api()
    scene = synth.box_surface_scene(600, n_boxes=5, seed=3)
    intr = synth.intrinsics(40)
    narrow = synth.orbit_cells(6, 1.0, seed=2)
    wide = synth.orbit_cells(6, 60.0, seed=2)
    sc = api.Scene(scene)
    plan = api.Plan(sc, intr, narrow)
    plan.set_cells(wide)
    st, replanned = plan.launch()
    assert replanned
    wlo, whi, _ = _batch(api, sc, intr, wide)
    plo, phi = _plan_images(plan)
    assert np.array_equal(plo, wlo) and np.array_equal(phi, whi)
    st, replanned = plan.launch()
    assert not replanned
    plo, phi = _plan_images(plan)
    assert np.array_equal(plo, wlo) and np.array_equal(phi, whi)
    plan.close()
    sc.close()


def test_plan_translation_cells_equal_the_batch():
    api = _api()
    scene = synth.random_scene(400, seed=12)
    intr = synth.intrinsics(40)
    cells = [synth.camera6_box(dt=(0.01 * (k + 1), 0.02, 0.005 * (k + 1))) for k in range(7)]
    sc = api.Scene(scene)
    opts = {"chunk": 48, "cells_per_launch": 4}
    blo, bhi, _ = _batch(api, sc, intr, cells, opts)
    plan = api.Plan(sc, intr, cells, opts)
    for _ in range(2):
        st, replanned = plan.launch()
        assert not replanned
        plo, phi = _plan_images(plan)
        assert np.array_equal(plo, blo) and np.array_equal(phi, bhi)
    plan.close()
    sc.close()


def test_plan_rejects_mixed_cells():
    api = _api()
    scene = synth.random_scene(50, seed=1)
    sc = api.Scene(scene)
    intr = synth.intrinsics(16)
    plan = api.Plan(sc, intr, [synth.camera6_box(dt=0.01), synth.camera6_box(dt=0.02)])
    with pytest.raises(api.ARError) as ei:
        plan.set_cells([synth.camera6_box(dt=0.01), synth.camera6_box(dt=0.01, drot=0.01)])
    assert ei.value.code == api.AR_E_INVALID
    plan.close()
    sc.close()
