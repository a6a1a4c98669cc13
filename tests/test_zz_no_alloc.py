"""ar_render_bounds_noalloc (every buffer in the library's static scratch array) against
ar_render_bounds, through the C ABI: the same kernels, so the images must be identical bit
for bit; two calls in a row, the second on a smaller input (the scratch keeps the first
call's contents), and the small case also against the FP64 oracle.  Limits: rotation
boxes and inputs beyond the scratch are rejected with a message, and a call after a
rejected one is still exact.
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


def _both(api, sc, intr, box, opts=None):
    import torch
    lo, hi, st = api.render_bounds(sc, intr, box, opts)
    nlo = torch.full_like(lo, float("nan"))
    nhi = torch.full_like(hi, float("nan"))
    nst = api.render_bounds_noalloc(sc, intr, box, (nlo, nhi), opts)
    torch.cuda.synchronize()
    return lo.cpu().numpy(), hi.cpu().numpy(), st, nlo.cpu().numpy(), nhi.cpu().numpy(), nst


def test_noalloc_equals_render_bounds_two_calls_smaller_second():
    api = _api()
    from oracle import splat
    # first call: the 10k-Gaussian 128x128 workload with a 3-D translation box
    scene2, intr2, box2, _ = synth.config(2)
    sc2 = api.Scene(scene2)
    lo, hi, st, nlo, nhi, nst = _both(api, sc2, intr2, box2)
    print("call 1: pairs", st["pairs"], nst["pairs"], flush=True)
    assert np.array_equal(lo, nlo) and np.array_equal(hi, nhi)
    assert nst["pairs"] == st["pairs"] and nst["tile_pairs"] == st["tile_pairs"]
    sc2.close()
    # second call, smaller: 64 Gaussians, 32x32, x-translation box
    scene1, intr1, box1, _ = synth.config(1)
    sc1 = api.Scene(scene1)
    lo, hi, st, nlo, nhi, nst = _both(api, sc1, intr1, box1)
    print("call 2: pairs", st["pairs"], nst["pairs"], flush=True)
    assert np.array_equal(lo, nlo) and np.array_equal(hi, nhi)
    ref = splat.oracle_bounds(scene1, intr1, box1)
    assert np.abs(nlo - ref["lo"]).max() <= TOL and np.abs(nhi - ref["hi"]).max() <= TOL
    # a ragged image (not a multiple of the tile) and a zero-width box
    intr = synth.intrinsics(37)
    for box in (synth.camera6_box(dt=(0.02, 0.01, 0.0)), synth.camera6_box()):
        lo, hi, st, nlo, nhi, nst = _both(api, sc1, intr, box)
        assert np.array_equal(lo, nlo) and np.array_equal(hi, nhi)
    sc1.close()


def test_noalloc_rejects_what_it_does_not_hold():
    api = _api()
    import torch
    scene = synth.random_scene(300, seed=4)
    intr = synth.intrinsics(32)
    sc = api.Scene(scene)
    lo = torch.empty((32, 32, 3), dtype=torch.float32, device="cuda")
    hi = torch.empty_like(lo)
    with pytest.raises(api.ARError) as ei:
        api.render_bounds_noalloc(sc, intr, synth.camera6_box(dt=0.01, drot=0.01), (lo, hi))
    assert ei.value.code == api.AR_E_UNSUPPORTED and "translation" in str(ei.value)
    # more Gaussians than the scratch holds records for: rejected before any launch
    big = api.Scene(synth.random_scene(250_000, seed=5))
    with pytest.raises(api.ARError) as ei:
        api.render_bounds_noalloc(big, intr, synth.camera6_box(dt=0.01), (lo, hi))
    assert ei.value.code == api.AR_E_UNSUPPORTED and "scratch" in str(ei.value)
    big.close()
    # lists beyond the scratch: rejected when they are sized, mid-way
    wide = api.Scene(synth.random_scene(60_000, seed=6))
    intr_w = synth.intrinsics(256)
    lw = torch.empty((256, 256, 3), dtype=torch.float32, device="cuda")
    hw = torch.empty_like(lw)
    with pytest.raises(api.ARError) as ei:
        api.render_bounds_noalloc(wide, intr_w, synth.camera6_box(dt=0.1), (lw, hw))
    assert ei.value.code == api.AR_E_UNSUPPORTED and "scratch" in str(ei.value)
    wide.close()
    # the next call is exact again
    box = synth.camera6_box(dt=0.03)
    rlo, rhi, _ = api.render_bounds(sc, intr, box)
    api.render_bounds_noalloc(sc, intr, box, (lo, hi))
    torch.cuda.synchronize()
    assert torch.equal(rlo, lo) and torch.equal(rhi, hi)
    sc.close()
