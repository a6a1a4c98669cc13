"""Sets of scenes (Sec. 4.6) on the GPU through the C ABI (ar_scene_create_set), against
the oracle on the same set: colour and opacity intervals, means moved by a scene
variable (with a fixed camera, as in the paper's experiments, and under pose boxes).
Bar: 1e-5 on lower and upper images; every concrete render at sampled (pose, scene)
points inside the GPU bounds; a set of zero width is the plain scene bit for bit;
rejections of what the library does not take.
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


def _render(api, scene, intr, box, opts=None):
    import torch
    sc = api.Scene(scene)
    lo, hi, st = api.render_bounds(sc, intr, box, opts)
    torch.cuda.synchronize()
    out = lo.cpu().numpy().astype(np.float64), hi.cpu().numpy().astype(np.float64), st
    sc.close()
    return out


def _samples(scene, intr, box, n, seed):
    from oracle import pose, render
    rng = np.random.default_rng(seed)
    lo = np.asarray(scene.get("set_lo", []), dtype=np.float64)
    hi = np.asarray(scene.get("set_hi", []), dtype=np.float64)
    ng = len(scene["opacity"])
    for k, p in enumerate(pose.sample_poses(box, n, rng)):
        s = lo + (hi - lo) * (rng.random(len(lo)) if k % 3 else (k // 3) % 2) if len(lo) else None
        t = (0.0, 0.0) if k % 4 == 0 else (1.0, 1.0) if k % 4 == 1 else (rng.random(ng), rng.random(ng))
        yield render.render(render.instantiate(scene, s, t[0], t[1]), intr, box, p)


CASES = [
    ("colour", ("colour",), synth.camera6_box(dt=0.03)),
    ("opacity", ("opacity",), synth.camera6_box(dt=0.03)),
    ("mean_fixed_camera", ("mean",), synth.camera6_box()),
    ("mean_rotation", ("mean",), synth.camera6_box(dt=(0.02, 0.0, 0.0), drot=(np.deg2rad(0.5), np.deg2rad(0.5), 0.0))),
    ("all_translation", ("colour", "mean", "opacity"), synth.camera6_box(dt=(0.02, 0.0, 0.02))),
]


@pytest.mark.parametrize("name,kinds,box", CASES, ids=[c[0] for c in CASES])
def test_scene_set_parity_and_soundness(name, kinds, box):
    from oracle import splat
    api = _api()
    base = synth.random_scene(300, seed=5)
    scene = synth.perturbed_scene(base, kinds, frac=0.4, shift=0.15)
    intr = synth.intrinsics(32)
    glo, ghi, st = _render(api, scene, intr, box)
    ref = splat.oracle_bounds(scene, intr, box)
    ok = ~ref["border"][..., None]
    dlo = np.abs(glo - ref["lo"])[np.broadcast_to(ok, glo.shape)].max()
    dhi = np.abs(ghi - ref["hi"])[np.broadcast_to(ok, ghi.shape)].max()
    print(f"[{name}] P {st['P']} max|dlo| {dlo:.3e} max|dhi| {dhi:.3e} mean width {(ghi - glo).mean():.4f} "
          f"lo > 1e-4 on {(ref['lo'] > 1e-4).mean():.2f}", flush=True)
    assert dlo <= TOL and dhi <= TOL
    assert (ref["lo"] > 1e-4).mean() > 0.1
    worst = -np.inf
    for img in _samples(scene, intr, box, 16, 3):
        worst = max(worst, (glo - img).max(), (img - ghi).max())
    assert worst <= 1e-7, worst


def test_zero_width_set_is_the_plain_scene_bit_for_bit():
    api = _api()
    scene = synth.random_scene(300, seed=2)
    intr = synth.intrinsics(40)
    box = synth.camera6_box(dt=0.04)
    s = dict(scene)
    s["rgb_hi"] = scene["rgb"].copy()
    s["opacity_lo"] = scene["opacity"].copy()
    a = _render(api, scene, intr, box)
    b = _render(api, s, intr, box)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_scene_set_rejections():
    import torch
    api = _api()
    base = synth.random_scene(50, seed=7)
    # more than six variables in all: a six-axis box and one scene variable
    s = synth.perturbed_scene(base, ("mean",))
    sc = api.Scene(s)
    with pytest.raises(api.ARError) as ei:
        api.render_bounds(sc, synth.intrinsics(16), synth.camera6_box(dt=0.01, drot=0.01))
    assert ei.value.code == api.AR_E_UNSUPPORTED
    # the allocation-free entry point takes plain scenes' translation boxes only
    lo = torch.empty((16, 16, 3), dtype=torch.float32, device="cuda")
    hi = torch.empty_like(lo)
    with pytest.raises(api.ARError) as ei:
        api.render_bounds_noalloc(sc, synth.intrinsics(16), synth.camera6_box(dt=0.01), (lo, hi))
    assert ei.value.code == api.AR_E_UNSUPPORTED
    sc.close()
    # bounds out of range
    bad = dict(base)
    bad["opacity_lo"] = base["opacity"] + np.float32(0.01)
    with pytest.raises(api.ARError) as ei:
        api.Scene(bad)
    assert ei.value.code == api.AR_E_INVALID
    bad = synth.perturbed_scene(base, ("mean",))
    bad["mean_var"] = np.where(bad["mean_var"] >= 0, 1, -1).astype(np.int32)
    with pytest.raises(api.ARError) as ei:
        api.Scene(bad)
    assert ei.value.code == api.AR_E_INVALID
