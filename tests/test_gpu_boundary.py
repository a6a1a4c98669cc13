"""Boundary inputs and outputs through the C ABI: scenes given by rotation quaternion and
scales (Mw = R(q) diag(s), formed by the library) and images written to host memory.

Bar: a scene given by quaternions and scales renders as the same scene given by its
covariance factors (within float32 rounding of the factors, and within 1e-5 of the
oracle); host outputs (pinned or pageable, single render and batch) equal the device
outputs bit for bit; bad quaternions, scales and mixed outputs are rejected.
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


def _quat_scene(n=300, seed=4):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, (n, 3)) + np.array([0.0, 0.0, 4.0])
    q = rng.standard_normal((n, 4))
    q[::7] *= 3.0                                   # not unit length: normalised by the library
    s = np.exp(rng.uniform(np.log(0.02), np.log(0.2), (n, 3)))
    op = rng.uniform(0.1, 0.9, n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    qs = {"mean": mean.astype(np.float32), "quat": q.astype(np.float32), "scale": s.astype(np.float32),
          "opacity": op.astype(np.float32), "rgb": rgb.astype(np.float32)}
    # the same scene by its factors, formed in FP64 from the float32 inputs
    cov = synth._pack(qs["mean"].astype(np.float64), synth._quat_to_rot(qs["quat"].astype(np.float64)),
                      qs["scale"].astype(np.float64), op, rgb)
    return qs, cov


@pytest.mark.parametrize("box", [synth.camera6_box(dt=0.03),
                                 synth.camera6_box(dt=0.01, drot=(np.deg2rad(0.5), np.deg2rad(0.3), 0.0))],
                         ids=["translation", "rotation"])
def test_quaternion_scale_scene_equals_its_factors(box):
    import torch
    from oracle import splat
    api = _api()
    qs, cov = _quat_scene()
    intr = synth.intrinsics(32)
    a, b = api.Scene(qs), api.Scene(cov)
    lo_q, hi_q, _ = api.render_bounds(a, intr, box)
    lo_c, hi_c, _ = api.render_bounds(b, intr, box)
    torch.cuda.synchronize()
    lo_q, hi_q, lo_c, hi_c = (t.cpu().numpy() for t in (lo_q, hi_q, lo_c, hi_c))
    a.close()
    b.close()
    d = max(np.abs(lo_q - lo_c).max(), np.abs(hi_q - hi_c).max())
    print(f"quaternion scene vs factors: max difference {d:.2e}", flush=True)
    assert d <= 1e-6
    ref = splat.oracle_bounds(cov, intr, box)
    assert np.abs(lo_q - ref["lo"]).max() <= TOL and np.abs(hi_q - ref["hi"]).max() <= TOL


def test_bad_quaternions_and_scales_are_rejected():
    api = _api()
    qs, _ = _quat_scene(20)
    for key, idx, val in (("quat", (3, slice(None)), 0.0), ("scale", (5, 1), -0.1), ("quat", (2, 0), np.nan)):
        bad = {k: v.copy() for k, v in qs.items()}
        bad[key][idx] = val
        with pytest.raises(api.ARError) as ei:
            api.Scene(bad)
        assert ei.value.code == api.AR_E_INVALID, key


@pytest.mark.parametrize("pinned", [False, True])
def test_host_outputs_equal_device_outputs(pinned):
    import torch
    api = _api()
    scene = synth.random_scene(400, seed=8)
    intr = synth.intrinsics(40)
    box = synth.camera6_box(dt=0.01, drot=np.deg2rad(0.3))
    sc = api.Scene(scene)
    dlo, dhi, _ = api.render_bounds(sc, intr, box)
    hlo = torch.empty((40, 40, 3), dtype=torch.float32, pin_memory=pinned)
    hhi = torch.empty_like(hlo, pin_memory=pinned)
    api.render_bounds(sc, intr, box, out=(hlo, hhi))
    assert np.array_equal(hlo.numpy(), dlo.cpu().numpy()) and np.array_equal(hhi.numpy(), dhi.cpu().numpy())
    cells = [synth.camera6_box(dt=0.01 * (k + 1)) for k in range(3)]
    blo, bhi, _ = api.render_batch(sc, intr, cells)
    hblo = torch.empty((3, 40, 40, 3), dtype=torch.float32, pin_memory=pinned)
    hbhi = torch.empty_like(hblo, pin_memory=pinned)
    api.render_batch(sc, intr, cells, out=(hblo, hbhi))
    assert np.array_equal(hblo.numpy(), blo.cpu().numpy()) and np.array_equal(hbhi.numpy(), bhi.cpu().numpy())
    # one output on the host and one on the device
    with pytest.raises(api.ARError) as ei:
        api.render_bounds(sc, intr, box, out=(hlo, dhi))
    assert ei.value.code == api.AR_E_INVALID
    sc.close()
