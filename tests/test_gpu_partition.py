"""Pose boxes cut into a grid of cells (Sec. 4.2: bounds computed per subset of the
cameras and united), through the C ABI.

The partitioned render must equal the union of the cells rendered one by one (bit for
bit with a fixed segment length), match the union of the oracle's bounds of the cells,
enclose sampled concrete renders, and be no looser than the whole box on average.
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


def _cells(box, splits):
    """The grid of cells, cut as the library cuts it."""
    na = 1 if box.get("model", 0) == 1 else 6
    s = [(splits[a] if box["hi"][a] > box["lo"][a] else 1) if a < na else 1 for a in range(6)]
    out = []
    for c in range(int(np.prod(s))):
        r = c
        cell = {k: (np.array(v, np.float64).copy() if isinstance(v, np.ndarray) else v) for k, v in box.items()}
        for a in range(na):
            k = r % s[a]
            r //= s[a]
            if s[a] == 1:
                continue
            lo, w = float(box["lo"][a]), float(box["hi"][a]) - float(box["lo"][a])
            cell["lo"][a] = lo + w * k / s[a]
            cell["hi"][a] = float(box["hi"][a]) if k + 1 == s[a] else lo + w * (k + 1) / s[a]
        out.append(cell)
    return out


def test_partition_equals_union_of_cells():
    api = _api()
    scene = synth.random_scene(300, seed=41)
    intr = synth.intrinsics(40)
    box = synth.camera6_box(dt=(0.06, 0.04, 0.0))
    sc = api.Scene(scene)
    opts = {"chunk": 32}
    plo, phi, st = api.render_partitioned(sc, intr, box, (3, 2), opts)
    plo, phi = plo.cpu().numpy(), phi.cpu().numpy()
    cells = _cells(box, (3, 2))
    assert len(cells) == 6
    ulo = np.full(plo.shape, np.inf, np.float32)
    uhi = np.full(phi.shape, -np.inf, np.float32)
    for c in cells:
        lo, hi, _ = api.render_bounds(sc, intr, c, opts)
        ulo = np.minimum(ulo, lo.cpu().numpy())
        uhi = np.maximum(uhi, hi.cpu().numpy())
    sc.close()
    print("partition stats", st, flush=True)
    assert np.array_equal(plo, ulo) and np.array_equal(phi, uhi)


def test_partition_parity_soundness_and_tightening():
    from oracle import pose, render, splat
    api = _api()
    scene = synth.random_scene(150, seed=42)
    intr = synth.intrinsics(32)
    box = synth.camera6_box(dt=(0.05, 0.0, 0.03), drot=(0.0, np.deg2rad(1.0), 0.0))
    splits = (2, 1, 2, 1, 2, 1)
    sc = api.Scene(scene)
    plo, phi, _ = api.render_partitioned(sc, intr, box, splits)
    wlo, whi, _ = api.render_bounds(sc, intr, box)
    sc.close()
    plo, phi = plo.cpu().numpy().astype(np.float64), phi.cpu().numpy().astype(np.float64)
    wlo, whi = wlo.cpu().numpy().astype(np.float64), whi.cpu().numpy().astype(np.float64)
    # the oracle's union over the same cells
    rlo = np.full(plo.shape, np.inf)
    rhi = np.full(phi.shape, -np.inf)
    border = np.zeros(plo.shape[:2], bool)
    for c in _cells(box, splits):
        ref = splat.oracle_bounds(scene, intr, c)
        rlo = np.minimum(rlo, ref["lo"])
        rhi = np.maximum(rhi, ref["hi"])
        border |= ref["border"]
    ok = np.broadcast_to(~border[..., None], plo.shape)
    dlo, dhi = np.abs(plo - rlo)[ok].max(), np.abs(phi - rhi)[ok].max()
    print(f"[partition] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
    assert dlo <= TOL and dhi <= TOL
    rng = np.random.default_rng(5)
    worst = -np.inf
    for p in pose.sample_poses(box, 24, rng):
        img = render.render(scene, intr, box, p)
        worst = max(worst, (plo - img).max(), (img - phi).max())
    print(f"[partition] soundness worst {worst:.3e}", flush=True)
    assert worst <= 1e-7
    wp, ww = (phi - plo).mean(), (whi - wlo).mean()
    print(f"[partition] mean width {wp:.4f} against {ww:.4f} for the whole box", flush=True)
    assert wp <= ww


def test_partition_rejects_bad_splits():
    api = _api()
    sc = api.Scene(synth.random_scene(50, seed=43))
    with pytest.raises(api.ARError):
        api.render_partitioned(sc, synth.intrinsics(16), synth.camera6_box(dt=0.01), (0, 1))
    with pytest.raises(api.ARError):
        api.render_partitioned(sc, synth.intrinsics(16), synth.camera6_box(dt=0.01), (300, 300, 300))
    sc.close()
