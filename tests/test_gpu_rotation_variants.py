"""Rotation path (Alg. BlendInd with three-valued Ind) against the FP64 oracle where the
lower bounds are informative, and every layout switch of that path compared bit for bit.

The rotation path picks three layouts from the size of a call (absolute running sums,
the compact copy for the Ind tests, stored Ind masks of long windows) and splits long
list sets into groups.  Small workloads never reach the automatic thresholds, so every
switch is forced on and off here on small scenes, with P = 1 and P = 4, 5, 6 pose
variables, and the Ind windows both narrow (default) and whole-list (every pair tested:
windows longer than 64 positions, the wave-wide walk and the stored masks).  Each case
asserts that a stated share of the oracle's lower bounds is informative (above 1e-4),
so the lower-transmittance arithmetic is compared at non-zero values.
"""
import itertools

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


def _render(api, handle, intr, box, opts=None):
    import torch
    lo, hi, st = api.render_bounds(handle, intr, box, opts)
    torch.cuda.synchronize()
    return lo.cpu().numpy().astype(np.float64), hi.cpu().numpy().astype(np.float64), st


def _compare(name, glo, ghi, ref):
    ok = ~ref["border"][..., None] & np.isfinite(ref["lo"])
    ok = np.broadcast_to(ok, ref["lo"].shape)
    dlo = np.abs(glo - ref["lo"])[ok]
    dhi = np.abs(ghi - ref["hi"])[ok]
    print(f"[{name}] max|dlo| {dlo.max():.3e} max|dhi| {dhi.max():.3e} "
          f"(oracle lo > 1e-4 at {(ref['lo'] > 1e-4).mean():.2f} of values)", flush=True)
    assert dlo.max() <= TOL and dhi.max() <= TOL


def _sound(name, scene, intr, box, glo, ghi, n=16):
    from oracle import pose, render
    rng = np.random.default_rng(5)
    worst = -np.inf
    for p in pose.sample_poses(box, n, rng):
        img = render.render(scene, intr, box, p)
        worst = max(worst, (glo - img).max(), (img - ghi).max())
    print(f"[{name}] soundness worst {worst:.3e}", flush=True)
    assert worst <= 1e-7


# (name, scene, side, box, stated share of oracle lower bounds above 1e-4)
def _cases():
    deg = np.deg2rad
    return {
        "P6": (synth.random_scene(200, seed=3), 32, synth.camera6_box(dt=0.01, drot=deg(0.2)), 0.4),
        "P5": (synth.random_scene(200, seed=3), 32,
               synth.camera6_box(dt=(0.01, 0.01, 0.0), drot=deg(0.2)), 0.4),
        "P4": (synth.random_scene(200, seed=3), 32,
               synth.camera6_box(dt=(0.01, 0.0, 0.0), drot=deg(0.2)), 0.4),
        "P1": (synth.random_scene(200, seed=3), 32, synth.camera6_box(drot=(0.0, 0.0, deg(0.5))), 0.4),
        # Gaussians on box faces cover part of the image only
        "boxes6": (synth.box_surface_scene(800, n_boxes=6, seed=2), 40,
                   synth.camera6_box(dt=0.002, drot=deg(0.03)), 0.1),
    }


@pytest.mark.parametrize("case", ["P6", "P5", "P4", "P1", "boxes6"])
def test_informative_lower_bounds_parity(case):
    from oracle import splat
    api = _api()
    scene, side, box, share = _cases()[case]
    intr = synth.intrinsics(side)
    h = api.Scene(scene)
    glo, ghi, st = _render(api, h, intr, box)
    h.close()
    ref = splat.oracle_bounds(scene, intr, box)
    frac = float((ref["lo"] > 1e-4).mean())
    print(f"[{case}] P {st['P']} runs {st['runs']} max window {st['max_window']} pairs {st['pairs']}", flush=True)
    assert frac >= share, frac
    assert st["P"] == ref["rec"]["P"]
    _compare(case, glo, ghi, ref)
    _sound(case, scene, intr, box, glo, ghi)


# every combination of the three layout switches (1 on, 2 off), with narrow and with
# whole-list Ind windows, and the Ind passes over small list groups
_SWITCHES = [dict(abs_sums=a, ind_copy=c, ind_masks=m) for a, c, m in itertools.product((1, 2), (1, 2), (1, 2))]


@pytest.mark.parametrize("case", ["P6", "P1", "boxes6"])
def test_layout_switches_bit_identical_and_pinned(case):
    from oracle import splat
    api = _api()
    scene, side, box, share = _cases()[case]
    intr = synth.intrinsics(side)
    h = api.Scene(scene)
    base = _render(api, h, intr, box)
    ref = splat.oracle_bounds(scene, intr, box)
    assert float((ref["lo"] > 1e-4).mean()) >= share
    _compare(f"{case}-auto", base[0], base[1], ref)
    n_long = 0
    for window in (0, 2):
        for sw in _SWITCHES + [dict(group_entries=37), dict(group_entries=1, abs_sums=1, ind_copy=1)]:
            opts = dict(sw, ind_window=window)
            lo, hi, st = _render(api, h, intr, box, opts)
            n_long += st["max_window"] > 64
            same = np.array_equal(lo, base[0]) and np.array_equal(hi, base[1])
            if not same:
                print(f"[{case}] {opts}: max diff lo {np.abs(lo - base[0]).max():.3e} "
                      f"hi {np.abs(hi - base[1]).max():.3e}", flush=True)
            assert same, opts
    h.close()
    # whole-list windows reach the wave-wide walk and the stored masks (windows > 64)
    print(f"[{case}] renders with windows longer than 64 positions: {n_long}", flush=True)
    if case != "P1":
        assert n_long > 0


def test_run_limit_regroups_lists_bit_identical():
    """A list group whose Ind runs exceed group_runs (the uint32 offsets at full size) is cut
    into smaller groups of whole lists and done again: the same images bit for bit; a
    single list over the limit is rejected."""
    api = _api()
    scene = synth.random_scene(400, seed=8)
    intr = synth.intrinsics(64)
    box = synth.camera6_box(dt=0.01, drot=np.deg2rad(0.3))
    h = api.Scene(scene)
    base = _render(api, h, intr, box)
    runs = int(base[2]["runs"])
    print(f"runs {runs}, list entries {base[2]['tile_pairs']}", flush=True)
    for cap in (runs // 2, runs // 5):
        lo, hi, st = _render(api, h, intr, box, {"group_runs": cap})
        assert np.array_equal(lo, base[0]) and np.array_equal(hi, base[1]), cap
        assert st["runs"] == runs
    with pytest.raises(api.ARError) as ei:
        _render(api, h, intr, box, {"group_runs": 1})
    assert ei.value.code == api.AR_E_UNSUPPORTED and "one tile list" in str(ei.value)
    h.close()


def test_quick_ind_test_changes_nothing():
    """The quick Ind test (options.ind_quick) fires only where the full identity bound
    decides the same way, so switching it off changes nothing but the number of tests
    (with it, whole chunks of 64 list positions it decides at once leave the windows):
    the same images, Ind runs, undecided and borderline counts, bit for bit, on the
    six-axis, one-angle and orbit cases and on the 100k-Gaussian object scene over six
    axes (400x400), whose windows hold millions of tests the quick test decides."""
    api = _api()
    cases = [(name, c[0], synth.intrinsics(c[1]), [c[2]]) for name, c in _cases().items()]
    cases.append(("orbit", synth.box_surface_scene(1500, n_boxes=8, seed=32), synth.intrinsics(48),
                  synth.orbit_cells(4, 10.0, seed=3)))
    scene3, intr3, box3, _ = synth.config(3)
    cases.append(("workload3", scene3, intr3, [box3]))
    for name, scene, intr, cells in cases:
        h = api.Scene(scene)
        got = []
        for opts in (None, {"ind_quick": 2}):
            lo, hi, st = api.render_batch(h, intr, cells, opts)
            und = api.count_ind_uncertain(h, intr, cells, opts)
            got.append((lo.cpu().numpy(), hi.cpu().numpy(), st, und))
        h.close()
        (l1, h1, s1, u1), (l2, h2, s2, u2) = got
        print(f"[{name}] runs {s1['runs']} / {s2['runs']}, Ind tests {s1['ind_tests']}, undecided "
              f"{int(u1.sum())} / {int(u2.sum())}, borderline {s1['ind_borderline']} / {s2['ind_borderline']}, "
              f"{s1['total_ms']:.1f} / {s2['total_ms']:.1f} ms", flush=True)
        assert s1["runs"] == s2["runs"] and s1["ind_tests"] <= s2["ind_tests"]
        assert s1["ind_borderline"] == s2["ind_borderline"]
        assert np.array_equal(u1, u2)
        assert np.array_equal(l1, l2) and np.array_equal(h1, h2)
