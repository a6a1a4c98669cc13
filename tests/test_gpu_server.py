"""Query server (continuous batching over resident scenes), through the C ABI.

Each query's bounds must be the same alone and in a mix of concurrent queries (same
kernels, its own workspace and stream), bit for bit; admission must follow the memory
budget; results are pinned to the oracle.
"""
import numpy as np
import pytest

from paper_2503_00308_amd import synth

pytestmark = pytest.mark.gpu


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_00308_amd import api
    api.load()
    return api


def _workload(seed=0, nq=24):
    scenes = [synth.box_surface_scene(1500, n_boxes=6, seed=21), synth.random_scene(3000, seed=22),
              synth.box_surface_scene(6000, n_boxes=10, seed=23)]
    rng = np.random.default_rng(seed)
    queries = []
    for _ in range(nq):
        s = int(rng.integers(0, 3))
        side = int(rng.choice([32, 48, 64]))
        if rng.uniform() < 0.5:
            box = synth.camera6_box(dt=0.5 * rng.uniform(0.01, 0.1, 3))
        else:
            box = synth.camera6_box(dt=0.5 * rng.uniform(0.01, 0.1, 3), drot=0.5 * np.deg2rad(rng.uniform(0, 2, 3)))
        queries.append((s, synth.intrinsics(side), box))
    return scenes, queries


def _alone(api, handles, queries):
    out = []
    for s, intr, box in queries:
        lo, hi, _ = api.render_bounds(handles[s], intr, box)
        out.append((lo.cpu().numpy(), hi.cpu().numpy()))
    return out


@pytest.mark.parametrize("overlap_queue", [0, 1])
def test_server_results_same_alone_and_in_mix(overlap_queue):
    """24 queries at once (a backlog, so queries overlap under either policy)."""
    api = _api()
    scenes, queries = _workload()
    handles = [api.Scene(sc) for sc in scenes]
    srv = api.Server(slots=4, overlap_queue=overlap_queue)
    ids = [srv.add_scene(h) for h in handles]
    tickets = [srv.submit(ids[s], intr, box) for s, intr, box in queries]
    mixed = []
    for t in tickets:
        lo, hi, res = srv.wait(t)
        assert res["status"] == 0
        mixed.append((lo.cpu().numpy(), hi.cpu().numpy()))
    rep = srv.report()
    srv.close()
    print("server report", rep, flush=True)
    assert rep["completed"] == len(queries) and rep["failed"] == 0
    assert rep["peak_inflight"] >= 2
    assert rep["p99_ms"] >= rep["p50_ms"] > 0.0
    alone = _alone(api, handles, queries)
    for k, ((ml, mh), (al, ah)) in enumerate(zip(mixed, alone)):
        assert np.array_equal(ml, al) and np.array_equal(mh, ah), k
    for h in handles:
        h.close()


def test_server_overlaps_only_under_a_backlog():
    """Two queries with overlap_queue 4: the second waits for the first (one in flight);
    with overlap_queue 1 it starts beside it."""
    api = _api()
    scenes, queries = _workload(seed=2, nq=2)
    handles = [api.Scene(sc) for sc in scenes]
    peaks = {}
    for ovq in (4, 1):
        srv = api.Server(slots=4, overlap_queue=ovq)
        ids = [srv.add_scene(h) for h in handles]
        tickets = [srv.submit(ids[s], intr, box) for s, intr, box in queries]
        for t in tickets:
            assert srv.wait(t)[2]["status"] == 0
        peaks[ovq] = srv.report()["peak_inflight"]
        srv.close()
    for h in handles:
        h.close()
    assert peaks[4] == 1
    assert peaks[1] in (1, 2)
    with pytest.raises(api.ARError):
        api.Server(slots=4, overlap_queue=-1)


@pytest.mark.parametrize("batch_max", [4, 1])
def test_server_shares_launches_under_a_backlog(batch_max):
    """Queued queries of one image size and pose variables over three scenes share
    launches (up to batch_max) and still equal their own renders bit for bit;
    translation queries share only with a fixed segment length (options.chunk)."""
    api = _api()
    scenes = [synth.box_surface_scene(900, n_boxes=5, seed=31), synth.random_scene(500, seed=32),
              synth.random_scene(1200, seed=33)]
    handles = [api.Scene(sc) for sc in scenes]
    rng = np.random.default_rng(7)
    intr = synth.intrinsics(48)
    queries = []
    for k in range(12):
        box = synth.camera6_box(dt=0.5 * rng.uniform(0.005, 0.02, 3), drot=0.5 * np.deg2rad(rng.uniform(0.1, 0.6, 3)))
        queries.append((k % 3, box, None, "rot"))
    for k in range(4):
        queries.append((k % 3, synth.camera6_box(dt=0.5 * rng.uniform(0.01, 0.1, 3)), {"chunk": 64}, "trans chunk"))
    for k in range(3):
        queries.append((k % 3, synth.camera6_box(dt=0.5 * rng.uniform(0.01, 0.1, 3)), None, "trans"))
    srv = api.Server(slots=2, overlap_queue=1, batch_max=batch_max)
    ids = [srv.add_scene(h) for h in handles]
    tickets = [srv.submit(ids[s], intr, box, opts) for s, box, opts, _ in queries]
    got = [srv.wait(t) for t in tickets]
    rep = srv.report()
    srv.close()
    print("server report", rep, flush=True)
    assert rep["completed"] == len(queries) and rep["failed"] == 0
    for (s, box, opts, kind), (lo, hi, res) in zip(queries, got):
        al, ah, _ = api.render_bounds(handles[s], intr, box, opts)
        assert np.array_equal(lo.cpu().numpy(), al.cpu().numpy()) and np.array_equal(hi.cpu().numpy(), ah.cpu().numpy())
        if kind == "trans" or batch_max == 1:
            assert res["batched"] == 1
        assert 1 <= res["batched"] <= batch_max
    shared = [res["batched"] for (_, _, _, kind), (_, _, res) in zip(queries, got) if kind == "rot"]
    print(f"batch_max {batch_max}: rotation queries per launch {shared}", flush=True)
    if batch_max > 1:
        assert rep["shared_launches"] >= 1 and rep["shared_queries"] >= 2 and max(shared) > 1
    else:
        assert rep["shared_launches"] == 0
    for h in handles:
        h.close()


def test_server_budget_admits_one_query_at_a_time():
    """A budget smaller than any query: each runs only when nothing else is in flight."""
    api = _api()
    scenes, queries = _workload(seed=1, nq=8)
    handles = [api.Scene(sc) for sc in scenes]
    srv = api.Server(slots=4, hbm_budget=1)
    ids = [srv.add_scene(h) for h in handles]
    tickets = [srv.submit(ids[s], intr, box) for s, intr, box in queries]
    mixed = [srv.wait(t)[:2] for t in tickets]
    rep = srv.report()
    srv.close()
    assert rep["peak_inflight"] == 1 and rep["completed"] == len(queries)
    alone = _alone(api, handles, queries)
    for (ml, mh), (al, ah) in zip(mixed, alone):
        assert np.array_equal(ml.cpu().numpy(), al) and np.array_equal(mh.cpu().numpy(), ah)
    for h in handles:
        h.close()


def test_server_parity_with_oracle():
    from oracle import splat
    api = _api()
    scene = synth.box_surface_scene(300, n_boxes=4, seed=24)
    h = api.Scene(scene)
    srv = api.Server(slots=2)
    sid = srv.add_scene(h)
    jobs = [(synth.intrinsics(32), synth.camera6_box(dt=0.03, drot=np.deg2rad(0.5))),
            (synth.intrinsics(40), synth.camera6_box(dt=(0.05, 0.02, 0.0)))]
    tickets = [srv.submit(sid, intr, box) for intr, box in jobs]
    for t, (intr, box) in zip(tickets, jobs):
        lo, hi, _ = srv.wait(t)
        ref = splat.oracle_bounds(scene, intr, box)
        ok = ~ref["border"][..., None]
        glo, ghi = lo.cpu().numpy(), hi.cpu().numpy()
        dlo = np.abs(glo - ref["lo"])[np.broadcast_to(ok, glo.shape)].max()
        dhi = np.abs(ghi - ref["hi"])[np.broadcast_to(ok, ghi.shape)].max()
        print(f"[server] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
        assert dlo <= 1e-5 and dhi <= 1e-5
    srv.close()
    h.close()


def test_server_heaviest_query_full_size_sampled_tiles():
    """The heaviest query of the serving workload at full size (750k Gaussians on 20
    boxes, 400x400, all six pose axes) through the server; 8x8 tiles (dense ones and
    sparse ones with upper bounds below 1) against the oracle's values stored by
    tests/golden/make_served_heavy_tiles.py, every pixel finite and ordered."""
    import os
    api = _api()
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "served_heavy_tiles.npz"))
    assert sum(int((gold[f"hi{k}"] < 1.0).sum()) for k in range(len(gold["tiles"]))) > 0
    s, side, box = synth.served_queries(48, 0)[int(gold["query"])]
    scene = synth.served_scenes(0)[s]
    h = api.Scene(scene)
    srv = api.Server(slots=1)
    sid = srv.add_scene(h)
    lo, hi, res = srv.wait(srv.submit(sid, synth.intrinsics(side), box))
    srv.close()
    h.close()
    print("heaviest query", res["latency_ms"], "ms", res["stats"], flush=True)
    glo, ghi = lo.cpu().numpy(), hi.cpu().numpy()
    assert np.all(np.isfinite(glo)) and np.all(np.isfinite(ghi)) and np.all(glo <= ghi)
    for k, (tx, ty) in enumerate(gold["tiles"]):
        sl = (slice(ty * 8, (ty + 1) * 8), slice(tx * 8, (tx + 1) * 8))
        ok = ~gold[f"border{k}"][..., None]
        dlo = np.abs(glo[sl] - gold[f"lo{k}"])[np.broadcast_to(ok, glo[sl].shape)].max()
        dhi = np.abs(ghi[sl] - gold[f"hi{k}"])[np.broadcast_to(ok, ghi[sl].shape)].max()
        print(f"[heaviest query tile {tx},{ty}] max|dlo| {dlo:.3e} max|dhi| {dhi:.3e}", flush=True)
        assert dlo <= 1e-5 and dhi <= 1e-5


@pytest.mark.parametrize("opts", [None, {"ind_copy": 1, "ind_window": 2}, {"group_entries": 5000}])
def test_server_admission_estimate_covers_the_workspace(opts):
    """The admission estimate of a query (at the list density of the scene's last query
    of the same kind) is at least the workspace its slot holds afterwards, for rotation
    boxes (Ind runs, windows, stored masks, the compact copy) and translation boxes."""
    api = _api()
    scene = synth.box_surface_scene(20000, n_boxes=12, seed=26)
    h = api.Scene(scene)
    jobs = [(synth.intrinsics(96), synth.camera6_box(dt=0.02, drot=np.deg2rad(0.5))),
            (synth.intrinsics(96), synth.camera6_box(dt=(0.05, 0.02, 0.01)))]
    for intr, box in jobs:
        srv = api.Server(slots=1)
        sid = srv.add_scene(h)
        first = srv.wait(srv.submit(sid, intr, box, opts))[2]
        second = srv.wait(srv.submit(sid, intr, box, opts))[2]
        srv.close()
        print(f"[admission {opts}] P {second['stats']['P']} runs {second['stats']['runs']}: first est "
              f"{first['est_bytes'] / 2**20:.1f} MiB held {first['ws_bytes'] / 2**20:.1f} MiB; second est "
              f"{second['est_bytes'] / 2**20:.1f} MiB held {second['ws_bytes'] / 2**20:.1f} MiB", flush=True)
        assert 0 < second["ws_bytes"] <= second["est_bytes"]
    h.close()


def test_server_rejects_bad_requests():
    api = _api()
    h = api.Scene(synth.random_scene(50, seed=25))
    srv = api.Server(slots=1)
    sid = srv.add_scene(h)
    with pytest.raises(api.ARError):
        srv.submit(sid + 1, synth.intrinsics(16), synth.camera6_box(dt=0.01))
    bad = synth.camera6_box(dt=0.01)
    bad["lo"][0], bad["hi"][0] = 0.1, -0.1
    with pytest.raises(api.ARError):
        srv.submit(sid, synth.intrinsics(16), bad)
    with pytest.raises(api.ARError):
        srv.wait(12345)
    srv.close()
    for bm in (-1, 257):
        with pytest.raises(api.ARError):
            api.Server(slots=1, batch_max=bm)
    h.close()
