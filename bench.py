#!/usr/bin/env python3
"""Benchmark of the abstract renderer on one MI355X.

One step = one abstract render (pose stage, per-Gaussian records, depth sort, tile
binning, per-pixel BlendInd loop) of the workload: 10k Gaussians, 128x128 image,
3-D camera-translation box of +-0.1 (P = 3 pose variables), synthetic scene.
Prints ONE JSON line with the throughput in bounded (pixel, Gaussian) pairs per
second, query latency percentiles, the roofline of the per-pixel kernel (timed with
HIP events inside the library, on the call's stream) and the FP64 CPU oracle timed
on a bounded sample of the same workload.  More objects in the same line:
"batched" (50k Gaussians on boxes, 200x200, a 30-degree orbit in 256 cells of uneven
widths, all cells through ar_render_batch with the segment length from ar_autotune,
against the per-query path), with --partitioned "partitioned" (the bench box cut into
2x2x2 cells whose bounds are united: time and mean bound width against the whole box), with
--refined "refined" (an orbit box over the batched scene bisected where MatrixInv fails), and
"served"
(Poisson queries over four resident scenes of 10k-750k Gaussians and images of
100^2-800^2 through the query server, p50/p99 latency against one-at-a-time service).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline (see the design notes for the derivation)
PEAK_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, non-packed FP32 = FP64 rate
PEAK_FP32_PACKED_TFLOPS = 157.3


# sources the translation pixel kernel (k_raster_seg) is compiled from
PIXEL_KERNEL_SOURCES = ("ar_raster.hip", "ar_blend.h", "ar_pair.h", "ar_expm.h", "ar_internal.h")


def kernel_fingerprint() -> str:
    """Hash of the pixel kernel's sources; a traffic measurement is only used while it matches."""
    h = hashlib.sha256()
    for f in [os.path.join(ROOT, "paper_2503_00308_amd", "csrc", n) for n in PIXEL_KERNEL_SOURCES]:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(path):
    """HBM bytes per launch of the per-pixel kernel from a committed counter summary
    ("key: value" lines), or None when absent or taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_fingerprint") != kernel_fingerprint():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(mib: int):
    """A plain device copy of known size, profiled with the same HBM counters to turn
    counter readings into bytes."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}), flush=True)


def served_query(index: int, seed: int = 0):
    """Query `index` of the seeded serving stream rendered alone (one warm-up, one timed
    call): one JSON line with its time and statistics, for profiling that query's kernels."""
    import torch
    from paper_2503_00308_amd import api, synth
    torch.cuda.set_device(0)
    api.load()
    s, side, box = synth.served_queries(48, seed)[index]
    scene = synth.served_scenes(seed)[s]
    h = api.Scene(scene)
    intr = synth.intrinsics(side)
    api.render_bounds(h, intr, box)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st = api.render_bounds(h, intr, box)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    h.close()
    print(json.dumps({"served_query": index, "gaussians": int(len(scene["opacity"])), "side": side,
                      "pose_vars": st["P"], "ms": ms, "stats": st}), flush=True)


def alg_flops_per_pair(P: int) -> int:
    """Algorithmic floating-point work of one (pixel, Gaussian) pair, counted on the
    operations of the method (FMA = 2 flops), F = P + 1 form coefficients:
    v = u D2 - DUP 4F FMA and its concretisation 4F; the six McCormick Mul of q
    24F + 12; the q sums 6F and their concretisation 6F; three Sqr 6F; the s sum and
    its concretisation 6F; Exp two exponentials and 2F; the alpha concretisation 2F;
    the transmittance two multiplications; the colour forms 6F + 6 FMA.  That is about
    66F + 70 operations, 110F + 70 flops.  Outward rounding is overhead, not counted."""
    return 110 * (P + 1) + 70


def cpu_baseline(scene, intr, box, budget_s=20.0):
    """FP64 oracle on a bounded sample: 4x4 pixel blocks spread over the image, as many
    as fit about budget_s seconds (at least one)."""
    import numpy as np
    from oracle import splat
    t0 = time.perf_counter()
    rec = splat.gaussian_forms(scene, intr, box, {"tile": 4})
    t_rec = time.perf_counter() - t0
    W, H = intr["width"], intr["height"]
    rng = np.random.default_rng(0)
    cand = [(int(x), int(y)) for x, y in zip(rng.integers(0, W // 4, 64), rng.integers(0, H // 4, 64))]
    pairs = 0
    blocks = 0
    t_pix = 0.0
    last = 0.0
    for tx, ty in cand:
        if blocks and t_pix + t_rec + last > budget_s:
            break
        t1 = time.perf_counter()
        r = splat.oracle_bounds(scene, intr, box, {"tile": 4}, tiles=[(tx, ty)], rec=rec)
        last = time.perf_counter() - t1
        t_pix += last
        pairs += int(r["pairs"][ty * 4:(ty + 1) * 4, tx * 4:(tx + 1) * 4].sum())
        blocks += 1
    # per-Gaussian stage is shared by the whole image: charge it pro rata to the sample
    frac = blocks * 16 / float(W * H)
    t = t_pix + t_rec * frac
    return {"value": pairs / t, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{blocks} random 4x4 pixel blocks of the workload ({pairs} pairs); the per-Gaussian "
                      f"stage ({t_rec:.1f} s for all {len(scene['mean'])} Gaussians) charged pro rata"}


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def batched_measure(api, synth, runs=2, per_query_cells=32, autotune=True):
    """All 256 orbit cells in one batched call, against one ar_render_bounds per cell."""
    import numpy as np
    import torch
    scene, intr, cells, desc = synth.config(4)
    sc = api.Scene(scene)
    opts = None
    if autotune:
        log("batched: autotune")
        opts, _, _, _ = api.autotune(sc, intr, cells, reps=1)    # also the warm-up
    else:
        log("batched: warm-up")
        api.render_batch(sc, intr, cells)       # warm-up (sizes the workspace)
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(runs):
        t0 = time.perf_counter()
        _, _, st = api.render_batch(sc, intr, cells, opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t_batch = float(np.median(times))
    log(f"batched: {t_batch:.3f} s for {len(cells)} cells; per-query path on {per_query_cells} cells")
    sub = cells[:per_query_cells]
    H, W = intr["height"], intr["width"]
    lo = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    hi = torch.empty_like(lo)
    api.render_bounds(sc, intr, sub[0], opts, out=(lo, hi))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs_sub = 0
    for c in sub:
        _, _, s1 = api.render_bounds(sc, intr, c, opts, out=(lo, hi))
        pairs_sub += s1["pairs"]
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / len(sub)
    sc.close()
    n = len(cells)
    return {"workload": desc, "cells": n, "segment_length": st["segment_length"], "autotuned": autotune,
            "pairs": int(st["pairs"]),
            "cells_per_s": n / t_batch,
            "pairs_per_s": st["pairs"] / t_batch, "ms_per_cell": t_batch / n * 1e3,
            "device_ms": st["total_ms"], "raster_ms": st["raster_ms"],
            "per_query_ms_per_cell": t_single * 1e3, "per_query_cells_timed": len(sub),
            "per_query_pairs_per_s": pairs_sub / (t_single * len(sub)),
            "speedup_vs_per_query": t_single * n / t_batch}


def partitioned_measure(api, sc, intr, box, splits=(2, 2, 2), runs=3):
    """The bench box cut into a grid of cells and united, against the whole box: time per
    partitioned render and the mean bound width of both."""
    import numpy as np
    import torch
    lo, hi, _ = api.render_partitioned(sc, intr, box, splits)     # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        lo, hi, st = api.render_partitioned(sc, intr, box, splits)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    wlo, whi, _ = api.render_bounds(sc, intr, box)
    torch.cuda.synchronize()
    width = float((hi - lo).mean().item())
    whole = float((whi - wlo).mean().item())
    cells = int(np.prod(splits))
    t = float(np.median(times))
    return {"splits": list(splits), "cells": cells, "ms": t * 1e3, "pairs_per_s": st["pairs"] / t,
            "mean_width": width, "mean_width_whole_box": whole}


def refined_measure(api, synth, deg=3.0, max_cells=64, runs=3):
    """Adaptive refinement (cells bisected where MatrixInv fails, united) of one orbit box
    over the batched workload's scene: time, leaves, and the mean bound width against the
    whole box and against an even cut into as many cells."""
    import numpy as np
    import torch
    scene = synth.box_surface_scene(50_000, n_boxes=20, seed=0)
    intr = synth.intrinsics(200)
    a = np.deg2rad(deg)
    box = {"model": synth.ORBIT, "R0": np.eye(3), "t0": np.zeros(3), "pivot": np.array([0.0, 0.0, 4.0]),
           "lo": np.array([-a, 0, 0, 0, 0, 0]), "hi": np.array([a, 0, 0, 0, 0, 0])}
    sc = api.Scene(scene)
    api.render_refined(sc, intr, box, max_cells)      # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        lo, hi, leaves, st = api.render_refined(sc, intr, box, max_cells)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    width = float((hi - lo).mean().item())
    wlo, whi, _ = api.render_bounds(sc, intr, box)
    plo, phi, _ = api.render_partitioned(sc, intr, box, (len(leaves),))
    torch.cuda.synchronize()
    counts = api.classify_cells(sc, intr, [box] + leaves)
    n = len(leaves)
    even = []
    for k in range(n):
        c = {**box, "lo": box["lo"].copy(), "hi": box["hi"].copy()}
        c["lo"][0] = -a + 2 * a * k / n
        c["hi"][0] = a if k + 1 == n else -a + 2 * a * (k + 1) / n
        even.append(c)
    even_counts = api.classify_cells(sc, intr, even)
    out = {"workload": f"50k Gaussians on 20 boxes, 200x200, orbit +-{deg:g} deg, at most {max_cells} cells",
           "ms": t * 1e3, "leaves": len(leaves), "pairs_per_s": st["pairs"] / t,
           "matinv_failures_whole_box": int(counts[0, 0]), "leaves_with_failures": int(np.count_nonzero(counts[1:, 0])),
           "mean_width": width, "mean_width_whole_box": float((whi - wlo).mean().item()),
           "mean_width_even_cut": float((phi - plo).mean().item()),
           "even_cut_cells_with_failures": int(np.count_nonzero(even_counts[:, 0]))}
    sc.close()
    return out


def served_measure(api, synth, nq=48, load=0.75, slots=4, seed=0):
    """Poisson arrivals at `load` x the one-at-a-time capacity; the server's latencies
    against a FIFO one-at-a-time queue with each query's measured solo service time."""
    import numpy as np
    import torch
    log("served: scenes")
    scenes = synth.served_scenes(seed)
    handles = [api.Scene(s) for s in scenes]
    queries = synth.served_queries(nq, seed)
    # solo service times (the plain per-query path), each query once after a warm-up
    for s in range(len(handles)):
        side = (100, 200, 400, 800)[s]
        api.render_bounds(handles[s], synth.intrinsics(side), synth.camera6_box(dt=0.01))
    torch.cuda.synchronize()
    service, pairs = [], 0
    for i, (s, side, box) in enumerate(queries):
        t0 = time.perf_counter()
        _, _, st = api.render_bounds(handles[s], synth.intrinsics(side), box)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        pairs += st["pairs"]
        log(f"served: solo query {i} scene {s} side {side}: {service[-1] * 1e3:.1f} ms, {st['pairs']} pairs")
    service = np.array(service)
    lam = load / service.mean()
    rng = np.random.default_rng(seed + 1)
    arrival = np.cumsum(rng.exponential(1.0 / lam, nq))
    arrival -= arrival[0]
    # one at a time, first come first served
    finish = np.empty(nq)
    t = 0.0
    for i in range(nq):
        t = max(t, arrival[i]) + service[i]
        finish[i] = t
    serial_lat = (finish - arrival) * 1e3
    # the server, queries submitted at their arrival times
    log(f"served: server run, {nq} queries at {lam:.1f} per s")
    srv = api.Server(slots=slots)
    ids = [srv.add_scene(h) for h in handles]
    tickets = []
    t0 = time.perf_counter()
    for i, (s, side, box) in enumerate(queries):
        now = time.perf_counter() - t0
        if arrival[i] > now:
            time.sleep(arrival[i] - now)
        tickets.append(srv.submit(ids[s], synth.intrinsics(side), box))
    lat = []
    for tk in tickets:
        _, _, res = srv.wait(tk)
        lat.append(res["latency_ms"])
    wall = time.perf_counter() - t0
    rep = srv.report()
    srv.close()
    for h in handles:
        h.close()
    lat = np.array(lat)
    return {"workload": "Poisson queries over resident scenes of 10k/100k/300k/750k Gaussians on boxes, "
                        "images 100^2-800^2, translation full widths U[0.01,0.1], rotation U[0,2] deg",
            "queries": nq, "load": load, "arrival_qps": lam, "slots": slots,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "throughput_qps": nq / wall, "pairs_per_s": pairs / wall, "peak_inflight": rep["peak_inflight"],
            "peak_workspace_bytes": rep["peak_bytes"],
            "one_at_a_time": {"p50_ms": float(np.percentile(serial_lat, 50)),
                              "p99_ms": float(np.percentile(serial_lat, 99)),
                              "mean_service_ms": float(service.mean() * 1e3),
                              "throughput_qps": nq / finish[-1]}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="batched workload: automatic segment length")
    ap.add_argument("--refined", action="store_true",
                    help="also an orbit box refined where MatrixInv fails (left out of the default run, as "
                         "--partitioned)")
    ap.add_argument("--partitioned", action="store_true",
                    help="also the bench box cut into 2x2x2 cells (its pixel-kernel launches are of another size, "
                         "so it is left out of the default run that the kernel trace covers)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_raster_seg_cfg2_traffic.txt"))
    ap.add_argument("--served-query", type=int, default=None, metavar="K",
                    help="only render query K of the seeded serving stream alone (twice) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: sharding over several GPUs is designed but not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.served_query is not None:
        served_query(args.served_query)
        return

    import numpy as np
    import torch
    from paper_2503_00308_amd import api, synth

    torch.cuda.set_device(0)
    scene, intr, box, desc = synth.config(2)
    sc = api.Scene(scene)
    H, W = intr["height"], intr["width"]
    lo = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    hi = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    opts = None   # the automatic segment length (measured rule); the batch below is autotuned
    for _ in range(args.warmup):
        api.render_bounds(sc, intr, box, opts, out=(lo, hi))
    torch.cuda.synchronize()
    lat, raster_ms, pairs = [], [], []
    stats = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, _, stats = api.render_bounds(sc, intr, box, opts, out=(lo, hi))
        lat.append(time.perf_counter() - ts)
        raster_ms.append(stats["raster_ms"])
        pairs.append(stats["pairs"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P = stats["P"]
    value = float(np.sum(pairs)) / elapsed
    mean_pairs = float(np.mean(pairs))
    mean_raster_s = float(np.mean(raster_ms)) * 1e-3
    achieved = alg_flops_per_pair(P) * mean_pairs / mean_raster_s / 1e12
    traffic = read_traffic(args.traffic)
    out = {
        "metric": "bounded pixel-Gaussian pairs/sec",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": len(scene["mean"]), "image": [W, H], "pose_vars": P,
                   "tile": 8, "segment_length": stats["segment_length"], "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "pairs_per_step": mean_pairs,
        "tile_pairs_per_step": stats["tile_pairs"],
        "raster_ms": float(np.mean(raster_ms)),
        "device_ms_per_step": stats["total_ms"],
        "roofline": {"bound": "alu", "kernel": "k_raster_seg", "achieved": achieved,
                     "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                     "frac_vs_packed_fp32_peak": achieved / PEAK_FP32_PACKED_TFLOPS,
                     "flops_per_pair": alg_flops_per_pair(P), "traffic": traffic},
    }
    log(f"headline workload done: {value:.4g} pairs/s")
    if args.partitioned:
        out["partitioned"] = partitioned_measure(api, sc, intr, box)
    sc.close()
    if args.refined:
        out["refined"] = refined_measure(api, synth)
    if not args.no_batched:
        out["batched"] = batched_measure(api, synth, autotune=not args.no_autotune)
    if not args.no_served:
        out["served"] = served_measure(api, synth)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, intr, box, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
