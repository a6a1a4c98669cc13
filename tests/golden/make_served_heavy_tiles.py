"""Writes served_heavy_tiles.npz: the oracle's bounds on 8x8 tiles of the heaviest query
of the serving workload (query 0 of the seeded stream: 750k Gaussians on 20 boxes,
400x400, all six pose axes), the largest scene and box the serving tests run: two dense
tiles (19k and 4.7k candidate Gaussians; bounds [0, 1]; about eight minutes for the FP64
oracle) and four sparse ones whose upper bounds fall below 1.  Calls only the oracle and
the seeded generators.

    python tests/golden/make_served_heavy_tiles.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import splat                       # noqa: E402
from paper_2503_00308_amd import synth         # noqa: E402

QUERY = 0
TILES = [(25, 25), (10, 40), (42, 33), (12, 9), (6, 21), (6, 12)]   # two dense, four with bounds below 1


def main():
    s, side, box = synth.served_queries(48, 0)[QUERY]
    scene = synth.served_scenes(0)[s]
    intr = synth.intrinsics(side)
    t0 = time.time()
    rec = splat.gaussian_forms(scene, intr, box, {"tile": 8})
    print(f"per-Gaussian stage of {len(scene['opacity'])} Gaussians: {time.time() - t0:.0f} s", flush=True)
    out = {"tiles": np.array(TILES, np.int32), "query": np.int32(QUERY)}
    for k, (tx, ty) in enumerate(TILES):
        t0 = time.time()
        r = splat.oracle_bounds(scene, intr, box, {"tile": 8}, tiles=[(tx, ty)], rec=rec)
        sl = (slice(ty * 8, (ty + 1) * 8), slice(tx * 8, (tx + 1) * 8))
        out[f"lo{k}"] = r["lo"][sl]
        out[f"hi{k}"] = r["hi"][sl]
        out[f"border{k}"] = r["border"][sl]
        out[f"pairs{k}"] = r["pairs"][sl]
        print(f"tile {tx},{ty}: {int(r['pairs'][sl].sum())} pairs, {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(os.path.dirname(os.path.abspath(__file__)), "served_heavy_tiles.npz"), **out)


if __name__ == "__main__":
    main()
