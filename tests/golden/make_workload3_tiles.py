"""Writes workload3_tiles.npz: the oracle's bounds on 8x8 tiles of the full-size
workload 3 (100k Gaussians on 20 boxes, 400x400, translation +-0.05 and yaw/pitch/roll
+-1 deg): two dense tiles (about a minute each for the FP64 oracle; their bounds are
[0, 1]) and three sparse ones whose upper bounds fall below 1.  Calls only the oracle and
the seeded scene generator.

    python tests/golden/make_workload3_tiles.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import splat                       # noqa: E402
from paper_2503_00308_amd import synth         # noqa: E402

TILES = [(25, 25), (10, 30), (9, 3), (6, 6), (42, 9)]   # two dense tiles, three with bounds below 1


def main():
    scene, intr, box, _ = synth.config(3)
    rec = splat.gaussian_forms(scene, intr, box, {"tile": 8})
    out = {"tiles": np.array(TILES, np.int32)}
    for k, (tx, ty) in enumerate(TILES):
        r = splat.oracle_bounds(scene, intr, box, {"tile": 8}, tiles=[(tx, ty)], rec=rec)
        sl = (slice(ty * 8, (ty + 1) * 8), slice(tx * 8, (tx + 1) * 8))
        out[f"lo{k}"] = r["lo"][sl]
        out[f"hi{k}"] = r["hi"][sl]
        out[f"border{k}"] = r["border"][sl]
        out[f"pairs{k}"] = r["pairs"][sl]
        print(f"tile {tx},{ty}: {int(r['pairs'][sl].sum())} pairs", flush=True)
    np.savez(os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload3_tiles.npz"), **out)


if __name__ == "__main__":
    main()
