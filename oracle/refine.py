"""Adaptive refinement of a pose box, FP64 (test infrastructure only).

Sec. 3.1 makes MatrixInv sound on a set of input matrices only where its convergence
assertion holds, and asks for the input range to be divided until it does; Sec. 4.2
renders subsets of the camera set and unites their bounds.  Here the divided range is
the pose box:

* a cell is flagged when it holds a Gaussian whose MatrixInv assertion fails and that
  the pruning test keeps at some pixel of the image (criterion `matinv`), or one that
  straddles the near plane, which gets alpha in [0, o] everywhere (criterion `near`), or
  when some depth-order test Ind of two Gaussians sharing a tile list stays undecided
  (criterion `ind`; Sec. 3.2: Ind is piecewise constant, tight on every part of the
  domain where its argument keeps its sign, splat.ind_uncertain_count);
* cells are taken level by level, in order; a flagged cell of depth k (k bisections
  from the whole box) is cut in two at the midpoint 0.5 (lo + hi) of its active axis
  number k mod (number of active axes), as long as the number of cells stays within
  max_cells and k < MAX_DEPTH; the halves join the next level, lower half first;
* the leaves, in the order they are settled, are the cells rendered; the bounds are
  the elementwise minimum of their lower and maximum of their upper images.

Pinned by tests/test_oracle_refine.py: the leaves tile the box, a box with nothing
flagged is its own single leaf, the budget caps the count, every sampled concrete
render lies inside the united bounds (the soundness theorem), and refinement removes
the failures it was made for.
"""
import copy

import numpy as np

from . import pose, splat

MAX_DEPTH = 24


def active_axes(box):
    """Axes of the box with a positive width (ORBIT: its angle only)."""
    na = 1 if box.get("model", pose.CAMERA6) == pose.ORBIT else 6
    return [a for a in range(na) if float(box["hi"][a]) > float(box["lo"][a])]


def flagged_counts(scene, intr, box, opts=None):
    """(Gaussians kept somewhere in the image whose MatrixInv assertion fails,
    Gaussians straddling the near plane) for one cell."""
    rec = splat.gaussian_forms(scene, intr, box, opts)
    keep = splat.tile_candidates(rec, intr, 0, int(intr["width"]), 0, int(intr["height"]))
    return int(np.count_nonzero(rec["fallback"][keep])), int(np.count_nonzero(rec["wild"]))


def _half(box, a, upper):
    out = copy.deepcopy(box)
    out["lo"] = np.array(box["lo"], np.float64).copy()
    out["hi"] = np.array(box["hi"], np.float64).copy()
    m = 0.5 * (float(box["lo"][a]) + float(box["hi"][a]))
    if upper:
        out["lo"][a] = m
    else:
        out["hi"][a] = m
    return out


def refine(scene, intr, box, max_cells, near=False, opts=None, matinv=True, ind=False):
    """Leaves of the refinement, in the order they are settled (criteria: MatrixInv
    failures kept in the image when matinv, near-plane straddlers when near, undecided
    Ind tests when ind)."""
    axes = active_axes(box)
    level = [(box, 0)]
    leaves = []
    total = 1
    while level:
        nxt = []
        for cell, depth in level:
            fb, wild = flagged_counts(scene, intr, cell, opts)
            flagged = (matinv and fb > 0) or (near and wild > 0)
            if ind and not flagged:
                flagged = splat.ind_uncertain_count(scene, intr, cell, opts)[0] > 0
            if flagged and axes and depth < MAX_DEPTH and total + 1 <= max_cells:
                a = axes[depth % len(axes)]
                lo, hi = float(cell["lo"][a]), float(cell["hi"][a])
                m = 0.5 * (lo + hi)
                if lo < m < hi:
                    total += 1
                    nxt.append((_half(cell, a, False), depth + 1))
                    nxt.append((_half(cell, a, True), depth + 1))
                    continue
            leaves.append(cell)
        level = nxt
    return leaves


def refined_bounds(scene, intr, box, max_cells, near=False, opts=None, matinv=True, ind=False):
    """United lower / upper images of the leaves (H, W, 3), and the leaves."""
    leaves = refine(scene, intr, box, max_cells, near, opts, matinv, ind)
    lo = hi = None
    for cell in leaves:
        r = splat.oracle_bounds(scene, intr, cell, opts)
        lo = r["lo"] if lo is None else np.minimum(lo, r["lo"])
        hi = r["hi"] if hi is None else np.maximum(hi, r["hi"])
    return lo, hi, leaves
