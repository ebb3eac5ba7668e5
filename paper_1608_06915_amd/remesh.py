"""Adaptive re-meshing driven by the entropic stabiliser.

Resolved flow drives the stabiliser gamma of Eq. gamma_min_approx to its LBGK value 2,
so its deviation measures under-resolution (Sec. IV, turbulent channel flow); the
conclusion (Sec. V) proposes it as the criterion of an adaptive refinement.  This
module turns the library's per-brick readout (elbm_gamma_indicator) into refinement
blocks of the next level and moves a running lattice onto the new layout
(elbm_transfer_state).  It holds geometry only: which bricks to refine, as boxes; the
transfer's arithmetic runs in the library's kernels.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Box = Tuple[Tuple[int, ...], Tuple[int, ...]]


def _dilate(mask: np.ndarray, r: int) -> np.ndarray:
    out = mask.copy()
    for _ in range(r):
        grown = out.copy()
        for ax in range(out.ndim):
            grown |= np.roll(out, 1, axis=ax) | np.roll(out, -1, axis=ax)
        out = grown
    return out


def _overlap(a: Box, b: Box, gap: int) -> bool:
    return all(a[0][k] <= b[1][k] + gap and b[0][k] <= a[1][k] + gap for k in range(len(a[0])))


def boxes_from_indicator(ind: np.ndarray, brick_dims: Sequence[int], level_lo: Sequence[int], threshold: float,
                         pad_bricks: int = 1, merge_gap: int = 8, lo_limit=None, hi_limit=None,
                         period=None) -> List[Box]:
    """Refinement boxes of the next level covering the bricks whose indicator exceeds
    `threshold`.

    ind: the level's per-brick indicator grid (numpy order z, y, x or y, x; -1 where a
    brick has no fluid node), brick_dims: nodes per brick along x, y, z, level_lo: the
    level index box origin (level coordinates).  Marked bricks are padded by
    `pad_bricks`, grouped into bounding boxes (boxes closer than `merge_gap` level nodes
    are merged, so that the parent keeps a bulk region between interfaces), optionally
    clipped to [lo_limit, hi_limit] (level coordinates), and returned in the next
    level's coordinates (twice the level's): (lo, hi) closed boxes, x first.  period:
    per axis the level's period (None for a non-periodic axis); a box covering a whole
    period becomes the next level's whole period (lo 0, hi 2 period - 1), which carries
    no interface along that axis.
    """
    D = ind.ndim
    marked = ind > threshold
    if not marked.any():
        return []
    marked = _dilate(marked, pad_bricks) & (ind > -1.0)
    bd = [int(brick_dims[a]) for a in range(D)]
    boxes: List[Box] = []
    for idx in zip(*np.nonzero(marked)):
        g = [int(v) for v in idx[::-1]]  # brick index along x, y, (z)
        lo = tuple(int(level_lo[a]) + g[a] * bd[a] for a in range(D))
        hi = tuple(lo[a] + bd[a] - 1 for a in range(D))
        boxes.append((lo, hi))
    # merge touching or close boxes until none are left
    merged = True
    while merged:
        merged = False
        out: List[Box] = []
        for b in boxes:
            for k, o in enumerate(out):
                if _overlap(b, o, merge_gap):
                    out[k] = (tuple(min(b[0][a], o[0][a]) for a in range(D)),
                              tuple(max(b[1][a], o[1][a]) for a in range(D)))
                    merged = True
                    break
            else:
                out.append(b)
        boxes = out
    res: List[Box] = []
    for lo, hi in boxes:
        if lo_limit is not None:
            lo = tuple(max(lo[a], int(lo_limit[a])) for a in range(D))
        if hi_limit is not None:
            hi = tuple(min(hi[a], int(hi_limit[a])) for a in range(D))
        if any(hi[a] <= lo[a] for a in range(D)):
            continue
        nlo, nhi = [2 * v for v in lo], [2 * v for v in hi]
        for a in range(D):
            if period is not None and period[a] and hi[a] - lo[a] + 1 >= period[a]:
                nlo[a], nhi[a] = 0, 2 * int(period[a]) - 1
        res.append((tuple(nlo), tuple(nhi)))
    return sorted(res)


def remesh(lat, spec, boxes, storage=None):
    """A new bound lattice with the same domain as `lat` and refinement `boxes`
    ({level: [(lo, hi), ...]} in level coordinates), taking over lat's current state
    (call at a coarse-step boundary).  `spec` supplies faces, solids and forcing."""
    from paper_1608_06915_amd import elbm, synth

    sp = synth.Spec(spec.name, spec.D, spec.N, spec.periodic, spec.nu0, spec.levels, boxes, spec.faces,
                    spec.bodies, spec.force, spec.init, spec.U, spec.body_level, spec.body_diameter)
    new = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage or lat.storage)
    synth.apply(sp, new)
    new.bind()
    launch = lat.get_launch()
    new.set_launch(**launch)
    new.transfer_from(lat)
    return new, sp
