"""Write the oracle's full-size multi-step references (tests/golden/fullsize_<workload>_<steps>.npz).

Each workload runs from its seeded inputs (paper_1608_06915_amd/synth.py, the same
generators the GPU tests use) for a fixed number of coarse steps in the FP64 oracle
(its OpenMP build: same arithmetic and results as the single-thread build).  Stored:
the total mass (owned volumes) before and after, and, per level, the density and
velocity (the mid-step velocity of the forcing scheme) on one z-plane of the level's
index box -- the plane through the middle of the box, which crosses the refinement
interfaces and any body -- as float32 deviations (rho - 1, u), enough for comparisons
at the 1e-7 level of U = 0.05.

Only the oracle and the input generators are called.  Usage:
    python tests/golden/make_fullsize.py [workload ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1608_06915_amd import synth  # noqa: E402

# (workload, coarse steps): short horizons at which FP32 parity is meaningful on these
# flows -- channel 50, sphere 25, 50 and 100, forest 20
RUNS = [("channel3d", 50), ("sphere3d", 25), ("sphere3d", 50), ("sphere3d", 100), ("forest3d", 20)]


def plane_index(n):
    """z index (within the level box) of the stored plane"""
    return int(n[2]) // 2


def make(name, steps):
    sp = getattr(synth, name)()
    t0 = time.time()
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library="omp")
    synth.apply(sp, o)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        o.init(l, rho, u, nz)
    mass0, _ = o.reduce()
    o.advance(steps)
    mass, mom = o.reduce()
    out = {"workload": np.array(name), "steps": np.array(steps), "mass0": np.array(mass0),
           "mass": np.array(mass), "momentum": np.array(mom), "levels": np.array(sp.levels)}
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        k = plane_index(n)
        rho, u, _ = o.moments(l)
        out["l%d_z" % l] = np.array(k)
        out["l%d_rho_m1" % l] = (rho[k] - 1.0).astype(np.float32)
        out["l%d_u" % l] = u[:, k].astype(np.float32)
    path = os.path.join(HERE, "fullsize_%s_%d.npz" % (name, steps))
    np.savez_compressed(path, **out)
    print("%s: %d steps in %.0f s, mass %.15g -> %.15g, wrote %s (%d bytes)" % (
        name, steps, time.time() - t0, mass0, mass, path, os.path.getsize(path)), flush=True)


if __name__ == "__main__":
    want = sys.argv[1:]
    for name, steps in RUNS:
        if not want or name in want or "%s_%d" % (name, steps) in want:
            make(name, steps)
