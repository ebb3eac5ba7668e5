"""The oracle's two builds and its stored full-size references (no GPU needed).

* The OpenMP build runs the same node loops on several threads; every parallel loop
  writes per-node values and every sum stays serial, so its results are bitwise those
  of the single-thread build.
* tests/golden/fullsize_<workload>.npz hold the oracle's state after many coarse steps
  of the full-size workloads (written by tests/golden/make_fullsize.py, which calls
  only the oracle); their planes must match the workloads' level boxes.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def run(sp, steps, library):
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    synth.apply(sp, o)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        o.init(l, rho, u, nz)
    o.advance(steps)
    return o


@pytest.mark.parametrize("case", ["sphere3", "forest4", "cylinder2"])
def test_openmp_build_is_bitwise_the_single_thread_build(case):
    if case == "sphere3":
        sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                            centre=(20, 12, 12), noise=1e-3)
    elif case == "forest4":
        sp = synth.forest3d(root=(4, 4, 4), counts=(8, 8, 1), block=8)
    else:
        sp = synth.cylinder2d(64, 32, ((10, 8), (30, 24)), (20, 16), 8.0)
    a = run(sp, 3, None)
    b = run(sp, 3, "omp")
    for l in range(sp.levels):
        assert np.array_equal(a.get_f(l), b.get_f(l), equal_nan=True)
    assert a.reduce()[0] == b.reduce()[0]
    if sp.body_level is not None:
        assert np.array_equal(a.drag(sp.body_level)[0], b.drag(sp.body_level)[0])


@pytest.mark.parametrize("name,steps", [("channel3d", 50), ("sphere3d", 25), ("sphere3d", 50), ("sphere3d", 100),
                                        ("forest3d", 20)])
def test_fullsize_references_match_the_workloads(name, steps):
    path = os.path.join(GOLDEN, "fullsize_%s_%d.npz" % (name, steps))
    ref = np.load(path)
    sp = getattr(synth, name)()
    assert str(ref["workload"]) == name and int(ref["levels"]) == sp.levels
    assert int(ref["steps"]) == steps
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, o)
    for l in range(sp.levels):
        _, n = o.level_box(l)
        k = int(ref["l%d_z" % l])
        assert k == int(n[2]) // 2
        assert ref["l%d_u" % l].shape == (3, int(n[1]), int(n[0]))
        assert ref["l%d_rho_m1" % l].shape == (int(n[1]), int(n[0]))
        assert np.isfinite(ref["l%d_rho_m1" % l]).sum() > 0
    # the oracle's own mass drift over the run (refinement is not exactly conservative)
    assert abs(float(ref["mass"]) / float(ref["mass0"]) - 1.0) < 1e-3
