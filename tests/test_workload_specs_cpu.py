"""Invariants of the paper-scale sphere workload that hold without building it (the full
build takes a minute and several GB of host memory): the refinement boxes nest with
margins, the sphere lies inside the finest box, the coarse population buffer stays
within what 32-bit brick offsets address, and Re, U, D match the paper's sphere case."""
import math

from paper_1608_06915_amd import synth


def test_sphere_paper3d_spec():
    sp = synth.sphere_paper3d()
    assert sp.levels == 4 and sp.D == 3
    nx, ny, nz = sp.N
    # level 0 population buffer: 27 FP32 values per node, addressed by 32-bit byte offsets
    assert nx * ny * nz * 27 * 4 < 2 ** 32
    # domain about 30D x 20D x 20D (D = 120 finest units = 15 coarse units)
    D_coarse = sp.body_diameter / 8.0
    assert abs(nx / D_coarse - 30) < 0.5 and abs(ny / D_coarse - 20) < 0.5 and abs(nz / D_coarse - 20) < 0.5
    # viscosity: Re = U D / nu on the finest level, convective scaling nu_l = 2^l nu_0
    assert math.isclose(sp.U * sp.body_diameter / (8.0 * sp.nu0), 3700.0, rel_tol=1e-12)
    # boxes nest: each level's box inside its parent's, at least 4 parent nodes from its faces
    prev_lo, prev_hi = (0, 0, 0), tuple(sp.N)
    for l in range(1, sp.levels):
        (lo, hi), = sp.boxes[l]
        plo = tuple(v * 2 for v in prev_lo)
        phi = tuple(v * 2 for v in prev_hi)
        for a in range(3):
            assert lo[a] >= plo[a] + 8 and hi[a] <= phi[a] - 8
        prev_lo, prev_hi = lo, hi
    # the sphere (finest-level centre and radius) lies inside the finest box with a margin
    (lo, hi), = sp.boxes[3]
    centre, radius = sp.bodies[3]
    for a in range(3):
        assert centre[a] - radius - lo[a] >= 32 and hi[a] - (centre[a] + radius) >= 32
