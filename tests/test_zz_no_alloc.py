"""elbm_init_fields_static (the entry point for callers that cannot allocate device
memory) against elbm_init_fields: bitwise the same initial populations, and the same
state after a few coarse steps, on two calls in a row -- a larger three-level 3-D
lattice with noise, then a smaller two-level 2-D one -- and the size limit of its static
staging buffer."""
import numpy as np
import pytest

from paper_1608_06915_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elbm():
    import torch

    assert torch.cuda.is_available()
    from paper_1608_06915_amd import elbm as e

    e.lib()
    return e


def lattice(elbm, sp, static):
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, "f32")
    synth.apply(sp, g)
    g.bind()
    for l in range(sp.levels):
        lo, n = g.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        (g.init_static if static else g.init)(l, rho, u, nz)
    return g


def test_static_staging_init_matches_the_allocating_init(elbm):
    cases = [synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                            centre=(20, 12, 12), noise=1e-3),
             synth.tgv2d(32, (8, 24), 0.04, 0.02, noise=1e-3)]
    for sp in cases:  # the second call stages a smaller input than the first
        print("case %s static staging" % sp.name, flush=True)
        a = lattice(elbm, sp, False)
        b = lattice(elbm, sp, True)
        for l in range(sp.levels):
            assert np.array_equal(a.get_f(l), b.get_f(l), equal_nan=True)
        a.advance(3)
        b.advance(3)
        for l in range(sp.levels):
            assert np.array_equal(a.get_f(l), b.get_f(l), equal_nan=True)


def test_static_staging_refuses_levels_beyond_its_size(elbm):
    sp = synth.Spec("box80", 3, (80, 64, 64), (True, True, True), 0.01, 1)
    r = synth.rng(3)

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[::-1])
        return np.ones(shp), r.uniform(-0.02, 0.02, size=(3,) + shp), synth.pop_noise(27, shp, 1e-3, 4)

    sp.init = init
    print("case box80 static staging limit", flush=True)
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, "f32")
    synth.apply(sp, g)
    g.bind()
    lo, n = g.level_box(0)
    rho, u, nz = sp.init(0, lo, n)
    # 80 x 64 x 64 nodes x (1 + 3 + 27) x 8 bytes = 81 MB > 32 MiB: refused, nothing written
    with pytest.raises(elbm.ElbmError) as e:
        g.init_static(0, rho, u, nz)
    assert e.value.status == 1
    # without the noise array it needs 80 x 64 x 64 x 4 x 8 = 10.5 MB
    g.init_static(0, rho, u)
    h = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, "f32")
    synth.apply(sp, h)
    h.bind()
    h.init(0, rho, u)
    assert np.array_equal(g.get_f(0), h.get_f(0), equal_nan=True)
