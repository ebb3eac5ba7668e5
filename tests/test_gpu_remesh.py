"""GPU re-meshing against the oracle: elbm_transfer_state (the state carried over to a
lattice with other refinement blocks) from identical states, then further steps on the
new layout; and the refinement loop driven by the stabiliser's per-brick readout."""
import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import remesh, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elbm():
    import torch

    assert torch.cuda.is_available()
    from paper_1608_06915_amd import elbm as e

    e.lib()
    return e


def noisy(D, seed=3, amp=0.03):
    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:D][::-1])
        r = synth.rng(seed + level)
        u = r.uniform(-amp, amp, size=(D,) + shp)
        return 1 + r.uniform(-0.01, 0.01, size=shp), u, synth.pop_noise(9 if D == 2 else 27, shp, 2e-3, seed + 9)

    return init


def build(elbm, sp, storage, init=None):
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, g)
    synth.apply(sp, o)
    g.bind()
    if init is not None:
        for l in range(sp.levels):
            lo, n = o.level_box(l)
            rho, u, nz = init(l, lo, n)
            g.init(l, rho, u, nz)
            o.init(l, rho, u, nz)
    return g, o


def max_df(g, o, L):
    e = 0.0
    for l in range(L):
        a, b = g.get_f(l), o.get_f(l)
        m = np.isfinite(b)
        assert np.array_equal(m, np.isfinite(a)), "node sets differ on level %d" % l
        e = max(e, float(np.max(np.abs(a[m] - b[m]))))
    return e


def max_du(g, o, L, U):
    e = 0.0
    for l in range(L):
        _, ug = g.moments(l)
        _, uo, _ = o.moments(l)
        m = np.isfinite(uo)
        e = max(e, float(np.max(np.abs(ug[m] - uo[m]))))
    return e / U


def spec(D, boxes, levels=2):
    if D == 2:
        return synth.Spec("rmg2", 2, (32, 32), (True, True), 0.02, levels, boxes)
    return synth.Spec("rmg3", 3, (32, 16, 16), (True, True, True), 0.02, levels, boxes)


CASES = {
    "2d-move": (2, {1: [((8, 8), (24, 24))]}, {1: [((12, 10), (28, 26))]}),
    "2d-add": (2, {1: [((8, 8), (24, 24))]}, {1: [((8, 8), (24, 24)), ((36, 36), (52, 52))]}),
    "3d-move": (3, {1: [((4, 8, 8), (16, 24, 24))]}, {1: [((8, 8, 10), (20, 24, 26))]}),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_transfer_matches_oracle_fp64(elbm, case):
    D, old, new = CASES[case]
    print("case remesh %s f64" % case, flush=True)
    sa = spec(D, old)
    ga, oa = build(elbm, sa, "f64", noisy(D))
    ga.advance(6)
    oa.advance(6)
    assert max_df(ga, oa, 2) < 1e-13
    sb = spec(D, new)
    gb, ob = build(elbm, sb, "f64")
    gb.transfer_from(ga)
    ob.transfer_from(oa)
    assert max_df(gb, ob, 2) < 1e-13
    gb.advance(6)
    ob.advance(6)
    assert max_df(gb, ob, 2) < 1e-13


def test_transfer_three_levels_fp64(elbm):
    """Three levels with inlet, outflow and a sphere on level 2: the level-2 box grows
    downstream (new fine nodes from level 1) and level 1 shifts."""
    def sp_of(l1, l2):
        return synth.sphere3d(48, 24, 24, D_fine=6.0, l1=l1, l2=l2, centre=(20, 12, 12), noise=1e-3)

    sa = sp_of(((12, 6, 6), (30, 18, 18)), ((16, 8, 8), (24, 16, 16)))
    sb = sp_of(((12, 6, 6), (34, 18, 18)), ((16, 8, 8), (28, 16, 16)))
    print("case remesh sphere 3 levels f64", flush=True)
    ga, oa = build(elbm, sa, "f64", sa.init)
    ga.advance(4)
    oa.advance(4)
    gb, ob = build(elbm, sb, "f64")
    gb.transfer_from(ga)
    ob.transfer_from(oa)
    assert max_df(gb, ob, 3) < 1e-13
    gb.advance(4)
    ob.advance(4)
    assert max_df(gb, ob, 3) < 1e-13
    Fg, _ = gb.drag(2)
    Fo, _ = ob.drag(2)
    assert np.max(np.abs(Fg - Fo)) < 1e-12 * np.max(np.abs(Fo))


@pytest.mark.parametrize("storage,bound", [("f32", 1e-5), ("f16s", 1e-3)])
def test_transfer_matches_oracle_reduced_storage(elbm, storage, bound):
    D, old, new = CASES["3d-move"]
    print("case remesh 3d-move %s" % storage, flush=True)
    sa = spec(D, old)
    ga, oa = build(elbm, sa, storage, noisy(D, amp=0.05))
    ga.advance(5)
    oa.advance(5)
    sb = spec(D, new)
    gb, ob = build(elbm, sb, storage)
    gb.transfer_from(ga)
    ob.transfer_from(oa)
    gb.advance(5)
    ob.advance(5)
    err = max_du(gb, ob, 2, 0.05)
    print("remesh %s max|du|/U %.3e" % (storage, err), flush=True)
    assert err < bound


def test_refinement_follows_the_gamma_indicator(elbm):
    """A 2-D double shear layer, under-resolved on level 0: the per-brick |gamma - 2| of
    level 0 picks the level-1 boxes (remesh.boxes_from_indicator), the lattice moves onto
    them (remesh.remesh), and the oracle, given the same boxes, agrees after the
    transfer and after further steps."""
    N = 64
    k = 2 * np.pi / N

    def init(level, lo, n):
        s = 2.0 ** level
        X, Y = synth.coords(lo, n, 2)
        x, y = X / s, Y / s
        ux = 0.05 * np.tanh(30.0 * (np.abs(y / N - 0.5) - 0.25))
        uy = 0.005 * np.sin(k * x)
        nz = synth.pop_noise(9, x.shape, 1e-3, 70 + level)
        return np.ones(x.shape), np.stack([ux, uy]), nz

    sa = synth.Spec("shear2", 2, (N, N), (True, True), 2e-4, 2, {1: [((16, 16), (48, 48))]}, init=init, U=0.05)
    print("case remesh driven by the gamma indicator", flush=True)
    ga, oa = build(elbm, sa, "f64", init)
    ga.set_gamma_output(True)
    ga.advance(10)
    oa.advance(10)
    ind = ga.gamma_indicator(0)
    thr = float(np.quantile(ind[ind >= 0], 0.8))
    lo0, n0 = ga.level_box(0)
    boxes = remesh.boxes_from_indicator(ind, ga.brick_dims(), lo0, thr, pad_bricks=0, merge_gap=12,
                                        lo_limit=(0, 4), hi_limit=(N - 1, N - 5), period=(N, N))
    assert boxes, "the indicator marks no brick"
    print("indicator threshold %.3e -> level-1 boxes %s" % (thr, boxes), flush=True)
    gb, sb = remesh.remesh(ga, sa, {1: boxes})
    ob = oracle.Oracle(sb.D, sb.N, sb.periodic, sb.nu0, sb.levels)
    synth.apply(sb, ob)
    ob.transfer_from(oa)
    assert max_df(gb, ob, 2) < 1e-13
    gb.advance(8)
    ob.advance(8)
    assert max_df(gb, ob, 2) < 1e-13
