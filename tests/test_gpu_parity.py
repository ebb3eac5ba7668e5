"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle on the
same seeded inputs.

Tolerances:
  FP64 storage and arithmetic: populations agree to 1e-13 (rounding-order only).
  FP32: max |u_gpu - u_oracle| / U <= 1e-5 (the target bound) at short horizons; the
  difference grows about linearly with the number of finest steps (the full-size
  sphere measured 1.01e-5 after 50 coarse steps and 2.0e-5 after 100).
  FP16 weight-shifted storage: <= 1e-3 (the target) on the full-size channel (50 steps),
  sphere (25 steps) and forest (20 steps); elsewhere the measured size is bounded: the
  small channel below measured 1.6e-3 after 30 steps (bound 3e-3), the sphere 1.1e-3
  after 50 steps and 2.0e-3 after 100.
  BF16 weight-shifted storage (8 significant bits of f - W, no target): the measured
  size is bounded -- full-size channel 6.6e-3 (bound 1e-2), sphere 2.3e-2 after 100
  steps and the small channel 1.3e-2 (bound 3e-2).
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elbm():
    import torch

    assert torch.cuda.is_available()
    from paper_1608_06915_amd import elbm as e

    e.lib()
    return e


def pair(elbm, sp, storage, steps, gamma=False, launch=None):
    print("case %s storage=%s levels=%d steps=%d" % (sp.name, storage, sp.levels, steps), flush=True)
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, g)
    synth.apply(sp, o)
    g.bind()
    if launch:
        g.set_launch(**launch)
    if gamma:
        g.set_gamma_output(True)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        g.init(l, rho, u, nz)
        o.init(l, rho, u, nz)
    if steps:
        g.advance(steps)
        o.advance(steps)
    g.synchronize()
    return g, o


def max_du(g, o, sp):
    e = 0.0
    for l in range(sp.levels):
        _, ug = g.moments(l)
        _, uo, _ = o.moments(l)
        m = np.isfinite(uo)
        assert np.array_equal(m, np.isfinite(ug)), "node sets differ on level %d" % l
        e = max(e, float(np.max(np.abs(ug[m] - uo[m]))))
    return e / sp.U


def max_df(g, o, sp):
    e = 0.0
    for l in range(sp.levels):
        a, b = g.get_f(l), o.get_f(l)
        m = np.isfinite(b)
        assert np.array_equal(m, np.isfinite(a)), "node sets differ on level %d" % l
        e = max(e, float(np.max(np.abs(a[m] - b[m]))))
    return e


# ----------------------------------------------------------------- FP64: exact parity
def test_single_node_updates_fp64_3d(elbm):
    """One step of a periodic D3Q27 box from generic non-equilibrium states."""
    sp = synth.Spec("box3", 3, (16, 8, 8), (True,) * 3, 0.004, 1)

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[::-1])
        r = synth.rng(7)
        u = r.uniform(-0.08, 0.08, size=(3,) + shp)
        return 1 + r.uniform(-0.02, 0.02, size=shp), u, synth.pop_noise(27, shp, 0.03, 8)

    sp.init = init
    g, o = pair(elbm, sp, "f64", 1)
    assert max_df(g, o, sp) < 1e-15


def test_taylor_green_two_level_fp64_full_horizon(elbm):
    """64^2 Taylor-Green with the [16,48]^2 refined patch, 1000 coarse steps, FP64."""
    sp = synth.tgv2d()
    g, o = pair(elbm, sp, "f64", 1000, gamma=True)
    # 1000 coarse steps of FP64 rounding-order differences
    assert max_df(g, o, sp) < 3e-13
    assert max_du(g, o, sp) < 3e-12
    # decay against the closed form in coarse time
    k = 2 * math.pi / 64
    ref = math.exp(-2 * 0.01 * k * k * 1000)
    _, u = g.moments(0)[:2]
    lo, n = g.level_box(0)
    X, Y = synth.coords(lo, n, 2)
    shape = -np.cos(k * X) * np.sin(k * Y)
    m = np.isfinite(u[0])
    amp = np.sum(u[0][m] * shape[m]) / np.sum(shape[m] ** 2) / 0.05
    assert amp == pytest.approx(ref, rel=1e-2)


def test_sphere_three_level_fp64(elbm):
    """D3Q27 FP64, three nested levels with inlet, outflow and a sphere: every population
    of every level to rounding order after 6 coarse steps."""
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12), noise=1e-3)
    g, o = pair(elbm, sp, "f64", 6)
    assert max_df(g, o, sp) < 1e-13
    Fg, _ = g.drag(2)
    Fo, _ = o.drag(2)
    # momentum-exchange sums cancel O(1) terms: absolute error relative to |F|
    assert np.max(np.abs(Fg - Fo)) < 1e-12 * np.max(np.abs(Fo))


def ragged_sphere():
    """The three-level sphere with a coarse domain of 40 nodes along the inlet/outflow
    axis: 2.5 bricks of 16, so the last coarse brick is partly outside the domain."""
    return synth.sphere3d(40, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                          centre=(20, 12, 12), noise=1e-3)


def test_ragged_domain_fp64(elbm):
    sp = ragged_sphere()
    g, o = pair(elbm, sp, "f64", 6)
    assert g.level_info(0)[3] == 3 * 6 * 6  # bricks of level 0: ceil(40 / 16) x 24 / 4 x 24 / 4
    assert max_df(g, o, sp) < 1e-13


@pytest.mark.parametrize("launch", [dict(use_graph=10, xcd_remap=8), dict(use_graph=1, wg_per_cu=2, xcd_remap=1),
                                    dict(use_graph=0, xcd_remap=32, threads=128)],
                         ids=["runs-8", "persistent-slabs", "eager-two-node"])
def test_ragged_domain_launch_configurations_bitwise_equal(elbm, launch):
    sp = ragged_sphere()
    g0, _ = pair(elbm, sp, "f32", 5)
    g1, _ = pair(elbm, sp, "f32", 5, launch=launch)
    for l in range(sp.levels):
        assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True)


def test_advance_zero_steps_changes_nothing(elbm):
    sp = ragged_sphere()
    g, _ = pair(elbm, sp, "f32", 2)
    f0 = [g.get_f(l) for l in range(sp.levels)]
    g.advance(0)
    g.synchronize()
    for l in range(sp.levels):
        assert np.array_equal(g.get_f(l), f0[l], equal_nan=True)


def test_mass_momentum_and_gamma_fp64(elbm):
    sp = synth.tgv2d(32, (8, 24), 0.04, 0.02, noise=1e-3)
    g, o = pair(elbm, sp, "f64", 20, gamma=True)
    mg, jg, bad = g.reduce()
    mo, jo = o.reduce()
    assert bad == 0
    assert mg == pytest.approx(mo, rel=1e-13)
    assert np.allclose(jg, jo, rtol=0, atol=1e-12)
    for l in range(sp.levels):
        _, _, gg = g.moments(l, gamma=True)
        _, _, go = o.moments(l)
        m = np.isfinite(go)
        # gamma is kept in an FP32 buffer
        assert np.max(np.abs(gg[m] - go[m]) / np.abs(go[m])) < 3e-7


@pytest.mark.parametrize("case", ["tgv2d", "channel3d"])
def test_gamma_indicator_matches_oracle(elbm, case):
    """Per brick, the largest |gamma - 2| over its fluid nodes (the under-resolution
    measure of Sec. IV / the refinement criterion of Sec. V), on the GPU against the
    oracle's reduction of its own gamma field, FP64, every level.  Blocks without a
    fluid node read -1 on both sides; values agree to the FP32 rounding of the stored
    gamma."""
    if case == "tgv2d":
        sp = synth.tgv2d(32, (8, 24), 0.04, 0.02, noise=1e-3)
    else:
        sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g, o = pair(elbm, sp, "f64", 12, gamma=True)
    bd = g.brick_dims()
    for l in range(sp.levels):
        ig = g.gamma_indicator(l)
        io = oracle.gamma_indicator(o.moments(l)[2], bd)
        assert ig.shape == io.shape
        empty = io == -1.0
        assert np.array_equal(ig == -1.0, empty)
        assert np.max(io[~empty]) > 1e-6  # the flow is not trivially resolved everywhere
        assert np.max(np.abs(ig[~empty] - io[~empty])) < 5e-7


def test_gamma_indicator_needs_gamma_output(elbm):
    sp = synth.tgv2d(32, (8, 24), 0.04, 0.02)
    g, _ = pair(elbm, sp, "f32", 1)
    with pytest.raises(elbm.ElbmError):
        g.gamma_indicator(0)


def test_cached_launch_hit_and_miss(elbm, tmp_path):
    """A cache hit applies the stored configuration without touching the state; a miss
    returns False and leaves the configuration unchanged (no search runs)."""
    sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g, _ = pair(elbm, sp, "f32", 2)
    f0 = [g.get_f(l) for l in range(sp.levels)]
    before = g.get_launch()
    assert not g.use_cached_launch(str(tmp_path / "absent.txt"))
    assert g.get_launch() == before
    key = "d%ds%d" % (sp.D, elbm.STORAGE["f32"]) + "".join("_%d" % g.level_info(l)[3] for l in range(sp.levels))
    cache = tmp_path / "cache.txt"
    cache.write_text('# comment\n"d9s9_1": [1, 0, 0, 64, 1, 0]\n"%s": [1, 4, 0, 128, 4, 0]\n' % key)
    assert g.use_cached_launch(str(cache))
    assert g.get_launch() == dict(use_graph=1, wg_per_cu=4, xcd_remap=0, threads=128, occupancy=4, pipeline=0)
    for l in range(sp.levels):
        assert np.array_equal(g.get_f(l), f0[l], equal_nan=True)


@pytest.mark.parametrize("launch", [dict(use_graph=0), dict(use_graph=1, wg_per_cu=2, xcd_remap=1, threads=128),
                                    dict(use_graph=1, wg_per_cu=0, xcd_remap=0, threads=64),
                                    dict(use_graph=1, wg_per_cu=4, xcd_remap=1, threads=256, occupancy=4),
                                    dict(use_graph=1, wg_per_cu=2, xcd_remap=1, pipeline=1),
                                    dict(use_graph=0, wg_per_cu=3, xcd_remap=0, pipeline=1),
                                    dict(use_graph=1, wg_per_cu=0, xcd_remap=2, threads=128),
                                    dict(use_graph=1, wg_per_cu=2, xcd_remap=3, pipeline=1),
                                    dict(use_graph=1, wg_per_cu=0, xcd_remap=2, pipeline=2),
                                    dict(use_graph=0, wg_per_cu=1, xcd_remap=0, pipeline=2),
                                    dict(use_graph=4, wg_per_cu=0, xcd_remap=32, threads=128),
                                    dict(use_graph=5, wg_per_cu=0, xcd_remap=32, pipeline=2)],
                         ids=["eager", "persistent-xcd", "oneperbrick", "regcap", "pipelined", "pipelined-eager",
                              "xcd-runs", "pipelined-xcd-runs", "plain-split", "plain-split-persistent",
                              "graph-4-steps", "graph-5-steps-split"])
def test_launch_configurations_bitwise_equal(elbm, launch):
    sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g0, o = pair(elbm, sp, "f32", 6)
    g1, _ = pair(elbm, sp, "f32", 6, launch=launch)
    for l in range(sp.levels):
        assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True)


def _lattice(elbm, sp, storage, launch):
    print("case %s storage=%s launch=%s" % (sp.name, storage, launch), flush=True)
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    synth.apply(sp, g)
    g.bind()
    g.set_launch(**launch)
    g.set_gamma_output(True)
    for l in range(sp.levels):
        lo, n = g.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        g.init(l, rho, u, nz)
    return g


@pytest.mark.parametrize("case", ["sphere-f32", "sphere-f16s", "forest-f32", "forest-bf16s", "channel-f16s"])
def test_graph_replays_bitwise_equal_to_eager(elbm, case):
    """Graph replays (the coupling of a tick on a parallel branch beside its
    stream-collide, Sec. III.C) compute what the one-stream eager order computes:
    populations, gamma and drag equal bit for bit over 13 coarse steps (a graph of ten
    steps, then single-step graphs of both parities), on two to four levels and in 32-
    and 16-bit storage."""
    name, storage = case.split("-")
    sp = {"sphere": lambda: synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)),
                                           l2=((16, 8, 8), (24, 16, 16)), centre=(20, 12, 12), noise=1e-3),
          "forest": lambda: synth.forest3d(root=(4, 4, 4), counts=(8, 8, 1), block=8),
          "channel": lambda: synth.channel3d(32, 20, 16, 4, nu0=0.01)}[name]()
    thr = 128 if storage != "f32" else 256
    g0 = _lattice(elbm, sp, storage, dict(use_graph=0, threads=thr))
    g1 = _lattice(elbm, sp, storage, dict(use_graph=10, xcd_remap=8, threads=thr))
    g0.advance(13)
    g1.advance(13)
    g0.synchronize()
    g1.synchronize()
    for l in range(sp.levels):
        assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True), "level %d" % l
        assert np.array_equal(g0.moments(l, gamma=True)[2], g1.moments(l, gamma=True)[2], equal_nan=True)
        F0, s0 = g0.drag(l)
        F1, s1 = g1.drag(l)
        assert s0 == s1 and np.array_equal(F0, F1)


@pytest.mark.parametrize("launch", [dict(use_graph=10, wg_per_cu=0, xcd_remap=8, threads=256),
                                    dict(use_graph=1, wg_per_cu=0, xcd_remap=2, pipeline=2)],
                         ids=["one-launch-per-tick", "split-ticks"])
def test_profiling_pass_advances_like_advance(elbm, launch):
    """elbm_profile times every stream-collide launch (a single launch through
    hipExtLaunchKernel with start and stop events, a tick split into two launches between
    recorded events) and advances the lattice exactly as elbm_advance does."""
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12))
    g0, _ = pair(elbm, sp, "f32", 0, launch=launch)
    g1, _ = pair(elbm, sp, "f32", 0, launch=launch)
    g0.advance(3)
    tot, sc, n = g1.profile(3)
    g0.synchronize()
    g1.synchronize()
    assert n == 3 * (1 << (sp.levels - 1))
    assert 0.0 < sc <= tot
    for l in range(sp.levels):
        assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True)
    F0, s0 = g0.drag(2)
    F1, s1 = g1.drag(2)
    assert s0 == s1 and np.array_equal(F0, F1)


# ----------------------------------------------------------------- FP32 workloads
def test_channel_two_level_fp32(elbm):
    sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g, o = pair(elbm, sp, "f32", 30)
    assert max_du(g, o, sp) < 1e-5
    mg, jg, bad = g.reduce()
    mo, jo = o.reduce()
    assert bad == 0
    assert abs(mg - mo) / mo < 1e-6


def test_sphere_three_level_inlet_outflow_drag_fp32(elbm):
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12))
    g, o = pair(elbm, sp, "f32", 20)
    assert max_du(g, o, sp) < 1e-5
    Fg, sg = g.drag(2)
    Fo, so = o.drag(2)
    assert sg == so == 80
    # momentum-exchange sums: FP32 populations, FP64 accumulation
    assert np.allclose(Fg, Fo, rtol=1e-5, atol=2e-6)


@pytest.mark.parametrize("pipeline", [1, 2])
def test_sphere_pipelined_bitwise_equal_with_drag(elbm, pipeline):
    """Special links (inlet, outflow, solid) and the drag reduction with the plain bricks
    in a kernel of their own: same populations and drag as the one-brick-per-workgroup
    kernel."""
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12))
    g0, _ = pair(elbm, sp, "f32", 5)
    g1, _ = pair(elbm, sp, "f32", 5, launch=dict(use_graph=1, wg_per_cu=2, xcd_remap=1, pipeline=pipeline))
    for l in range(sp.levels):
        assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True)
    assert np.array_equal(g0.drag(2)[0], g1.drag(2)[0])


def test_forest_four_level_fp32(elbm):
    sp = synth.forest3d(root=(4, 4, 4), counts=(8, 8, 1), block=8)
    g, o = pair(elbm, sp, "f32", 4)
    assert max_du(g, o, sp) < 1e-5


def test_sphere_drag_coefficient_across_storage_forms(elbm):
    """The full-size sphere (Re = 300, D = 20 finest units, three levels): mean drag
    coefficient C_d = F_x / (rho U^2 pi R^2 / 2) over coarse steps 2000-3000 (about ten
    convective times D/U after a twenty-step start), with populations stored in FP32,
    FP16s and BF16s.  FP16s (11 significant bits of h = f - W) reproduces the FP32 value
    to 0.9 %; BF16s (8 bits) shifts it by 9.7 % -- the bound below records that bias,
    it does not claim BF16 storage is accurate for forces.  The paper prints no C_d at
    this Reynolds number, so the FP32 value is only checked to be of the physical order.
    The run is deterministic (the kernels' results do not depend on scheduling)."""
    import torch

    sp = synth.sphere3d()
    cd = {}
    for st in ("f32", "f16s", "bf16s"):
        print("case sphere3d drag storage=%s" % st, flush=True)
        g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, st)
        synth.apply(sp, g)
        g.bind()
        for l in range(sp.levels):
            lo, n = g.level_box(l)
            rho, u, nz = sp.init(l, lo, n)
            g.init(l, rho, u, nz)
        g.use_cached_launch()
        g.advance(2000)
        g.drag(sp.body_level, reset=True)
        g.advance(1000)
        F, steps = g.drag(sp.body_level)
        assert g.check() and steps == 1000 * (1 << sp.body_level)
        R = sp.body_diameter / 2.0
        cd[st] = 2.0 * (F[0] / steps) / (sp.U ** 2 * math.pi * R * R)
        del g
        torch.cuda.empty_cache()
    print("sphere3d C_d: " + ", ".join("%s %.4f" % kv for kv in cd.items()), flush=True)
    assert 0.3 < cd["f32"] < 1.5
    assert abs(cd["f16s"] / cd["f32"] - 1.0) < 0.015
    assert abs(cd["bf16s"] / cd["f32"] - 1.0) < 0.15


def test_cylinder_two_level_force_field_drag_fp32(elbm):
    import torch

    sp = synth.cylinder2d(64, 32, ((10, 8), (30, 24)), (20, 16), 8.0)
    g, o = pair(elbm, sp, "f32", 0)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        F = synth.rng(99 + l).uniform(-1e-6, 1e-6, size=(2,) + o.shape(l))
        o.set_force_field(l, F)
        g.set_force_field(l, torch.from_numpy(F).cuda())
    g.advance(40)
    o.advance(40)
    assert max_du(g, o, sp) < 1e-5
    Fg, _ = g.drag(1)
    Fo, _ = o.drag(1)
    assert np.allclose(Fg, Fo, rtol=1e-4, atol=2e-6)


# ----------------------------------------------------------------- shifted half storage
# FP16 keeps 11 significant bits of f - W ~ 3 u W: max-norm velocity errors of a few
# 1e-4 .. 2e-3 of U at U = 0.05 are the quantisation itself; BF16 keeps 8 bits.
# Measured after 30 steps: FP16s 1.6e-3, BF16s 1.3e-2.
@pytest.mark.parametrize("storage,bound", [("f16s", 3e-3), ("bf16s", 3e-2)])
def test_channel_half_storage(elbm, storage, bound):
    sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g, o = pair(elbm, sp, storage, 30)
    err = max_du(g, o, sp)
    print("%s max|du|/U = %.3e" % (storage, err))
    assert err < bound


# The 3-level sphere (inlet, outflow, drag) and the 4-level forest in 16-bit storage on
# small grids, against the FP64 oracle from identical inputs: the error is the storage
# quantisation of h over the horizon.  Measured on MI355X: sphere (20 steps) FP16s 8.3e-4
# of U and 9.8e-5 of the drag, BF16s 7.1e-3 and 5.3e-4; forest (10 steps) FP16s 1.7e-4,
# BF16s 1.8e-3.  Bounds about twice that.
@pytest.mark.parametrize("storage,bound,dbound", [("f16s", 2e-3, 3e-4), ("bf16s", 1.5e-2, 2e-3)])
def test_sphere_three_level_half_storage(elbm, storage, bound, dbound):
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12))
    g, o = pair(elbm, sp, storage, 20)
    err = max_du(g, o, sp)
    print("sphere %s max|du|/U = %.3e" % (storage, err))
    assert err < bound
    Fg, sg = g.drag(2)
    Fo, so = o.drag(2)
    assert sg == so
    derr = float(np.max(np.abs(Fg - Fo)) / np.max(np.abs(Fo)))
    print("sphere %s drag relative error %.3e" % (storage, derr))
    assert derr < dbound


@pytest.mark.parametrize("storage,bound", [("f16s", 4e-4), ("bf16s", 4e-3)])
def test_forest_four_level_half_storage(elbm, storage, bound):
    sp = synth.forest3d(root=(4, 4, 4), counts=(8, 8, 1), block=8)
    g, o = pair(elbm, sp, storage, 10)
    err = max_du(g, o, sp)
    print("forest %s max|du|/U = %.3e" % (storage, err))
    assert err < bound


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_half_storage_launch_configurations_bitwise_equal(elbm, storage):
    """16-bit storage has its own store policy and graph capture order: the cached kind of
    launch (graphs of several steps, XCD slab table, two nodes per thread) and the split
    mode give the same populations as the library default."""
    sp = synth.channel3d(32, 20, 16, 4, nu0=0.01)
    g0, _ = pair(elbm, sp, storage, 7)
    for launch in (dict(use_graph=3, wg_per_cu=0, xcd_remap=1, threads=128),
                   dict(use_graph=2, wg_per_cu=0, xcd_remap=32, threads=256, pipeline=2)):
        g1, _ = pair(elbm, sp, storage, 7, launch=launch)
        for l in range(sp.levels):
            assert np.array_equal(g0.get_f(l), g1.get_f(l), equal_nan=True)


def test_two_dimensional_xcd_slabs_bitwise_equal(elbm):
    """The XCD slab table of a 2-D lattice (slabs along y), with a force field and drag."""
    import torch

    sp = synth.cylinder2d(64, 32, ((10, 8), (30, 24)), (20, 16), 8.0)
    out = []
    for launch in (None, dict(use_graph=4, wg_per_cu=0, xcd_remap=1, threads=256),
                   dict(use_graph=1, wg_per_cu=0, xcd_remap=1, threads=256, pipeline=2)):
        g, o = pair(elbm, sp, "f32", 0, launch=launch)
        for l in range(sp.levels):
            F = synth.rng(99 + l).uniform(-1e-6, 1e-6, size=(2,) + o.shape(l))
            g.set_force_field(l, torch.from_numpy(F).cuda())
        g.advance(9)
        out.append(([g.get_f(l) for l in range(sp.levels)], g.drag(1)[0]))
    for f, d in out[1:]:
        for l in range(sp.levels):
            assert np.array_equal(out[0][0][l], f[l], equal_nan=True)
        assert np.array_equal(out[0][1], d)


def test_deterministic_repeat(elbm):
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12))
    a, _ = pair(elbm, sp, "f32", 5)
    b, _ = pair(elbm, sp, "f32", 5)
    for l in range(sp.levels):
        assert np.array_equal(a.get_f(l), b.get_f(l), equal_nan=True)
    ra, rb = a.reduce(), b.reduce()
    assert ra[0] == rb[0] and np.array_equal(ra[1], rb[1]) and ra[2] == rb[2]


# ----------------------------------------------------------------- full-size workloads
# The oracle cannot run the full-size workloads for many steps (9-18 s per coarse
# step).  After k coarse steps on the GPU, in the cached launch configuration the
# benchmark times (library default where the cache has none), the GPU state of every
# level is loaded into the oracle and both advance one more coarse step; every
# population of every node is compared.
@pytest.mark.parametrize("name,storage,k,bound", [
    ("channel3d", "f32", 50, 1e-5),
    ("channel3d", "f16s", 50, 1e-3),
    ("channel3d", "bf16s", 50, 3e-2),
    ("sphere3d", "f32", 20, 1e-5),
    ("forest3d", "f32", 20, 1e-5),
    ("cylinder2d", "f32", 200, 1e-5),
])
def test_full_size_one_step_from_gpu_state(elbm, name, storage, k, bound):
    import torch

    sp = getattr(synth, name)()
    print("full-size case %s storage=%s k=%d" % (name, storage, k), flush=True)
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    synth.apply(sp, g)
    g.bind()
    for l in range(sp.levels):
        lo, n = g.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        g.init(l, rho, u, nz)
    g.use_cached_launch()  # the benchmark's configuration where the cache has one
    g.advance(k)
    assert g.check()
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, o)
    for l in range(sp.levels):
        o.set_f(l, g.get_f(l))
    g.advance(1)
    g.synchronize()
    o.advance(1)
    e_u = max_du(g, o, sp)
    e_f = max_df(g, o, sp)
    mg, _, bad = g.reduce()
    mo, _ = o.reduce()
    print("%s %s: max|du|/U %.3e  max|df| %.3e  mass rel %.3e" % (name, storage, e_u, e_f, abs(mg - mo) / mo))
    assert bad == 0
    assert e_u < bound
    del g
    torch.cuda.empty_cache()


# ----------------------------------------------------------------- full size, many steps
# From identical seeded inputs the GPU runs the full-size workload for the stored number
# of coarse steps in the launch configuration the benchmark times; the oracle's state
# after the same steps (FP64, stored by tests/golden/make_fullsize.py, which calls only
# the oracle) is compared on one z-plane of every level (through the interfaces and the
# body), with the total mass.
# Bounds: FP32 <= 1e-5 and FP16s <= 1e-3 where the targets hold.  The difference to FP64
# grows about linearly with the number of finest steps (the rounding of the stored
# populations, correlated from step to step).  The sphere's finest level takes 4 steps
# per coarse step: the targets hold there after 25 coarse steps; after 50 it measured
# 1.01e-5 (FP32) and 1.10e-3 (FP16s), after 100 2.0e-5 and 2.0e-3, so those horizons
# carry bounds of 1.5x the measured values.  BF16s (8 significant bits of f - W) has no
# target: its bounds record the measured size (channel 6.6e-3, sphere 2.3e-2).
FULLSIZE = [
    ("channel3d", 50, "f32", 1e-5), ("channel3d", 50, "f16s", 1e-3), ("channel3d", 50, "bf16s", 1e-2),
    ("sphere3d", 25, "f32", 1e-5), ("sphere3d", 25, "f16s", 1e-3),
    ("sphere3d", 50, "f32", 1.5e-5), ("sphere3d", 50, "f16s", 1.6e-3),
    ("sphere3d", 100, "f32", 3e-5), ("sphere3d", 100, "f16s", 3e-3), ("sphere3d", 100, "bf16s", 3e-2),
    ("forest3d", 20, "f32", 1e-5), ("forest3d", 20, "f16s", 1e-3),
]


@pytest.mark.parametrize("name,steps,storage,bound", FULLSIZE, ids=["%s-%d-%s" % c[:3] for c in FULLSIZE])
def test_full_size_many_steps_against_oracle(elbm, name, steps, storage, bound):
    import torch

    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "fullsize_%s_%d.npz" % (name, steps)))
    assert int(ref["steps"]) == steps
    sp = getattr(synth, name)()
    print("full-size case %s storage=%s steps=%d" % (name, storage, steps), flush=True)
    g = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    synth.apply(sp, g)
    g.bind()
    for l in range(sp.levels):
        lo, n = g.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        g.init(l, rho, u, nz)
    g.use_cached_launch()
    g.advance(steps)
    mass, _, bad = g.reduce()
    e_u, e_r = 0.0, 0.0
    for l in range(sp.levels):
        k = int(ref["l%d_z" % l])
        rho, u = g.moments(l)
        ro = ref["l%d_rho_m1" % l].astype(np.float64) + 1.0
        uo = ref["l%d_u" % l].astype(np.float64)
        m = np.isfinite(ro)
        assert np.array_equal(m, np.isfinite(rho[k])), "node sets differ on level %d" % l
        du = np.where(m[None], np.abs(u[:, k] - uo), 0.0)
        arg = np.unravel_index(int(np.argmax(du)), du.shape)
        print("  level %d: max|du|/U %.3e at component %d, (y, x) index %s of plane %d; max|drho| %.3e" % (
            l, du.max() / sp.U, arg[0], arg[1:], k, float(np.max(np.abs(rho[k][m] - ro[m])))), flush=True)
        e_u = max(e_u, float(du.max()) / sp.U)
        e_r = max(e_r, float(np.max(np.abs(rho[k][m] - ro[m]))))
    m_ref, m0 = float(ref["mass"]), float(ref["mass0"])
    print("%s %s after %d steps: max|du|/U %.3e  max|drho| %.3e  mass vs oracle %.3e  oracle mass drift %.3e" % (
        name, storage, steps, e_u, e_r, (mass - m_ref) / m_ref, (m_ref - m0) / m0), flush=True)
    assert bad == 0
    assert e_u < bound
    del g
    torch.cuda.empty_cache()


def test_child_process_tuner_writes_a_cache_the_library_applies(elbm, tmp_path):
    """The tuner times each candidate in a child process, writes the fastest; the
    library then applies that entry (elbm_tune cache hit)."""
    from paper_1608_06915_amd import tune

    cache = str(tmp_path / "cache.txt")
    print("case tuner channel3d(32,20,16,4) f32 small candidates", flush=True)
    key, best, results = tune.tune("tests.tune_workloads:small_channel", "f32", cache, kind="small", steps=5,
                                   warmup=2, windows=2, timeout=110)
    assert sum("ms_per_step" in r for r in results) == len(results)
    assert tune.read_cache(cache)[key] == [best[f] for f in tune.FIELDS]
    from tests.tune_workloads import small_channel

    sp = small_channel()
    g, _ = pair(elbm, sp, "f32", 0)
    assert g.use_cached_launch(cache)
    assert g.get_launch() == best
