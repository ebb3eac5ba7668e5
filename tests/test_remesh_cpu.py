"""Re-meshing on the CPU: the oracle's state transfer between refinement layouts, and
the choice of refinement boxes from the stabiliser's per-brick readout.

The transfer (reading R15 of the oracle: same node copied, coalescence from the old
finer node, Eq. interp reconstruction with composite values, post-collision
non-equilibrium scaled by beta_c (1 - 2 beta_f) / (2 beta_f (1 - 2 beta_c))) is pinned by
* the identity onto the same layout;
* uniform equilibrium flow carried unchanged onto any layout;
* fields whose density, velocity and non-equilibrium part are cubic polynomials (given
  on every level at the scale the factor relates) reconstructed exactly on a newly
  refined region and coalesced exactly where refinement is removed;
* refining and coarsening back returning the coarse state (explosion then coalescence
  at twin positions is the identity);
and a copy of the oracle with the factor's inverse planted fails the cubic pin.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import remesh, synth


def vel(D):
    Q = 9 if D == 2 else 27
    c = np.zeros((Q, 3), dtype=np.int64)
    for i in range(Q):
        c[i, 0] = i % 3 - 1
        c[i, 1] = (i // 3) % 3 - 1
        if D == 3:
            c[i, 2] = i // 9 - 1
    return c[:, :D]


def layout(D, boxes):
    if D == 2:
        return synth.Spec("rm2", 2, (32, 32), (True, True), 0.02, 2, boxes)
    return synth.Spec("rm3", 3, (32, 16, 16), (True, True, True), 0.02, 2, boxes)


# level-1 boxes (level-1 coordinates): A, B (A moved, overlapping it), AB (A and a
# second box apart from it)
BOXES = {2: {"A": {1: [((8, 8), (24, 24))]}, "B": {1: [((12, 10), (28, 26))]},
             "AB": {1: [((8, 8), (24, 24)), ((36, 36), (52, 52))]}},
         3: {"A": {1: [((4, 8, 8), (16, 24, 24))]}, "B": {1: [((8, 8, 10), (20, 24, 26))]},
             "AB": {1: [((4, 8, 8), (16, 24, 24)), ((36, 8, 8), (48, 24, 24))]}}}


def make(D, key, library=None, init=None):
    sp = layout(D, BOXES[D][key])
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    synth.apply(sp, o)
    if init is not None:
        for l in range(sp.levels):
            lo, n = o.level_box(l)
            rho, u, nz = init(l, lo, n)
            o.init(l, rho, u, nz)
    return o, sp


def noisy(D, seed=3):
    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:D][::-1])
        r = synth.rng(seed + level)
        u = r.uniform(-0.03, 0.03, size=(D,) + shp)
        return 1 + r.uniform(-0.01, 0.01, size=shp), u, synth.pop_noise(9 if D == 2 else 27, shp, 2e-3, seed + 9)

    return init


@pytest.mark.parametrize("D", [2, 3])
def test_transfer_onto_the_same_layout_is_the_identity(D):
    a, _ = make(D, "A", init=noisy(D))
    a.advance(3)
    b, _ = make(D, "A")
    b.transfer_from(a)
    for l in range(2):
        assert np.array_equal(a.get_f(l), b.get_f(l), equal_nan=True)


@pytest.mark.parametrize("D", [2, 3])
def test_uniform_flow_is_carried_onto_another_layout(D):
    U = (0.04, -0.02, 0.01)[:D]

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:D][::-1])
        return np.ones(shp), np.stack([np.full(shp, U[a]) for a in range(D)]), None

    a, _ = make(D, "A", init=init)
    a.advance(2)
    b, _ = make(D, "B")
    b.transfer_from(a)
    ref = oracle.feq(D, 1.0, U)
    for l in range(2):
        f = b.get_f(l)
        m = np.isfinite(f[0])
        assert np.max(np.abs(f[:, m] - ref[:, None])) < 1e-15
    b.advance(3)
    for l in range(2):
        f = b.get_f(l)
        m = np.isfinite(f[0])
        assert np.max(np.abs(f[:, m] - ref[:, None])) < 1e-14


def zero_moment_vectors(D):
    c = vel(D).astype(float)
    W = np.prod(np.where(c == 0, 2.0 / 3.0, 1.0 / 6.0), axis=1)
    if D == 2:
        basis = [c[:, 0] * c[:, 1], c[:, 0] ** 2 - c[:, 1] ** 2]
    else:
        basis = [c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2], c[:, 0] ** 2 - c[:, 1] ** 2]
    return np.array([W * b for b in basis])


def cubic(D, seed):
    r = synth.rng(seed)
    terms = [e for e in itertools.product(range(4), repeat=D) if sum(e) <= 3]
    coef = r.uniform(-1, 1, size=len(terms)) / len(terms)
    return lambda xi: sum(a * np.prod([xi[k] ** e[k] for k in range(D)], axis=0) for a, e in zip(coef, terms))


def set_cubic_state(o, D, scale_of_level):
    """post-collision populations f^eq(rho, u) + s_l n on every node of every level, with
    rho, u, n cubic in the position (coarse units)"""
    V = zero_moment_vectors(D)
    pr, pu = cubic(D, 11), [cubic(D, 20 + a) for a in range(D)]
    pn = [cubic(D, 40 + k) for k in range(len(V))]
    centre = 16.0 if D == 2 else 10.0
    for l in range(2):
        lo, n = o.level_box(l)
        X = [x / 2.0 ** l for x in synth.coords(lo, n, D)]
        xi = [(X[a] - centre) / 10.0 for a in range(D)]
        rho = 1.0 + 0.02 * pr(xi)
        u = [0.04 * pu[a](xi) for a in range(D)]
        neq = sum(2e-2 * pn[k](xi)[None] * V[k].reshape((-1,) + (1,) * D) for k in range(len(V)))
        Q = V.shape[1]
        f = np.full((Q,) + rho.shape, np.nan)
        for idx in np.ndindex(*rho.shape):
            f[(slice(None),) + idx] = oracle.feq(D, rho[idx], [u[a][idx] for a in range(D)]) + \
                scale_of_level[l] * neq[(slice(None),) + idx]
        o.set_f(l, f)
    return f


def post_factor(o):
    bc, bf = o.level_info(0)[2], o.level_info(1)[2]
    return bc * (1 - 2 * bf) / (2 * bf * (1 - 2 * bc))


def pin_cubic_transfer(D, library=None):
    """A -> B moves the refined box: B's new fine nodes are reconstructed, B's coarse
    nodes where A was refined and B is not are coalesced; every node must equal the
    cubic field at its level's scale."""
    a, _ = make(D, "A", library=library)
    b, _ = make(D, "B", library=library)
    k = post_factor(a)
    set_cubic_state(a, D, {0: 1.0 / k, 1: 1.0})
    want, _ = make(D, "B")
    set_cubic_state(want, D, {0: 1.0 / k, 1: 1.0})
    b.transfer_from(a)
    for l in range(2):
        fb, fw = b.get_f(l), want.get_f(l)
        m = np.isfinite(fw[0])
        assert np.array_equal(m, np.isfinite(fb[0]))
        err = float(np.max(np.abs(fb[:, m] - fw[:, m])))
        assert err < 1e-14, "level %d off the cubic field by %.3e" % (l, err)


@pytest.mark.parametrize("D", [2, 3])
def test_cubic_fields_are_reconstructed_and_coalesced_exactly(D):
    pin_cubic_transfer(D)


@pytest.mark.parametrize("D", [2, 3])
def test_refine_then_coarsen_returns_the_coarse_state(D):
    """A -> AB refines a second region from level 0 alone (explosion at twin positions,
    reconstruction elsewhere); AB -> A coalesces it back: level 0 returns to its state
    (explosion then coalescence is the identity) and level 1 is copied both ways."""
    a, _ = make(D, "A", init=noisy(D))
    a.advance(4)
    b, _ = make(D, "AB")
    b.transfer_from(a)
    c, _ = make(D, "A")
    c.transfer_from(b)
    for l in range(2):
        fa, fc = a.get_f(l), c.get_f(l)
        m = np.isfinite(fa[0])
        assert np.array_equal(m, np.isfinite(fc[0]))
        assert np.max(np.abs(fa[:, m] - fc[:, m])) < 1e-15, "level %d" % l
    # the second region was reconstructed: its twin nodes carry the coarse density
    rb, _, _ = b.moments(1)
    assert np.isfinite(rb).sum() > np.isfinite(a.moments(1)[0]).sum()


def test_transfer_refuses_a_different_domain():
    a, _ = make(2, "A", init=noisy(2))
    sp = synth.Spec("rm2b", 2, (32, 32), (True, True), 0.03, 2, BOXES[2]["A"])
    b = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, b)
    with pytest.raises(oracle.OracleError):
        b.transfer_from(a)


def test_planted_factor_inverse_fails_the_cubic_pin(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "elbm_oracle.c")).read()
    old = "return bc * (1.0 - 2.0 * bf) / (2.0 * bf * (1.0 - 2.0 * bc));"
    assert src.count(old) == 1
    (tmp_path / "elbm_oracle.c").write_text(src.replace(old, "return (2.0 * bf * (1.0 - 2.0 * bc)) / (bc * (1.0 - 2.0 * bf));"))
    (tmp_path / "elbm_oracle.h").write_text(open(os.path.join(os.path.dirname(oracle.__file__), "elbm_oracle.h")).read())
    lib = oracle.load_library(oracle.compile_library(str(tmp_path / "elbm_oracle.c"), str(tmp_path / "libmut.so")))
    with pytest.raises(AssertionError):
        pin_cubic_transfer(2, lib)


# ---------------------------------------------------------------- refinement boxes
def test_boxes_cover_marked_bricks_and_merge_neighbours():
    ind = np.full((8, 12), 0.0)  # (y, x) bricks
    ind[2, 3] = 0.5
    ind[2, 5] = 0.4  # close to the first: merged
    ind[6, 10] = 0.3  # far: its own box
    ind[0, 0] = -1.0  # no fluid
    boxes = remesh.boxes_from_indicator(ind, (16, 16), (0, 0), threshold=0.1, pad_bricks=0, merge_gap=20)
    assert len(boxes) == 2
    (lo0, hi0), (lo1, hi1) = boxes
    # next-level coordinates: twice the level's
    assert lo0 == (2 * 3 * 16, 2 * 2 * 16) and hi0 == (2 * (6 * 16 - 1), 2 * (3 * 16 - 1))
    assert lo1 == (2 * 10 * 16, 2 * 6 * 16) and hi1 == (2 * (11 * 16 - 1), 2 * (7 * 16 - 1))
    assert remesh.boxes_from_indicator(ind, (16, 16), (0, 0), threshold=1.0) == []


def test_boxes_are_padded_and_clipped():
    ind = np.zeros((4, 4, 4))  # (z, y, x) bricks of 16 x 4 x 4
    ind[1, 1, 1] = 1.0
    boxes = remesh.boxes_from_indicator(ind, (16, 4, 4), (0, 0, 0), threshold=0.5, pad_bricks=1,
                                        lo_limit=(4, 4, 4), hi_limit=(59, 11, 11))
    assert boxes == [((8, 8, 8), (2 * 47, 2 * 11, 2 * 11))]
