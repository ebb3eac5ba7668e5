"""Pins of the oracle's drag, inlet/outflow faces and interface coupling.

These parts of the oracle have no printed values to compare with; they are fixed
here by balance laws and exactness properties that hold whatever the flow:

* drag (momentum exchange on solid links, reading R10): on a single-level grid the
  momentum of the fluid changes in one step by the body force on every fluid node,
  minus the exchange recorded at the previous collision, minus the exchange with the
  bounce-back walls (computed here from the populations);
* inlet and outflow faces (reading R9): a uniform equilibrium flow at the inlet
  velocity is carried unchanged through inlet, outflow and every refinement
  interface; on a single level the mass changes in one step by what the inlet
  brings in, minus what leaves through both faces, plus what the outflow copies in
  (all computed here from the populations and the closed-form equilibrium moments);
* coupling (Sec. III.C steps 3-4, Eq. interp, Eq. f_neq_rescaling_iso): fields whose
  density, velocity and non-equilibrium part are cubic polynomials, given on both
  levels at consistent scales, are reconstructed exactly at every child interface
  node and every parent ring node; twin and ring nodes keep the density and velocity
  of their source and scale its non-equilibrium part by beta_c / (2 beta_f) and its
  inverse.

The last test compiles copies of the oracle with one plausible mistake each (a
dropped factor, a wrong population, a wrong weight or factor) and checks that the
pin meant to catch it fails.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import synth


def vel(D):
    Q = 9 if D == 2 else 27
    c = np.zeros((Q, 3), dtype=np.int64)
    for i in range(Q):
        c[i, 0] = i % 3 - 1
        c[i, 1] = (i // 3) % 3 - 1
        if D == 3:
            c[i, 2] = i // 9 - 1
    return c[:, :D]


def start(sp, library=None):
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    synth.apply(sp, o)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        o.init(l, rho, u, nz)
    return o


def noisy_init(D, u_mean, amp_u, amp_noise, seed):
    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:D][::-1])
        r = synth.rng(seed + level)
        u = np.stack([u_mean[a] + amp_u * r.uniform(-1, 1, size=shp) for a in range(D)])
        rho = 1.0 + 0.01 * r.uniform(-1, 1, size=shp)
        return rho, u, synth.pop_noise(9 if D == 2 else 27, shp, amp_noise, seed + 50 + level)

    return init


# ---------------------------------------------------------------- drag: momentum budget
def drag_case(kind):
    if kind == "periodic2d":
        sp = synth.Spec("mb2", 2, (24, 16), (True, True), 0.02, 1, bodies={0: ((11.3, 7.6), 3.2)},
                        force=(2e-6, -1e-6, 0.0))
    elif kind == "walls2d":
        sp = synth.Spec("mb2w", 2, (24, 16), (True, False), 0.02, 1, bodies={0: ((11.3, 7.6), 3.2)},
                        faces={2: (synth.FACE_WALL, (0, 0, 0)), 3: (synth.FACE_WALL, (0, 0, 0))},
                        force=(3e-6, 0.0, 0.0))
    else:
        sp = synth.Spec("mb3", 3, (12, 10, 8), (True, True, True), 0.02, 1, bodies={0: ((5.6, 4.7, 3.9), 2.4)},
                        force=(1e-6, 2e-6, -1e-6))
    sp.init = noisy_init(sp.D, (0.03, -0.01, 0.01), 0.01, 2e-3, 77)
    return sp


def fluid_momentum(o, D):
    f = o.get_f(0)  # post-collision, NaN at solid nodes
    c = vel(D)
    m = np.isfinite(f[0])
    J = np.array([np.sum(c[:, a].reshape((-1,) + (1,) * D) * np.where(m, f, 0.0)) for a in range(D)])
    return J, int(m.sum()), f, m


def wall_exchange(f, m, D, periodic):
    """sum over fluid nodes x and populations i whose x + c_i lies beyond a wall of
    2 c_i f'_i(x): the momentum the walls take in one streaming step"""
    c = vel(D)
    shape = f.shape[1:]
    W = np.zeros(D)
    for i in range(len(c)):
        hit = np.zeros(shape, dtype=bool)
        for a in range(D):
            if periodic[a] or c[i, a] == 0:
                continue
            ax = D - 1 - a  # numpy axis of coordinate a
            sl = [slice(None)] * D
            sl[ax] = -1 if c[i, a] > 0 else 0
            h = np.zeros(shape, dtype=bool)
            h[tuple(sl)] = True
            hit |= h
        fi = np.where(hit & m, f[i], 0.0)
        W += 2.0 * c[i] * fi.sum()
    return W


def pin_momentum_budget(kind, library=None):
    sp = drag_case(kind)
    o = start(sp, library)
    o.advance(1)
    J0, nfl, f0, m0 = fluid_momentum(o, sp.D)
    D0, _ = o.drag(0, reset=True)
    F = np.array(sp.force[: sp.D])
    worst = 0.0
    for _ in range(6):
        W0 = wall_exchange(f0, m0, sp.D, sp.periodic)
        o.advance(1)
        J1, n1, f1, m1 = fluid_momentum(o, sp.D)
        D1, k = o.drag(0, reset=True)
        assert n1 == nfl and k == 1
        resid = (J1 - J0) - (nfl * F - D0 - W0)
        worst = max(worst, float(np.max(np.abs(resid))))
        J0, D0, f0, m0 = J1, D1, f1, m1
    assert np.max(np.abs(D0)) > 1e-4  # the exchange is not negligible
    assert worst < 1e-13, "momentum budget residual %.3e" % worst


@pytest.mark.parametrize("kind", ["periodic2d", "walls2d", "periodic3d"])
def test_drag_closes_the_momentum_budget(kind):
    pin_momentum_budget(kind)


# ---------------------------------------------------------------- inlet / outflow
def open_case(D, levels, body=False):
    U = (0.05, 0.01, -0.005)[:D] + (0.0,) * (3 - D)
    if D == 2:
        boxes = {1: [((16, 8), (48, 24))], 2: [((40, 24), (80, 40))]}
        sp = synth.Spec("io2", 2, (40, 16), (False, True), 0.02, levels,
                        {l: b for l, b in boxes.items() if l < levels},
                        faces={0: (synth.FACE_INLET, U), 1: (synth.FACE_OUTFLOW, (0, 0, 0))})
    else:
        boxes = {1: [((16, 8, 8), (40, 24, 24))], 2: [((40, 24, 24), (72, 40, 40))]}
        sp = synth.Spec("io3", 3, (28, 16, 16), (False, True, True), 0.02, levels,
                        {l: b for l, b in boxes.items() if l < levels},
                        faces={0: (synth.FACE_INLET, U), 1: (synth.FACE_OUTFLOW, (0, 0, 0))})
    return sp, U


def pin_uniform_flow_through_open_faces(D, levels, library=None):
    sp, U = open_case(D, levels)

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:D][::-1])
        return np.ones(shp), np.stack([np.full(shp, U[a]) for a in range(D)]), None

    sp.init = init
    o = start(sp, library)
    o.advance(15)
    ref = oracle.feq(D, 1.0, U)
    for l in range(levels):
        f = o.get_f(l)
        m = np.isfinite(f[0])
        assert m.sum() > 0
        err = float(np.max(np.abs(f[:, m] - ref[:, None])))
        assert err < 1e-14, "level %d: uniform flow changed by %.3e" % (l, err)


@pytest.mark.parametrize("D,levels", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_uniform_flow_passes_inlet_outflow_and_interfaces(D, levels):
    pin_uniform_flow_through_open_faces(D, levels)


def incoming_equilibrium_sum(rho, ux):
    """sum of f^eq_i over the populations with c_ix = +1, from the closed-form first and
    second x-moments of the product equilibrium (pinned separately):
    (sum c_x f^eq + sum c_x^2 f^eq) / 2 = (rho u_x + rho (2 sqrt(1 + 3u_x^2) - 1)/3) / 2"""
    return 0.5 * (rho * ux + rho * (2.0 * math.sqrt(1.0 + 3.0 * ux * ux) - 1.0) / 3.0)


def pin_mass_budget_open_faces(D, library=None):
    sp, U = open_case(D, 1)
    sp.init = noisy_init(D, U, 0.01, 2e-3, 91)
    o = start(sp, library)
    o.advance(1)
    c = vel(D)
    face_nodes = int(np.prod(sp.N[1:D]))
    inflow = face_nodes * incoming_equilibrium_sum(1.0, U[0])
    m0, _ = o.reduce()
    worst = 0.0
    for _ in range(6):
        f = o.get_f(0)
        xm, xp = (f[(slice(None),) + (Ellipsis, 0)], f[(slice(None),) + (Ellipsis, -1)])  # x = 0 and x = N-1 faces
        out = xm[c[:, 0] == -1].sum() + xp[c[:, 0] == 1].sum()
        copied = xp[c[:, 0] == -1].sum()  # the outflow copies these populations back in
        o.advance(1)
        m1, _ = o.reduce()
        resid = (m1 - m0) - (inflow + copied - out)
        worst = max(worst, abs(resid))
        m0 = m1
    assert worst < 1e-13 * m0, "mass budget residual %.3e" % worst


@pytest.mark.parametrize("D", [2, 3])
def test_mass_budget_across_inlet_and_outflow(D):
    pin_mass_budget_open_faces(D)


# ---------------------------------------------------------------- coupling: exactness
def zero_moment_vectors(D):
    """population vectors with zero mass and momentum: W_i times deviatoric quadratics"""
    c = vel(D).astype(float)
    W = np.prod(np.where(c == 0, 2.0 / 3.0, 1.0 / 6.0), axis=1)
    if D == 2:
        basis = [c[:, 0] * c[:, 1], c[:, 0] ** 2 - c[:, 1] ** 2]
    else:
        basis = [c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2], c[:, 0] ** 2 - c[:, 1] ** 2,
                 c[:, 0] ** 2 - c[:, 2] ** 2]
    V = np.array([W * b for b in basis])
    assert np.allclose(V.sum(axis=1), 0, atol=1e-17)
    assert np.allclose(V @ c, 0, atol=1e-17)
    return V


def cubic(D, seed):
    """a random polynomial of total degree 3 in D variables, bounded by 1 on [-1, 1]^D"""
    r = synth.rng(seed)
    terms = [e for e in itertools.product(range(4), repeat=D) if sum(e) <= 3]
    coef = r.uniform(-1, 1, size=len(terms)) / len(terms)

    def p(xi):
        return sum(a * np.prod([xi[k] ** e[k] for k in range(D)], axis=0) for a, e in zip(coef, terms))

    return p


def couple_case(D):
    if D == 2:
        return synth.Spec("cp2", 2, (32, 32), (True, True), 0.02, 2, {1: [((16, 16), (48, 48))]}), 16.0
    return synth.Spec("cp3", 3, (16, 16, 16), (True, True, True), 0.02, 2, {1: [((8, 8, 8), (24, 24, 24))]}), 8.0


def field_states(o, sp, level, scale, fields):
    """populations f^eq(rho, u) + scale * neq over the level box, from polynomial
    fields of the position in coarse units; NaN where the level has no node"""
    D = sp.D
    lo, n = o.level_box(level)
    X = [x / 2.0 ** level for x in synth.coords(lo, n, D)]
    rho, u, neq = fields(X)
    cls = o.node_class(level)
    Q = 9 if D == 2 else 27
    g = np.full((Q,) + cls.shape, np.nan)
    for idx in zip(*np.nonzero(cls >= 0)):
        uu = [u[a][idx] for a in range(D)]
        g[(slice(None),) + idx] = oracle.feq(D, rho[idx], uu) + scale * neq[(slice(None),) + idx]
    return g, cls


def polynomial_fields(D, centre, half):
    V = zero_moment_vectors(D)
    pr = cubic(D, 11)
    pu = [cubic(D, 20 + a) for a in range(D)]
    pn = [cubic(D, 40 + k) for k in range(len(V))]

    def fields(X):
        xi = [(X[a] - centre) / half for a in range(D)]
        rho = 1.0 + 0.02 * pr(xi)
        u = [0.04 * pu[a](xi) for a in range(D)]
        neq = sum(2e-2 * pn[k](xi)[None] * V[k].reshape((-1,) + (1,) * D) for k in range(len(V)))
        return rho, u, neq

    return fields


def pin_coupling_reconstructs_cubic_fields(D, library=None):
    sp, centre = couple_case(D)
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    synth.apply(sp, o)
    bc, bf = o.level_info(0)[2], o.level_info(1)[2]
    kappa = 2.0 * bf / bc  # parent non-equilibrium = child's times the inverse rescaling
    fields = polynomial_fields(D, centre, 10.0)
    gp, cp = field_states(o, sp, 0, kappa, fields)
    gc, cc = field_states(o, sp, 1, 1.0, fields)
    ring = (cp >= 0) & ((cp & 2) != 0)
    layer = (cc >= 0) & (((cc >> 2) & 3) <= 1)
    assert ring.sum() > 0 and layer.sum() > 0
    gp_in, gc_in = gp.copy(), gc.copy()
    gp_in[:, ring] = np.nan  # outputs of the coupling: never read by it
    gc_in[:, layer] = np.nan
    gp_out, gc_out = o.couple_states(0, gp_in, gc_in)
    ep = float(np.max(np.abs(gp_out[:, ring] - gp[:, ring])))
    ec = float(np.max(np.abs(gc_out[:, layer] - gc[:, layer])))
    # every other value passes unchanged
    assert np.array_equal(gp_out[:, ~ring & (cp >= 0)], gp[:, ~ring & (cp >= 0)])
    assert np.array_equal(gc_out[:, ~layer & (cc >= 0)], gc[:, ~layer & (cc >= 0)])
    assert ec < 1e-14, "child interface nodes off the cubic field by %.3e" % ec
    assert ep < 1e-14, "parent ring nodes off the field by %.3e" % ep


@pytest.mark.parametrize("D", [2, 3])
def test_coupling_reconstructs_cubic_fields_exactly(D):
    pin_coupling_reconstructs_cubic_fields(D)


def moments(g, D):
    c = vel(D).astype(float)
    rho = g.sum(axis=0)
    u = np.stack([np.tensordot(c[:, a], g, axes=(0, 0)) / rho for a in range(D)])
    return rho, u


def pin_twin_and_ring_rescaling(D, library=None):
    """Random (non-polynomial) states: at twin nodes (child outer layer on parent nodes)
    and parent ring nodes the coupling keeps the source node's density and velocity and
    multiplies its non-equilibrium part by beta_c / (2 beta_f) resp. 2 beta_f / beta_c."""
    sp, centre = couple_case(D)
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    synth.apply(sp, o)
    bc, bf = o.level_info(0)[2], o.level_info(1)[2]
    r = synth.rng(5)
    V = zero_moment_vectors(D)
    Q = V.shape[1]

    def random_states(level):
        lo, n = o.level_box(level)
        cls = o.node_class(level)
        g = np.full((Q,) + cls.shape, np.nan)
        for idx in zip(*np.nonzero(cls >= 0)):
            u = r.uniform(-0.05, 0.05, size=D)
            g[(slice(None),) + idx] = oracle.feq(D, 1 + r.uniform(-0.02, 0.02), u) + \
                (r.uniform(-0.01, 0.01, size=len(V)) @ V)
        return g, cls, lo

    gp, cp, lop = random_states(0)
    gc, cc, loc = random_states(1)
    gp_out, gc_out = o.couple_states(0, gp, gc)
    checked = 0
    for idx in zip(*np.nonzero((cc >= 0) & (((cc >> 2) & 3) == 0))):
        x = [loc[a] + idx[D - 1 - a] for a in range(D)]
        if any(v % 2 for v in x):
            continue  # hanging node, not a twin
        X = [x[a] // 2 - lop[a] for a in range(D)]
        src = gp[(slice(None),) + tuple(X[::-1])]
        out = gc_out[(slice(None),) + idx]
        rs, us = moments(src[:, None], D)
        ro, uo = moments(out[:, None], D)
        assert abs(ro[0] - rs[0]) < 1e-15 and np.max(np.abs(uo - us)) < 1e-15
        feq = oracle.feq(D, rs[0], us[:, 0])
        assert np.max(np.abs((out - feq) - bc / (2 * bf) * (src - feq))) < 1e-15
        checked += 1
    for idx in zip(*np.nonzero((cp >= 0) & ((cp & 2) != 0))):
        X = [lop[a] + idx[D - 1 - a] for a in range(D)]
        xc = [2 * X[a] - loc[a] for a in range(D)]
        src = gc[(slice(None),) + tuple(xc[::-1])]
        out = gp_out[(slice(None),) + idx]
        rs, us = moments(src[:, None], D)
        feq = oracle.feq(D, rs[0], us[:, 0])
        assert np.max(np.abs((out - feq) - 2 * bf / bc * (src - feq))) < 1e-15
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("D", [2, 3])
def test_twin_and_ring_rescaling_keep_moments_and_scale_nonequilibrium(D):
    pin_twin_and_ring_rescaling(D)


# ---------------------------------------------------------------- planted mistakes
MUTATIONS = {
    "drag_from_precollision_state": (
        "step_drag[a] += 2.0 * o->c[i][a] * L->f[(size_t)n * Q + i];",
        "step_drag[a] += 2.0 * o->c[i][a] * L->g[(size_t)n * Q + i];",
        lambda lib: pin_momentum_budget("periodic2d", lib)),
    "drag_without_factor_two": (
        "step_drag[a] += 2.0 * o->c[i][a] * L->f[(size_t)n * Q + i];",
        "step_drag[a] += 1.0 * o->c[i][a] * L->f[(size_t)n * Q + i];",
        lambda lib: pin_momentum_budget("periodic3d", lib)),
    "drag_on_links_out_of_solids": (
        "for (int a = 0; a < 3; ++a) y[a] = L->pos[3 * n + a] + o->c[i][a];\n  if (!canon(o, l, y)) return 0;",
        "for (int a = 0; a < 3; ++a) y[a] = L->pos[3 * n + a] - o->c[i][a];\n  if (!canon(o, l, y)) return 0;",
        lambda lib: pin_momentum_budget("walls2d", lib)),
    "inlet_opposite_population": (
        "val = feq[i];", "val = feq[Q - 1 - i];",
        lambda lib: pin_uniform_flow_through_open_faces(3, 1, lib)),
    "inlet_rest_density_missing": (
        "ora_feq(o->D, 1.0, o->face_u[face], feq);", "ora_feq(o->D, 1.001, o->face_u[face], feq);",
        lambda lib: pin_mass_budget_open_faces(2, lib)),
    "outflow_two_nodes_upstream": (
        "y[a] += (fc & 1) ? -1 : 1;", "y[a] += (fc & 1) ? -2 : 2;",
        lambda lib: pin_mass_budget_open_faces(3, lib)),
    "interpolation_weights": (
        "{-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};\n  /* error code per child node",
        "{1.0 / 16.0, 7.0 / 16.0, 7.0 / 16.0, 1.0 / 16.0};\n  /* error code per child node",
        lambda lib: pin_coupling_reconstructs_cubic_fields(2, lib)),
    "coalescence_factor_inverted": (
        "double fac = 2.0 * C->beta / P->beta;", "double fac = P->beta / (2.0 * C->beta);",
        lambda lib: pin_twin_and_ring_rescaling(3, lib)),
    "explosion_without_rescaling": (
        "double fac = P->beta / (2.0 * C->beta);\n  for (int i = 0; i < o->Q; ++i) fneq[i] *= fac;",
        "double fac = 1.0;\n  for (int i = 0; i < o->Q; ++i) fneq[i] *= fac;",
        lambda lib: pin_coupling_reconstructs_cubic_fields(3, lib)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_its_pin(name, tmp_path):
    old, new, pin = MUTATIONS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "elbm_oracle.c")).read()
    assert src.count(old) == 1, "mutation anchor not unique in the oracle source"
    path = tmp_path / "elbm_oracle.c"
    path.write_text(src.replace(old, new))
    header = os.path.join(os.path.dirname(oracle.__file__), "elbm_oracle.h")
    (tmp_path / "elbm_oracle.h").write_text(open(header).read())
    so = oracle.compile_library(str(path), str(tmp_path / "libmut.so"))
    lib = oracle.load_library(so)
    with pytest.raises((AssertionError, oracle.OracleError)):
        pin(lib)
