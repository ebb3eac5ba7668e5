"""Pins of the FP64 oracle's discrete adjoint against central finite differences of
the oracle's own forward map (the adjoint is not in the paper; it is defined as the
exact transpose of the discrete coarse step).  States are generic (seeded
non-equilibrium noise), where the KBC map is differentiable."""
import numpy as np
import pytest

import oracle
from paper_1608_06915_amd import synth


@pytest.mark.parametrize("D", [2, 3])
def test_collision_adjoint_dot_product(D):
    Q = 9 if D == 2 else 27
    r = np.random.default_rng(10 + D)
    for k, f in enumerate(synth.random_states(D, 8, seed=40 + D, spread=0.2)):
        F = np.zeros(3)
        if k % 2:  # the force derivative must also be right at F = 0
            F[:D] = r.uniform(-1e-3, 1e-3, D)
        lo, v = r.normal(size=Q), r.normal(size=Q)
        vF = np.zeros(3)
        vF[:D] = r.normal(size=D)
        for beta in (0.6, 0.97):
            lf, lF = oracle.kbc_adj(D, beta, f, lo, F)
            eps = 1e-6
            a, *_ = oracle.kbc(D, beta, f + eps * v, F + eps * vF)
            b, *_ = oracle.kbc(D, beta, f - eps * v, F - eps * vF)
            fd = lo @ (a - b) / (2 * eps)
            assert lf @ v + lF @ vF[:D] == pytest.approx(fd, rel=1e-7)


def _cyl():
    return synth.cylinder2d(48, 32, ((8, 8), (40, 24)), (20, 16), 8.0, noise=1e-3)


def _make(sp, fields=None, du0=None):
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels)
    synth.apply(sp, o)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        if du0 is not None:
            u = u + du0[l]
        o.init(l, rho, u, nz)
        o.set_force_field(l, fields[l] if fields is not None else np.zeros((sp.D,) + o.shape(l)))
    return o


def test_refined_drag_gradient_wrt_force_field_matches_fd():
    """Mean drag over every fine substep of 6 coarse steps, two levels, bounce-back
    cylinder inside the patch, gradient wrt the per-node force field of both levels,
    along seeded random directions."""
    sp = _cyl()
    o = _make(sp)
    shapes = [o.shape(l) for l in range(sp.levels)]
    o.adjoint(6, "drag", body_level=1, direction=(1, 0, 0))
    grads = [o.adjoint_force(l) for l in range(sp.levels)]
    r = np.random.default_rng(16)
    for _ in range(4):
        V = [r.normal(size=(2,) + s) for s in shapes]
        eps = 1e-7
        jp = _make(sp, [eps * v for v in V]).adjoint(6, "drag", body_level=1, direction=(1, 0, 0))
        jm = _make(sp, [-eps * v for v in V]).adjoint(6, "drag", body_level=1, direction=(1, 0, 0))
        fd = (jp - jm) / (2 * eps)
        ad = sum((g * v).sum() for g, v in zip(grads, V))
        assert ad == pytest.approx(fd, rel=1e-6)


def test_refined_kinetic_energy_gradient_wrt_initial_velocity_matches_fd():
    sp = _cyl()
    o = _make(sp)
    shapes = [o.shape(l) for l in range(sp.levels)]
    o.adjoint(6, "ke")
    gu = []
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        gu.append(oracle.init_adjoint_u(2, rho, u, nz, o.adjoint_state(l)))
    r = np.random.default_rng(17)
    for _ in range(3):
        V = [r.normal(size=(2,) + s) * 1e-3 for s in shapes]
        eps = 1e-6
        jp = _make(sp, None, [eps * v for v in V]).adjoint(6, "ke")
        jm = _make(sp, None, [-eps * v for v in V]).adjoint(6, "ke")
        fd = (jp - jm) / (2 * eps)
        ad = sum((g * v).sum() for g, v in zip(gu, V))
        assert ad == pytest.approx(fd, rel=1e-5)


def test_three_level_ke_gradient_wrt_force_matches_fd():
    """D3Q27, three nested levels with inlet/outflow: KE gradient wrt the force field."""
    sp = synth.sphere3d(48, 24, 24, D_fine=6.0, l1=((12, 6, 6), (30, 18, 18)), l2=((16, 8, 8), (24, 16, 16)),
                        centre=(20, 12, 12), noise=1e-3)
    o = _make(sp)
    shapes = [o.shape(l) for l in range(sp.levels)]
    o.adjoint(2, "ke")
    grads = [o.adjoint_force(l) for l in range(sp.levels)]
    r = np.random.default_rng(18)
    V = [r.normal(size=(3,) + s) for s in shapes]
    eps = 1e-7
    jp = _make(sp, [eps * v for v in V]).adjoint(2, "ke")
    jm = _make(sp, [-eps * v for v in V]).adjoint(2, "ke")
    fd = (jp - jm) / (2 * eps)
    ad = sum((g * v).sum() for g, v in zip(grads, V))
    assert ad == pytest.approx(fd, rel=1e-5)
